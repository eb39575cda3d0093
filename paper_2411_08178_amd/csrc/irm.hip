// The alternating minimisation method (Alg. 2) for the l_p - l_q problem
//   min_x 1/p sum_m |(A x - y)_m|^p + lambda/q sum_l |(L x)_l|^q,
// L the first differences (each component its own group).  The half-quadratic
// representation of |r|^p turns the x-update into the linear system
//   Phi_k x = A^T W_f y,   Phi_k = A^T W_f A + lambda L^T W_g L,
// with W_f = diag(|A x - y|^{p-2}) and W_g = diag(|L x|^{q-2}) (|r| smoothed to
// sqrt(r^2 + eps)), solved by conjugate gradients, or by PCG with the Nystrom
// preconditioner of eq. (11) rebuilt from a sketch of Phi_k at every outer
// iteration (Alg. 1 on Y = Phi_k Omega).  Every x-update starts from the
// previous iterate.
//
// Scalars of CG (step lengths, residual norms) are FP64 device reductions
// read back once or twice per CG iteration; the vectors stay in T.

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace nys {

template <class T> nys_status fill_zero(T* p, size_t n, hipStream_t st);

namespace {

constexpr int kIrmRed = 256;

// w = ((a - y)^2 + eps)^{pw / 2}  (y may be null)
template <class T>
__global__ __launch_bounds__(256) void irm_weight_kernel(const T* __restrict__ a,
                                                         const T* __restrict__ y, int64_t n,
                                                         double pw, double eps, T* __restrict__ w) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double r = static_cast<double>(a[i]) - (y ? static_cast<double>(y[i]) : 0.0);
    w[i] = static_cast<T>(pow(r * r + eps, 0.5 * pw));
  }
}

// v[c][i] *= w[i] for ncols columns of n entries
template <class T>
__global__ __launch_bounds__(256) void mul_cols_kernel(T* __restrict__ v, const T* __restrict__ w,
                                                       int64_t n, int64_t ncols) {
  const int64_t total = n * ncols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[e] *= w[e % n];
}

// out[c] = first differences of x[c]: channel 0 X[i,j] - X[i-1,j] (0 on row
// 0), channel 1 X[i,j] - X[i,j-1] (0 on column 0); out is [c][2][n1][n2]
template <class T>
__global__ __launch_bounds__(256) void grad_cols_kernel(const T* __restrict__ x, int n1, int n2,
                                                        T* __restrict__ out) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  const size_t N = static_cast<size_t>(n1) * n2, o = static_cast<size_t>(i) * n2 + j;
  const T* xc = x + blockIdx.z * N;
  T* oc = out + 2 * blockIdx.z * N;
  const T v = xc[o];
  oc[o] = i >= 1 ? v - xc[o - n2] : T(0);
  oc[N + o] = j >= 1 ? v - xc[o - 1] : T(0);
}

// out[c] += lam * (adjoint of the first differences)(q[c])
template <class T>
__global__ __launch_bounds__(256) void grad_adj_add_kernel(const T* __restrict__ q, int n1, int n2,
                                                           T lam, T* __restrict__ out) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  const size_t N = static_cast<size_t>(n1) * n2, o = static_cast<size_t>(i) * n2 + j;
  const T* q1 = q + 2 * blockIdx.z * N;
  const T* q2 = q1 + N;
  T v = 0;
  if (i >= 1) v += q1[o];
  if (i + 1 < n1) v -= q1[o + n2];
  if (j >= 1) v += q2[o];
  if (j + 1 < n2) v -= q2[o + 1];
  out[blockIdx.z * N + o] += lam * v;
}

// block partials of <a, b> and <c, d> (c may be null)
template <class T>
__global__ __launch_bounds__(256) void dot2_partial_kernel(const T* __restrict__ a,
                                                           const T* __restrict__ b,
                                                           const T* __restrict__ c,
                                                           const T* __restrict__ d, int64_t n,
                                                           double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  double s0 = 0, s1 = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    s0 += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    if (c) s1 += static_cast<double>(c[i]) * static_cast<double>(d[i]);
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      r0[threadIdx.x] += r0[threadIdx.x + k];
      r1[threadIdx.x] += r1[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r0[0];
    part[gridDim.x + blockIdx.x] = r1[0];
  }
}

// out[0..1] = sums of the two partial rows (fixed order)
__global__ void dot2_tail_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double r0[256], r1[256];
  double s0 = 0, s1 = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s0 += part[i];
    s1 += part[nb + i];
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      r0[threadIdx.x] += r0[threadIdx.x + k];
      r1[threadIdx.x] += r1[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

// y = a x + b y
template <class T>
__global__ __launch_bounds__(256) void axpby_kernel(T a, const T* __restrict__ x, T b,
                                                    T* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

template <class T>
__global__ __launch_bounds__(256) void sub_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                  T* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = a[i] - b[i];
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>(std::min<int64_t>(cdiv(n, 256), 2048)); }

template <class T>
struct Irm {
  const nys_problem& p;
  hipStream_t st;
  int64_t N, M;
  int n1, n2;
  T *wf, *wg, *meas, *g, *b, *r, *z, *d, *q, *xprev;
  double *part, *dots;
  Scratch* scr = nullptr;   // the caller's workspace (vectors, sketch temporaries)

  Irm(const nys_problem& pr, hipStream_t s) : p(pr), st(s) {
    N = p.op->N;
    M = p.op->M;
    n1 = p.op->d.n1;
    n2 = p.op->d.n2;
  }

  static size_t vec_bytes(int64_t N, int64_t M) {
    return ws_round(sizeof(T) * (2 * static_cast<size_t>(M) + 10 * N)) +
           ws_round(sizeof(double) * (2 * kIrmRed + 8));
  }
  nys_status alloc() {
    // meas, wf (M each); g, wg (2N each); b, r, z, d, q, xprev (N each)
    const size_t vecs = 2 * static_cast<size_t>(M) + 4 * N + 6 * N;
    T* base = nullptr;
    NYS_TAKE(scr, T, base, vecs);
    meas = base;
    wf = meas + M;
    g = wf + M;
    wg = g + 2 * N;
    b = wg + 2 * N;
    r = b + N;
    z = r + N;
    d = z + N;
    q = d + N;
    xprev = q + N;
    NYS_TAKE(scr, double, part, 2 * kIrmRed + 8);
    dots = part + 2 * kIrmRed;
    return NYS_OK;
  }

  // out[c] = Phi v[c] for ncols columns (scratch: meas-sized and g-sized per column)
  nys_status phi(const T* v, T* out, int64_t ncols, T* scrM, T* scrG) {
    NYS_TRY(op_fwd<T>(p.op, v, scrM, ncols, st));
    hipLaunchKernelGGL((mul_cols_kernel<T>), dim3(grid_for(M * ncols)), dim3(256), 0, st, scrM, wf,
                       M, ncols);
    NYS_TRY(launch_check("mul_cols_kernel"));
    NYS_TRY(op_adj<T>(p.op, scrM, out, ncols, st));
    const dim3 gg(cdiv(n2, 64), cdiv(n1, 4), static_cast<unsigned>(ncols));
    hipLaunchKernelGGL((grad_cols_kernel<T>), gg, dim3(256), 0, st, v, n1, n2, scrG);
    NYS_TRY(launch_check("grad_cols_kernel"));
    hipLaunchKernelGGL((mul_cols_kernel<T>), dim3(grid_for(2 * N * ncols)), dim3(256), 0, st, scrG,
                       wg, 2 * N, ncols);
    NYS_TRY(launch_check("mul_cols_kernel"));
    hipLaunchKernelGGL((grad_adj_add_kernel<T>), gg, dim3(256), 0, st, scrG, n1, n2,
                       static_cast<T>(p.lambda), out);
    return launch_check("grad_adj_add_kernel");
  }

  // host[0] = <a, b>, host[1] = <c, d>
  nys_status dot2(const T* a, const T* bb, const T* c, const T* dd, int64_t n, double* host) {
    hipLaunchKernelGGL((dot2_partial_kernel<T>), dim3(kIrmRed), dim3(256), 0, st, a, bb, c, dd, n,
                       part);
    NYS_TRY(launch_check("dot2_partial_kernel"));
    hipLaunchKernelGGL(dot2_tail_kernel, dim3(1), dim3(256), 0, st, part, kIrmRed, dots);
    NYS_TRY(launch_check("dot2_tail_kernel"));
    NYS_CHECK_HIP(hipMemcpyAsync(host, dots, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    return NYS_OK;
  }

  nys_status axpby(T a, const T* x, T bcoef, T* y, int64_t n) {
    hipLaunchKernelGGL((axpby_kernel<T>), dim3(grid_for(n)), dim3(256), 0, st, a, x, bcoef, y, n);
    return launch_check("axpby_kernel");
  }
};

// Workspace of irm_impl: the vectors, the multi-column temporaries of the
// sketch of Phi_k, the operator's scratch on as many columns and, with a
// preconditioner, the scratch of Alg. 1 and of its applications.
template <class T>
size_t irm_ws_bytes(const nys_problem& p, int64_t ell) {
  const int64_t N = p.op->N, M = p.op->M;
  const int64_t ncs = ell > 0 ? ell : 1;
  size_t b = Irm<T>::vec_bytes(N, M) +
             ws_round(sizeof(T) * (static_cast<size_t>(M) + 2 * N + (ell > 0 ? N : 0)) * ncs) +
             op_ws_bytes(p.op, sizeof(T), ncs);
  if (ell > 0) {
    const int64_t Lp = (ell + 15) / 16 * 16;
    b += factor_ws_bytes(N, static_cast<int>(ell)) + ws_round(sizeof(double) * ell) +
         ws_round(sizeof(double) * 256 * Lp);
  }
  return b;
}

template <class T>
nys_status irm_impl(const nys_problem& p, const nys_irm_opts& o, const T* omega, int64_t ell,
                    const T* x0, T* x, int32_t* cg_iters, int32_t* outer_done, double* info,
                    Scratch* scr, hipStream_t st) {
  Irm<T> w(p, st);
  w.scr = scr;
  NYS_TRY(w.alloc());
  const int64_t N = w.N, M = w.M;
  const int64_t ncs = ell > 0 ? ell : 1;
  T* scrM = nullptr;
  NYS_TAKE(scr, T, scrM, (static_cast<size_t>(M) + 2 * N + (ell > 0 ? N : 0)) * ncs);
  T* scrG = scrM + M * ncs;
  T* Y = scrG + 2 * N * ncs;
  if (x0 && x0 != x) NYS_CHECK_HIP(hipMemcpyAsync(x, x0, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
  else if (!x0) NYS_TRY(fill_zero<T>(x, N, st));
  nys_pc pc = nullptr;
  nys_factor_opts fo{o.nu_mode, o.tail, o.mu, 6, sizeof(T) == 8 ? NYS_F64 : NYS_F32};
  const nys_dtype dt = sizeof(T) == 8 ? NYS_F64 : NYS_F32;
  nys_status status = NYS_OK;
  int k = 0;
  for (k = 1; k <= o.max_outer; ++k) {
    // weights at the previous iterate
    NYS_TRY(op_fwd<T>(p.op, x, w.meas, 1, st));
    hipLaunchKernelGGL((irm_weight_kernel<T>), dim3(grid_for(M)), dim3(256), 0, st, w.meas,
                       static_cast<const T*>(p.y), M, o.p - 2.0, o.eps, w.wf);
    NYS_TRY(launch_check("irm_weight_kernel"));
    const dim3 gg(cdiv(w.n2, 64), cdiv(w.n1, 4), 1);
    hipLaunchKernelGGL((grad_cols_kernel<T>), gg, dim3(256), 0, st, x, w.n1, w.n2, w.g);
    NYS_TRY(launch_check("grad_cols_kernel"));
    hipLaunchKernelGGL((irm_weight_kernel<T>), dim3(grid_for(2 * N)), dim3(256), 0, st, w.g,
                       static_cast<const T*>(nullptr), 2 * N, o.q - 2.0, o.eps, w.wg);
    NYS_TRY(launch_check("irm_weight_kernel"));
    // b = A^T W_f y
    NYS_CHECK_HIP(hipMemcpyAsync(w.meas, p.y, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL((mul_cols_kernel<T>), dim3(grid_for(M)), dim3(256), 0, st, w.meas, w.wf, M,
                       int64_t(1));
    NYS_TRY(launch_check("mul_cols_kernel"));
    NYS_TRY(op_adj<T>(p.op, w.meas, w.b, 1, st));
    // preconditioner of Phi_k: sketch, then Alg. 1
    if (ell > 0) {
      NYS_TRY(w.phi(omega, Y, ell, scrM, scrG));
      if (!pc) {
        // the preconditioner handle of this call (its buffers), bound to the
        // caller's workspace for Alg. 1 and the applications
        status = pc_create(N, ell, fo, &pc, st);
        if (status != NYS_OK) return status;
        pc->scr = scr;
      }
      status = factor_refresh(pc, omega, Y, dt, fo, st);
      if (status != NYS_OK) { nys_pc_destroy(pc); return status; }
      if (info) {
        double nu = 0;
        int32_t keff = 0, fst = 0;
        status = nys_pc_info(pc, nullptr, &nu, &keff, &fst, st);
        if (status != NYS_OK) { nys_pc_destroy(pc); return status; }
        info[3 * (k - 1) + 0] = fst;
        info[3 * (k - 1) + 1] = keff;
        info[3 * (k - 1) + 2] = nu;
      }
    }
    // PCG from x
    NYS_CHECK_HIP(hipMemcpyAsync(w.xprev, x, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    auto fail = [&](nys_status s) { if (pc) nys_pc_destroy(pc); return s; };
    nys_status s2 = w.phi(x, w.q, 1, scrM, scrG);
    if (s2 != NYS_OK) return fail(s2);
    hipLaunchKernelGGL((sub_kernel<T>), dim3(grid_for(N)), dim3(256), 0, st, w.b, w.q, w.r, N);
    if ((s2 = launch_check("sub_kernel")) != NYS_OK) return fail(s2);
    double hd[2];
    if ((s2 = w.dot2(w.b, w.b, w.r, w.r, N, hd)) != NYS_OK) return fail(s2);
    const double nb = std::sqrt(hd[0]);
    int it = 0;
    if (nb == 0.0) {
      if ((s2 = fill_zero<T>(x, N, st)) != NYS_OK) return fail(s2);   // Phi x = 0
    } else if (std::sqrt(hd[1]) > o.cg_tol * nb) {
      if (pc) { if ((s2 = pc_apply<T>(pc, true, w.r, w.z, 1, st)) != NYS_OK) return fail(s2); }
      else NYS_CHECK_HIP(hipMemcpyAsync(w.z, w.r, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
      NYS_CHECK_HIP(hipMemcpyAsync(w.d, w.z, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
      if ((s2 = w.dot2(w.r, w.z, nullptr, nullptr, N, hd)) != NYS_OK) return fail(s2);
      double rz = hd[0];
      while (it < o.max_cg) {
        if ((s2 = w.phi(w.d, w.q, 1, scrM, scrG)) != NYS_OK) return fail(s2);
        if ((s2 = w.dot2(w.d, w.q, nullptr, nullptr, N, hd)) != NYS_OK) return fail(s2);
        const double alpha = rz / hd[0];
        if ((s2 = w.axpby(static_cast<T>(alpha), w.d, T(1), x, N)) != NYS_OK) return fail(s2);
        if ((s2 = w.axpby(static_cast<T>(-alpha), w.q, T(1), w.r, N)) != NYS_OK) return fail(s2);
        ++it;
        if (pc) { if ((s2 = pc_apply<T>(pc, true, w.r, w.z, 1, st)) != NYS_OK) return fail(s2); }
        else NYS_CHECK_HIP(hipMemcpyAsync(w.z, w.r, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
        if ((s2 = w.dot2(w.r, w.r, w.r, w.z, N, hd)) != NYS_OK) return fail(s2);
        if (std::sqrt(hd[0]) <= o.cg_tol * nb || !std::isfinite(hd[0])) break;
        const double beta = hd[1] / rz;
        rz = hd[1];
        if ((s2 = w.axpby(T(1), w.z, static_cast<T>(beta), w.d, N)) != NYS_OK) return fail(s2);
      }
    }
    if (cg_iters) cg_iters[k - 1] = it;
    // outer stopping test ||x - x_prev|| <= tol ||x||
    hipLaunchKernelGGL((sub_kernel<T>), dim3(grid_for(N)), dim3(256), 0, st, x, w.xprev, w.q, N);
    if ((s2 = launch_check("sub_kernel")) != NYS_OK) return fail(s2);
    if ((s2 = w.dot2(w.q, w.q, x, x, N, hd)) != NYS_OK) return fail(s2);
    if (std::sqrt(hd[0]) <= o.outer_tol * std::sqrt(hd[1])) break;
  }
  if (outer_done) *outer_done = std::min(k, o.max_outer);
  if (pc) nys_pc_destroy(pc);
  return NYS_OK;
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" nys_status irm_workspace_size(const nys_problem* prob, nys_dtype dt, int64_t ell,
                                         size_t* bytes) {
  NYS_REQUIRE(prob && prob->op && bytes && ell >= 0 && ell <= PcMeta::kMaxEll,
              "irm_workspace_size: bad argument");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "irm_workspace_size: dtype must be F64 or F32");
  *bytes = dt == NYS_F64 ? irm_ws_bytes<double>(*prob, ell) : irm_ws_bytes<float>(*prob, ell);
  return NYS_OK;
}

extern "C" nys_status irm_solve(const nys_problem* prob, nys_dtype dt, const nys_irm_opts* opts,
                                const void* omega, int64_t ell, const void* x0, void* x,
                                int32_t* cg_iters, int32_t* outer_done, double* info, void* ws,
                                size_t ws_bytes, void* stream) {
  NYS_REQUIRE(prob && prob->op && prob->y && opts && x, "irm_solve: bad argument");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "irm_solve: dtype must be F64 or F32");
  const nys_irm_opts& o = *opts;
  NYS_REQUIRE(o.p > 0 && o.p <= 2 && o.q > 0 && o.q <= 2 && o.eps > 0,
              "irm_solve: need 0 < p, q <= 2 and eps > 0");
  NYS_REQUIRE(o.max_outer >= 1 && o.max_cg >= 0 && o.cg_tol > 0, "irm_solve: bad iteration limits");
  NYS_REQUIRE(prob->op->d.kind != NYS_OP_IDENTITY || prob->op->d.wavelet_levels == 0,
              "irm_solve: the regulariser acts on the image (no wavelet reparametrisation)");
  NYS_REQUIRE(prob->op->d.wavelet_levels == 0, "irm_solve: operator must act on the image");
  NYS_REQUIRE(ell == 0 || (omega && ell >= 1 && ell <= PcMeta::kMaxEll && ell <= prob->op->N),
              "irm_solve: ell must be 0 (plain CG) or in [1, %d] with omega", PcMeta::kMaxEll);
  NYS_REQUIRE(o.tail == 0 || o.tail == 1, "irm_solve: tail must be 0 or 1");
  NYS_REQUIRE(o.nu_mode == 0 || o.nu_mode == 1, "irm_solve: nu_mode must be 0 or 1");
  size_t need = 0;
  NYS_TRY(irm_workspace_size(prob, dt, ell, &need));
  NYS_TRY(check_workspace(ws, ws_bytes, need, "irm_solve"));
  WsBind bind(ws, ws_bytes, prob->op, nullptr);
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return irm_impl<double>(*prob, o, static_cast<const double*>(omega), ell,
                            static_cast<const double*>(x0), static_cast<double*>(x), cg_iters,
                            outer_done, info, &bind.s, st);
  return irm_impl<float>(*prob, o, static_cast<const float*>(omega), ell,
                         static_cast<const float*>(x0), static_cast<float*>(x), cg_iters,
                         outer_done, info, &bind.s, st);
}
