// Unrolled WAPG (Alg. 3) with the P-weighted TV prox (dual FISTA, eqs.
// (21)-(29)) for a fixed number of outer and inner iterations, and its exact
// reverse pass (vector-Jacobian products) with respect to the measurements y
// and the regularisation weight lambda.
//
// Forward, per instance: u_0 = x_0 = 0, Q_0 = 0 and for k < K
//   s     = u_k - alpha P^{-1} A^T (A u_k - y)
//   inner: R_0 = Q_k, for i < n:  z_i = s - lb P^{-1} L^T R_i,
//          v_i = R_i + eta L z_i,  Q_{i+1} = Proj(v_i),
//          R_{i+1} = Q_{i+1} + b_i (Q_{i+1} - Q_i)
//   x_{k+1} = s - lb P^{-1} L^T Q_n,   Q_{k+1} = Q_n   (warm start)
//   u_{k+1} = x_{k+1} + g_k (x_{k+1} - x_k)
// with lb = alpha lambda, eta = 1 / (lb ||L||^2 ||P^{-1}||), and the FISTA
// coefficients b_i (inner, restarted per prox) and g_k (outer).
// Checkpoints per outer iteration: u_k and Q_k.  The reverse pass recomputes
// one outer iteration at a time from its checkpoint (storing z_i and v_i),
// then runs the adjoint recursion; Proj is the l2-ball projection (isotropic
// TV) or the box clip (anisotropic TV), differentiated where it is smooth.

#include <cmath>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace nys {

template <class T> nys_status fill_zero(T* p, size_t n, hipStream_t st);

namespace {

// out = L x (first differences, zero on the first row / column)
template <class T>
__global__ __launch_bounds__(256) void l_apply_kernel(const T* __restrict__ x, int n1, int n2,
                                                      T* __restrict__ out) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  const size_t N = static_cast<size_t>(n1) * n2, o = static_cast<size_t>(i) * n2 + j;
  const T xc = x[o];
  out[o] = i >= 1 ? xc - x[o - n2] : T(0);
  out[N + o] = j >= 1 ? xc - x[o - 1] : T(0);
}

// out = L^T q
template <class T>
__global__ __launch_bounds__(256) void lt_apply_kernel(const T* __restrict__ q, int n1, int n2,
                                                       T* __restrict__ out) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  const size_t N = static_cast<size_t>(n1) * n2, o = static_cast<size_t>(i) * n2 + j;
  const T* q1 = q;
  const T* q2 = q + N;
  T v = 0;
  if (i >= 1) v += q1[o];
  if (i + 1 < n1) v -= q1[o + n2];
  if (j >= 1) v += q2[o];
  if (j + 1 < n2) v -= q2[o + 1];
  out[o] = v;
}

// Q+ = Proj(v); R+ = Q+ + beta (Q+ - Qprev)   (Q+ may alias Qprev)
template <class T>
__global__ void proj_momentum_kernel(const T* __restrict__ v, const T* Qprev, T beta, int aniso,
                                     int64_t N, T* Qn, T* __restrict__ Rn) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T a = v[n], b = v[N + n];
  if (aniso) {
    a = fmin(T(1), fmax(T(-1), a));
    b = fmin(T(1), fmax(T(-1), b));
  } else {
    const T nrm = sqrt(a * a + b * b);
    if (nrm > T(1)) { a /= nrm; b /= nrm; }
  }
  const T pa = Qprev[n], pb = Qprev[N + n];
  Qn[n] = a;
  Qn[N + n] = b;
  Rn[n] = a + beta * (a - pa);
  Rn[N + n] = b + beta * (b - pb);
}

// bar_v = J_Proj(v)^T bar_q  (J symmetric)
template <class T>
__global__ void proj_vjp_kernel(const T* __restrict__ v, const T* __restrict__ bq, int aniso,
                                int64_t N, T* __restrict__ bv) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  const T a = v[n], b = v[N + n], ga = bq[n], gb = bq[N + n];
  if (aniso) {
    bv[n] = fabs(a) <= T(1) ? ga : T(0);
    bv[N + n] = fabs(b) <= T(1) ? gb : T(0);
    return;
  }
  const T nrm = sqrt(a * a + b * b);
  if (nrm <= T(1)) {
    bv[n] = ga;
    bv[N + n] = gb;
  } else {
    const T qa = a / nrm, qb = b / nrm;
    const T dotq = qa * ga + qb * gb;
    bv[n] = (ga - qa * dotq) / nrm;
    bv[N + n] = (gb - qb * dotq) / nrm;
  }
}

// out = a x + b y
template <class T>
__global__ void axpby_kernel(T a, const T* x, T b, const T* y, int64_t n, T* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  out[i] = a * x[i] + (y ? b * y[i] : T(0));
}

// r = (A u) - y   in place on r
template <class T>
__global__ void sub_kernel(T* __restrict__ r, const T* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  r[i] -= y[i];
}

// block partials of <x, y - z> (z may be null), FP64
template <class T>
__global__ __launch_bounds__(256) void dot_partial_kernel(const T* __restrict__ x,
                                                          const T* __restrict__ y,
                                                          const T* __restrict__ z, int64_t n,
                                                          double* __restrict__ part) {
  double s = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s += static_cast<double>(x[i]) * (static_cast<double>(y[i]) - (z ? static_cast<double>(z[i]) : 0.0));
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// acc += coef * sum(part[0:np])
__global__ void dot_finish_kernel(const double* __restrict__ part, int np, double coef,
                                  double* __restrict__ acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0;
  for (int i = 0; i < np; ++i) s += part[i];
  *acc += coef * s;
}

constexpr int kDotBlocks = 128;

}  // namespace

// -------------------------------------------------------------- host side
template <class T>
struct Unroll {
  nys_op op;
  nys_pc pc;
  int n1, n2, K, nin, aniso;
  int64_t N, M;
  double alpha, lnorm2, pinv_norm;
  hipStream_t st;
  std::vector<double> g, b;     // outer and inner FISTA coefficients
  // per-instance checkpoint block: u_k (N) and Q_k (2N) for k < K
  static size_t ckpt_elems(int64_t N, int K) { return static_cast<size_t>(K) * 3 * N; }
  // scratch: meas (M), s, t, w, xo (4N), R, Rn, Qc, Lz (8N), z_i (nin N), v_i (2 nin N),
  //          bar: bx, bu, bs, bz (4N), bQ, bR, bQn, bv (8N), by (M); part (kDotBlocks + 8 doubles)
  static size_t scratch_elems(int64_t N, int64_t M, int nin) {
    return 2 * static_cast<size_t>(M) + 24 * static_cast<size_t>(N) + 3 * static_cast<size_t>(nin) * N;
  }

  dim3 g2() const { return dim3(cdiv(n2, 64), cdiv(n1, 4)); }
  unsigned g1(int64_t n) const { return cdiv(n, 256); }

  nys_status pinv(const T* v, T* out) {
    if (!pc) {
      if (v != out) NYS_CHECK_HIP(hipMemcpyAsync(out, v, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
      return NYS_OK;
    }
    return pc_apply<T>(pc, true, v, out, 1, st);
  }
  nys_status axpby(double a, const T* x, double bb, const T* y, int64_t n, T* out) {
    hipLaunchKernelGGL((axpby_kernel<T>), dim3(g1(n)), dim3(256), 0, st, static_cast<T>(a), x,
                       static_cast<T>(bb), y, n, out);
    return launch_check("axpby_kernel");
  }
  nys_status L(const T* x, T* out) {
    hipLaunchKernelGGL((l_apply_kernel<T>), g2(), dim3(256), 0, st, x, n1, n2, out);
    return launch_check("l_apply_kernel");
  }
  nys_status Lt(const T* q, T* out) {
    hipLaunchKernelGGL((lt_apply_kernel<T>), g2(), dim3(256), 0, st, q, n1, n2, out);
    return launch_check("lt_apply_kernel");
  }
  // acc += coef * <x, y - z>
  nys_status dot_acc(const T* x, const T* y, const T* z, int64_t n, double coef, double* part,
                     double* acc) {
    hipLaunchKernelGGL((dot_partial_kernel<T>), dim3(kDotBlocks), dim3(256), 0, st, x, y, z, n, part);
    NYS_TRY(launch_check("dot_partial_kernel"));
    hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(64), 0, st, part, kDotBlocks, coef, acc);
    return launch_check("dot_finish_kernel");
  }
  // s = u - alpha P^{-1} A^T (A u - y)
  nys_status grad_step(const T* u, const T* y, T* meas, T* t, T* s) {
    NYS_TRY(op_fwd<T>(op, u, meas, 1, st));
    hipLaunchKernelGGL((sub_kernel<T>), dim3(g1(M)), dim3(256), 0, st, meas, y, M);
    NYS_TRY(launch_check("sub_kernel"));
    NYS_TRY(op_adj<T>(op, meas, t, 1, st));
    NYS_TRY(pinv(t, t));
    return axpby(1.0, u, -alpha, t, N, s);
  }
  // z = s - lb P^{-1} L^T R
  nys_status z_of(const T* s, const T* R, double lb, T* t, T* z) {
    NYS_TRY(Lt(R, t));
    NYS_TRY(pinv(t, t));
    return axpby(1.0, s, -lb, t, N, z);
  }
  // one inner step from (R, Qprev): v = R + eta L z; Q+ = Proj(v); R+ = ...
  nys_status inner_step(const T* z, const T* R, const T* Qprev, double eta, double beta, T* Lz,
                        T* v, T* Qn, T* Rn) {
    NYS_TRY(L(z, Lz));
    NYS_TRY(axpby(1.0, R, eta, Lz, 2 * N, v));
    hipLaunchKernelGGL((proj_momentum_kernel<T>), dim3(g1(N)), dim3(256), 0, st, v, Qprev,
                       static_cast<T>(beta), aniso, N, Qn, Rn);
    return launch_check("proj_momentum_kernel");
  }
};

template <class T>
static nys_status unroll_setup(Unroll<T>& U, const nys_problem& p, nys_pc pc,
                               const nys_unroll_opts& o, hipStream_t st) {
  U.op = p.op;
  U.pc = pc;
  U.n1 = p.reg.n1;
  U.n2 = p.reg.n2;
  U.K = o.n_outer;
  U.nin = o.n_inner;
  U.aniso = p.reg.kind == NYS_REG_TV_ANISO ? 1 : 0;
  U.N = p.op->N;
  U.M = p.op->M;
  U.alpha = o.alpha;
  U.lnorm2 = p.reg.lnorm2 > 0 ? p.reg.lnorm2 : 8.0;
  U.st = st;
  U.pinv_norm = 1.0;
  if (pc) {
    double hm[PcMeta::kTotal];
    NYS_CHECK_HIP(hipMemcpyAsync(hm, pc->meta.p, sizeof hm, hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    U.pinv_norm = hm[PcMeta::kPinvNorm];
  }
  double t = 1.0;
  U.g.resize(U.K);
  for (int k = 0; k < U.K; ++k) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    U.g[k] = (t - 1.0) / tn;
    t = tn;
  }
  double tau = 1.0;
  U.b.resize(U.nin);
  for (int i = 0; i < U.nin; ++i) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
    U.b[i] = (tau - 1.0) / tn;
    tau = tn;
  }
  return NYS_OK;
}

template <class T>
static nys_status unroll_forward(const nys_problem& p, nys_pc pc, const nys_unroll_opts& o,
                                 int batch, const T* y, const double* lam, T* x, T* ws,
                                 hipStream_t st) {
  Unroll<T> U;
  NYS_TRY(unroll_setup<T>(U, p, pc, o, st));
  const int64_t N = U.N, M = U.M;
  const size_t ck = Unroll<T>::ckpt_elems(N, U.K);
  T* scratch = ws + static_cast<size_t>(batch) * ck;
  T* meas = scratch;
  T* s = meas + M;
  T* t = s + N;
  T* xo = t + N;
  T* u = xo + N;
  T* R = u + N;
  T* Rn = R + 2 * N;
  T* Q = Rn + 2 * N;
  T* Lz = Q + 2 * N;
  T* v = Lz + 2 * N;
  T* z = v + 2 * N;
  for (int b = 0; b < batch; ++b) {
    T* ckb = ws + static_cast<size_t>(b) * ck;
    const T* yb = y + static_cast<size_t>(b) * M;
    T* xb = x + static_cast<size_t>(b) * N;
    const double lb = U.alpha * lam[b];
    const double eta = 1.0 / (lb * U.lnorm2 * U.pinv_norm);
    NYS_TRY(fill_zero<T>(xb, N, st));
    NYS_TRY(fill_zero<T>(u, N, st));
    NYS_TRY(fill_zero<T>(Q, 2 * N, st));
    for (int k = 0; k < U.K; ++k) {
      T* cu = ckb + static_cast<size_t>(k) * 3 * N;
      NYS_CHECK_HIP(hipMemcpyAsync(cu, u, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
      NYS_CHECK_HIP(hipMemcpyAsync(cu + N, Q, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, st));
      NYS_TRY(U.grad_step(u, yb, meas, t, s));
      NYS_CHECK_HIP(hipMemcpyAsync(R, Q, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, st));
      for (int i = 0; i < U.nin; ++i) {
        NYS_TRY(U.z_of(s, R, lb, t, z));
        NYS_TRY(U.inner_step(z, R, Q, eta, U.b[i], Lz, v, Q, Rn));
        std::swap(R, Rn);
      }
      NYS_TRY(U.z_of(s, Q, lb, t, xo));              // x_{k+1}
      // u = x_{k+1} + g (x_{k+1} - x_k);  x_k <- x_{k+1}
      NYS_TRY(U.axpby(1.0 + U.g[k], xo, -U.g[k], xb, N, u));
      NYS_CHECK_HIP(hipMemcpyAsync(xb, xo, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    }
  }
  return NYS_OK;
}

template <class T>
static nys_status unroll_backward(const nys_problem& p, nys_pc pc, const nys_unroll_opts& o,
                                  int batch, const T* y, const double* lam, const T* barx_in,
                                  T* bary, double* barlam, T* ws, hipStream_t st) {
  Unroll<T> U;
  NYS_TRY(unroll_setup<T>(U, p, pc, o, st));
  const int64_t N = U.N, M = U.M;
  const int nin = U.nin;
  const size_t ck = Unroll<T>::ckpt_elems(N, U.K);
  T* scratch = ws + static_cast<size_t>(batch) * ck;
  T* meas = scratch;
  T* s = meas + M;
  T* t = s + N;
  T* w = t + N;
  T* xo = w + N;
  T* R = xo + N;
  T* Rn = R + 2 * N;
  T* Qc = Rn + 2 * N;
  T* Lz = Qc + 2 * N;
  T* bx = Lz + 2 * N;
  T* bu = bx + N;
  T* bs = bu + N;
  T* bz = bs + N;
  T* bQ = bz + N;
  T* bR = bQ + 2 * N;
  T* bQn = bR + 2 * N;
  T* bv = bQn + 2 * N;
  T* Z = bv + 2 * N;                          // z_i, nin x N
  T* V = Z + static_cast<size_t>(nin) * N;    // v_i, nin x 2N
  double* part = reinterpret_cast<double*>(V + static_cast<size_t>(nin) * 2 * N);
  part = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(part) + 255) & ~uintptr_t(255));
  double* acc = part + kDotBlocks;             // [0] d/d lb, [1] d/d eta
  for (int b = 0; b < batch; ++b) {
    T* ckb = ws + static_cast<size_t>(b) * ck;
    const T* yb = y + static_cast<size_t>(b) * M;
    T* byb = bary + static_cast<size_t>(b) * M;
    const double lb = U.alpha * lam[b];
    const double eta = 1.0 / (lb * U.lnorm2 * U.pinv_norm);
    NYS_CHECK_HIP(hipMemcpyAsync(bx, barx_in + static_cast<size_t>(b) * N, sizeof(T) * N,
                                 hipMemcpyDeviceToDevice, st));
    NYS_TRY(fill_zero<T>(bu, N, st));
    NYS_TRY(fill_zero<T>(bQ, 2 * N, st));
    NYS_TRY(fill_zero<T>(byb, M, st));
    NYS_TRY(fill_zero<double>(acc, 2, st));
    for (int k = U.K - 1; k >= 0; --k) {
      const T* cu = ckb + static_cast<size_t>(k) * 3 * N;
      const T* cq = cu + N;
      const double gk = U.g[k];
      // momentum: bar x_{k+1} += (1 + g) bar u_{k+1}; bar x_k = -g bar u_{k+1}
      NYS_TRY(U.axpby(1.0, bx, 1.0 + gk, bu, N, bx));
      NYS_TRY(U.axpby(-gk, bu, 0.0, nullptr, N, w));          // w = bar x_k (held)
      // recompute s and the inner iterates of this outer iteration
      NYS_TRY(U.grad_step(cu, yb, meas, t, s));
      NYS_CHECK_HIP(hipMemcpyAsync(R, cq, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, st));
      NYS_CHECK_HIP(hipMemcpyAsync(Qc, cq, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, st));
      for (int i = 0; i < nin; ++i) {
        T* zi = Z + static_cast<size_t>(i) * N;
        T* vi = V + static_cast<size_t>(i) * 2 * N;
        NYS_TRY(U.z_of(s, R, lb, t, zi));
        NYS_TRY(U.inner_step(zi, R, Qc, eta, U.b[i], Lz, vi, Qc, Rn));
        std::swap(R, Rn);
      }
      NYS_TRY(U.z_of(s, Qc, lb, t, xo));                       // x_{k+1}
      // x_{k+1} = s - lb P^{-1} L^T Q_n
      NYS_CHECK_HIP(hipMemcpyAsync(bs, bx, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
      NYS_TRY(U.pinv(bx, t));
      NYS_TRY(U.L(t, Lz));
      NYS_TRY(U.axpby(1.0, bQ, -lb, Lz, 2 * N, bQn));          // bar Q_n
      NYS_TRY(U.dot_acc(bx, s, xo, N, -1.0 / lb, part, acc));  // d/d lb: -<bx, (s - x)/lb>
      // inner reverse: bQn = bar Q_{i+1}, bR = bar R_{i+1}
      NYS_TRY(fill_zero<T>(bR, 2 * N, st));
      for (int i = nin - 1; i >= 0; --i) {
        const T* zi = Z + static_cast<size_t>(i) * N;
        const T* vi = V + static_cast<size_t>(i) * 2 * N;
        const double bi = U.b[i];
        // R_{i+1} = (1 + b) Q_{i+1} - b Q_i
        NYS_TRY(U.axpby(1.0, bQn, 1.0 + bi, bR, 2 * N, bQn));   // total bar Q_{i+1}
        NYS_TRY(U.axpby(-bi, bR, 0.0, nullptr, 2 * N, Rn));      // partial bar Q_i (kept in Rn)
        // Q_{i+1} = Proj(v_i)
        hipLaunchKernelGGL((proj_vjp_kernel<T>), dim3(U.g1(N)), dim3(256), 0, st, vi, bQn,
                           U.aniso, N, bv);
        NYS_TRY(launch_check("proj_vjp_kernel"));
        // v_i = R_i + eta L z_i
        NYS_TRY(U.L(zi, Lz));
        NYS_TRY(U.dot_acc(bv, Lz, nullptr, 2 * N, 1.0, part, acc + 1));   // d/d eta
        NYS_TRY(U.Lt(bv, bz));
        NYS_TRY(U.axpby(eta, bz, 0.0, nullptr, N, bz));          // bar z_i
        // z_i = s - lb P^{-1} L^T R_i
        NYS_TRY(U.axpby(1.0, bs, 1.0, bz, N, bs));
        NYS_TRY(U.dot_acc(bz, s, zi, N, -1.0 / lb, part, acc));  // -<bz, (s - z_i)/lb>
        NYS_TRY(U.pinv(bz, t));
        NYS_TRY(U.L(t, Lz));
        NYS_TRY(U.axpby(1.0, bv, -lb, Lz, 2 * N, bR));           // bar R_i
        // step to i: bar Q_i (partial) -> bQn
        NYS_CHECK_HIP(hipMemcpyAsync(bQn, Rn, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, st));
      }
      // Q_0 = R_0 = Q_k
      NYS_TRY(U.axpby(1.0, bQn, 1.0, bR, 2 * N, bQ));
      // s = u_k - alpha P^{-1} A^T (A u_k - y)
      NYS_TRY(U.pinv(bs, t));
      NYS_TRY(op_fwd<T>(U.op, t, meas, 1, st));
      NYS_TRY(U.axpby(1.0, byb, U.alpha, meas, M, byb));       // bar y += alpha A P^{-1} bar s
      NYS_TRY(op_adj<T>(U.op, meas, t, 1, st));
      NYS_TRY(U.axpby(1.0, bs, -U.alpha, t, N, bu));          // bar u_k
      NYS_CHECK_HIP(hipMemcpyAsync(bx, w, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    }
    // bar lambda = alpha (bar lb + bar eta d eta / d lb),  d eta / d lb = -eta / lb
    double hacc[2];
    NYS_CHECK_HIP(hipMemcpyAsync(hacc, acc, sizeof hacc, hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    barlam[b] = U.alpha * (hacc[0] - hacc[1] * eta / lb);
  }
  return NYS_OK;
}

// Workspace: the checkpoints and iteration buffers (kept from the forward to
// the backward call), then the scratch of the operator and the
// preconditioner's applications (one column).
template <class T>
static size_t unroll_state_bytes(int64_t N, int64_t M, int K, int nin, int batch) {
  return ws_round(sizeof(T) * (static_cast<size_t>(batch) * Unroll<T>::ckpt_elems(N, K) +
                               Unroll<T>::scratch_elems(N, M, nin)) +
                  sizeof(double) * (kDotBlocks + 8) + 512);
}

template <class T>
static size_t unroll_ws_bytes(nys_op op, nys_pc pc, int K, int nin, int batch) {
  return unroll_state_bytes<T>(op->N, op->M, K, nin, batch) + op_ws_bytes(op, sizeof(T), 1) +
         (pc ? pc_ws_bytes(pc, 1) : 0);
}

}  // namespace nys

using namespace nys;

static nys_status check_unroll(const nys_problem* p, nys_pc pc, nys_dtype dt,
                               const nys_unroll_opts* o, int32_t batch) {
  NYS_REQUIRE(p && p->op && o, "unrolled: null problem, operator or options");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "unrolled: dtype must be F64 or F32");
  NYS_REQUIRE(p->reg.kind == NYS_REG_TV || p->reg.kind == NYS_REG_TV_ANISO,
              "unrolled: regulariser must be TV or anisotropic TV");
  NYS_REQUIRE(!p->reg.box, "unrolled: no box constraint");
  NYS_REQUIRE(static_cast<int64_t>(p->reg.n1) * p->reg.n2 == p->op->N,
              "unrolled: regulariser size != number of unknowns");
  NYS_REQUIRE(p->loss == NYS_LOSS_LS, "unrolled: least-squares data term only");
  NYS_REQUIRE(o->n_outer >= 1 && o->n_inner >= 1 && o->alpha > 0, "unrolled: bad options");
  NYS_REQUIRE(batch >= 1, "unrolled: batch must be >= 1");
  if (pc) {
    NYS_REQUIRE(pc->N == p->op->N, "unrolled: pc size != number of unknowns");
    NYS_REQUIRE(pc->u_dtype == static_cast<int32_t>(dt), "unrolled: pc u_dtype != dtype");
  }
  return NYS_OK;
}

extern "C" nys_status nys_unrolled_workspace(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                             const nys_unroll_opts* opts, int32_t batch,
                                             size_t* bytes) {
  NYS_TRY(check_unroll(prob, pc, dt, opts, batch));
  NYS_REQUIRE(bytes, "nys_unrolled_workspace: null bytes");
  *bytes = dt == NYS_F64 ? unroll_ws_bytes<double>(prob->op, pc, opts->n_outer, opts->n_inner, batch)
                         : unroll_ws_bytes<float>(prob->op, pc, opts->n_outer, opts->n_inner, batch);
  return NYS_OK;
}

extern "C" nys_status unrolled_forward(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                       const nys_unroll_opts* opts, int32_t batch, const void* y,
                                       const double* lambda, void* x, void* ws, size_t ws_bytes,
                                       void* stream) {
  NYS_TRY(check_unroll(prob, pc, dt, opts, batch));
  NYS_REQUIRE(y && lambda && x && ws, "unrolled_forward: null argument");
  size_t need = 0;
  NYS_TRY(nys_unrolled_workspace(prob, pc, dt, opts, batch, &need));
  NYS_TRY(check_workspace(ws, ws_bytes, need, "unrolled_forward"));
  for (int b = 0; b < batch; ++b) NYS_REQUIRE(lambda[b] > 0, "unrolled_forward: lambda must be > 0");
  const size_t keep = dt == NYS_F64
      ? unroll_state_bytes<double>(prob->op->N, prob->op->M, opts->n_outer, opts->n_inner, batch)
      : unroll_state_bytes<float>(prob->op->N, prob->op->M, opts->n_outer, opts->n_inner, batch);
  WsBind bind(static_cast<char*>(ws) + keep, ws_bytes - keep, prob->op, pc);
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return unroll_forward<double>(*prob, pc, *opts, batch, static_cast<const double*>(y), lambda,
                                  static_cast<double*>(x), static_cast<double*>(ws), st);
  return unroll_forward<float>(*prob, pc, *opts, batch, static_cast<const float*>(y), lambda,
                               static_cast<float*>(x), static_cast<float*>(ws), st);
}

extern "C" nys_status unrolled_backward(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                        const nys_unroll_opts* opts, int32_t batch, const void* y,
                                        const double* lambda, const void* bar_x, void* bar_y,
                                        double* bar_lambda, void* ws, size_t ws_bytes,
                                        void* stream) {
  NYS_TRY(check_unroll(prob, pc, dt, opts, batch));
  NYS_REQUIRE(y && lambda && bar_x && bar_y && bar_lambda && ws, "unrolled_backward: null argument");
  size_t need = 0;
  NYS_TRY(nys_unrolled_workspace(prob, pc, dt, opts, batch, &need));
  NYS_TRY(check_workspace(ws, ws_bytes, need, "unrolled_backward"));
  for (int b = 0; b < batch; ++b) NYS_REQUIRE(lambda[b] > 0, "unrolled_backward: lambda must be > 0");
  const size_t keep = dt == NYS_F64
      ? unroll_state_bytes<double>(prob->op->N, prob->op->M, opts->n_outer, opts->n_inner, batch)
      : unroll_state_bytes<float>(prob->op->N, prob->op->M, opts->n_outer, opts->n_inner, batch);
  WsBind bind(static_cast<char*>(ws) + keep, ws_bytes - keep, prob->op, pc);
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return unroll_backward<double>(*prob, pc, *opts, batch, static_cast<const double*>(y), lambda,
                                   static_cast<const double*>(bar_x), static_cast<double*>(bar_y),
                                   bar_lambda, static_cast<double*>(ws), st);
  return unroll_backward<float>(*prob, pc, *opts, batch, static_cast<const float*>(y), lambda,
                                static_cast<const float*>(bar_x), static_cast<float*>(bar_y),
                                bar_lambda, static_cast<float*>(ws), st);
}
