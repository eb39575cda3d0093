// WAPG (Alg. 3), its step size by the power method (eq. (20) constant), and
// the cost F = f + lambda g with FP64 accumulation.

#include <cmath>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "stencil.hpp"

namespace nys {

template <class T> nys_status fill_zero(T* p, size_t n, hipStream_t st);

// ---------------------------------------------------------------- elementwise
// r = (A u) - y, then psi'(r) = clip(r / delta, -1, 1) for the Huber loss
template <class T>
__global__ void residual_kernel(T* __restrict__ r, const T* __restrict__ y, int64_t M, int loss,
                                T delta) {
  const int64_t m = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (m >= M) return;
  T v = r[m] - y[m];
  if (loss == NYS_LOSS_HUBER) v = fmin(T(1), fmax(T(-1), v / delta));
  r[m] = v;
}

// s = u - alpha g
template <class T>
__global__ void step_kernel(const T* __restrict__ u, const T* __restrict__ g, T alpha, int64_t N,
                            T* __restrict__ s) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  s[n] = u[n] - alpha * g[n];
}

// u = x+ + beta (x+ - x);  x = x+.  With betas given, beta is
// betas[*ctr + j] (a graph replayed over the iterations).
template <class T>
__global__ void momentum_kernel(const T* __restrict__ xn, T* __restrict__ x, T* __restrict__ u,
                                T beta, int64_t N, const double* __restrict__ betas,
                                const int32_t* __restrict__ ctr, int j) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  if (betas != nullptr) beta = static_cast<T>(betas[*ctr + j]);
  T a = xn[n];
  u[n] = a + beta * (a - x[n]);
  x[n] = a;
}

// *ctr = 0, or *ctr += step
__global__ void counter_kernel(int32_t* ctr, int step, int reset) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = reset ? 0 : *ctr + step;
}

// status = NYS_ENOTFINITE when any of v[0:n] is NaN or infinite (the word
// was cleared at the start of the call)
template <class T>
__global__ __launch_bounds__(256) void finite_check_kernel(const T* __restrict__ v, int64_t n,
                                                           int32_t* __restrict__ status) {
  bool bad = false;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    bad |= !isfinite(v[i]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) status[0] = NYS_ENOTFINITE;
}

__global__ void status_clear_kernel(int32_t* status) {
  if (threadIdx.x < 2) status[threadIdx.x] = 0;
}

// ---------------------------------------------------------------- reductions
template <class T>
__global__ __launch_bounds__(256) void term_sum_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                       int64_t n, int which, T delta, int n1, int n2,
                                                       double* __restrict__ part) {
  double s = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s += term_at(a, b, i, which, delta, n1, n2);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = w0 * sum(part0[0:n0]) + w1 * sum(part1[0:n1]) on one wave (lane
// sums over a fixed stride, then a fixed butterfly: the same order on every
// call); with ctr given, out[*ctr + j] (a graph replayed over the iterations)
__global__ __launch_bounds__(64) void combine_kernel(const double* __restrict__ p0, int n0,
                                                     double w0, const double* __restrict__ p1,
                                                     int n1, double w1, double* __restrict__ out,
                                                     const int32_t* __restrict__ ctr, int j) {
  const int l = threadIdx.x;
  double a = 0, b = 0;
  for (int i = l; i < n0; i += 64) a += p0[i];
  for (int i = l; i < n1; i += 64) b += p1[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (l == 0) out[ctr != nullptr ? *ctr + j : 0] = w0 * a + w1 * b;
}

// v = w / ||w||, norm[it] = ||w|| (power method, FP64 norm)
template <class T>
__global__ void scale_by_norm_kernel(const T* __restrict__ w, T* __restrict__ v, int64_t N,
                                     const double* __restrict__ part, int np,
                                     double* __restrict__ norm_out) {
  __shared__ double nrm;
  if (threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < np; ++i) s += part[i];
    nrm = sqrt(s);
    if (blockIdx.x == 0) *norm_out = nrm;
  }
  __syncthreads();
  const T inv = static_cast<T>(nrm > 0 ? 1.0 / nrm : 0.0);
  for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[n] = w[n] * inv;
}

template <class T>
__global__ __launch_bounds__(256) void sumsq_kernel(const T* __restrict__ a, int64_t n,
                                                    double* __restrict__ part) {
  double s = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double v = static_cast<double>(a[i]);
    s += v * v;
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

constexpr int kRedBlocks = 256;

// Workspace of one solve, carved from one device buffer:
// meas (M), g, s, xn, u, v (N each), state (TV/HS dual or SSN gamma),
// part (2 kRedBlocks doubles), norms (8 doubles), prox work.
template <class T>
struct SolveWs {
  T *meas, *g, *s, *xn, *u, *v;
  T* au;      // A applied to the rows of U (ell_pad rows, pitch ldau), when M < N; else null
  T* ucopy;   // U's rows without the pitch (ell_pad x N), the input of A U
  T* aucont;  // A U as the operator writes it (ell_pad x M)
  int64_t ldau = 0;
  void* state;
  double *part, *norms;
  void* prox;
  static int nch(const nys_reg_desc& r) { return reg_hessian(r.kind) ? 3 : (r.kind == NYS_REG_L1 ? 0 : 2); }
  static size_t state_bytes(const nys_problem& p, nys_pc pc) {
    const int c = nch(p.reg);
    return c ? sizeof(T) * c * p.op->N : (pc ? sizeof(double) * pc->ell : 0);
  }
  // U^T g with g = A^T psi is (A U)^T psi: a pass over M values per column of
  // U instead of N, once A U is formed (per solve)
  static bool use_au(const nys_problem& p, nys_pc pc) { return pc && p.op->M < p.op->N; }
  // row pitch of A U: a multiple of 4 values, padded off a power-of-two
  // stride (rows read together would fall on the same memory channels)
  static int64_t au_pitch(int64_t M) { return (M + 3) / 4 * 4 + (M >= 16384 ? 96 : 0); }
  static size_t au_bytes(const nys_problem& p, nys_pc pc) {
    return use_au(p, pc) ? sizeof(T) * static_cast<size_t>(pc->ell_pad) *
                               (au_pitch(p.op->M) + p.op->N + p.op->M)
                         : 0;
  }
  static size_t bytes(const nys_problem& p, nys_pc pc) {
    auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
    return r256(sizeof(T) * (p.op->M + 5 * p.op->N)) + r256(state_bytes(p, pc)) +
           r256(sizeof(double) * (2 * kRedBlocks + 8)) + r256(prox_ws_bytes<T>(p.reg) + 256) +
           r256(au_bytes(p, pc));
  }
  SolveWs(const nys_problem& p, nys_pc pc, void* base_v) {
    auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
    char* base = static_cast<char*>(base_v);
    const int64_t N = p.op->N, M = p.op->M;
    meas = reinterpret_cast<T*>(base);
    g = meas + M;
    s = g + N;
    xn = s + N;
    u = xn + N;
    v = u + N;
    char* after = base + r256(sizeof(T) * (M + 5 * N));
    const size_t sb = state_bytes(p, pc);
    state = sb ? after : nullptr;
    after += r256(sb);
    part = reinterpret_cast<double*>(after);
    norms = part + 2 * kRedBlocks;
    after += r256(sizeof(double) * (2 * kRedBlocks + 8));
    prox = after;
    after += r256(prox_ws_bytes<T>(p.reg) + 256);
    au = use_au(p, pc) ? reinterpret_cast<T*>(after) : nullptr;
    ldau = au ? au_pitch(M) : 0;
    ucopy = au ? au + static_cast<size_t>(pc->ell_pad) * ldau : nullptr;
    aucont = au ? ucopy + static_cast<size_t>(pc->ell_pad) * N : nullptr;
  }
};

template <class T>
static int reg_term(const nys_reg_desc& r) {
  return reg_term_of(r.kind);
}

template <class T>
static nys_status cost_impl(const nys_problem& p, const T* x, double* cost, T* meas, double* part,
                            hipStream_t st, const int32_t* ctr = nullptr, int j = 0) {
  nys_op op = p.op;
  NYS_TRY(op_fwd<T>(op, x, meas, 1, st));
  const int which = p.loss == NYS_LOSS_HUBER ? kHuber : kSq;
  hipLaunchKernelGGL((term_sum_kernel<T>), dim3(kRedBlocks), dim3(256), 0, st, meas,
                     static_cast<const T*>(p.y), op->M, which, static_cast<T>(p.delta), 0, 1, part);
  NYS_TRY(launch_check("term_sum_kernel"));
  hipLaunchKernelGGL((term_sum_kernel<T>), dim3(kRedBlocks), dim3(256), 0, st, x,
                     static_cast<const T*>(nullptr), op->N, reg_term<T>(p.reg),
                     static_cast<T>(0), p.reg.n1, p.reg.n2, part + kRedBlocks);
  NYS_TRY(launch_check("term_sum_kernel"));
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, st, part, kRedBlocks, 1.0,
                     part + kRedBlocks, kRedBlocks, p.lambda, cost, ctr, j);
  return launch_check("combine_kernel");
}

// One power-method step: w = P^{-1} A^T A v (into g), norm, v = w / ||w||.
template <class T>
static nys_status power_step(const nys_problem& p, nys_pc pc, T* v, T* g, T* meas, double* part,
                             double* norm_out, hipStream_t st) {
  nys_op op = p.op;
  const int64_t N = op->N;
  NYS_TRY(op_fwd<T>(op, v, meas, 1, st));
  NYS_TRY(op_adj<T>(op, meas, g, 1, st));
  if (pc) NYS_TRY(pc_apply<T>(pc, true, g, g, 1, st));
  hipLaunchKernelGGL((sumsq_kernel<T>), dim3(kRedBlocks), dim3(256), 0, st, g, N, part);
  NYS_TRY(launch_check("sumsq_kernel"));
  hipLaunchKernelGGL((scale_by_norm_kernel<T>), dim3(std::min<int64_t>(cdiv(N, 256), 1024)),
                     dim3(256), 0, st, g, v, N, part, kRedBlocks, norm_out);
  return launch_check("scale_by_norm_kernel");
}

// Power method (no host synchronisation): the estimate of
// lambda_max(P^{-1} A^T A) is left in w.norms[0] on the device.
template <class T>
nys_status power_enqueue(const nys_problem& p, nys_pc pc, const T* v0, int iters, void* wsb,
                         hipStream_t st) {
  SolveWs<T> w(p, pc, wsb);
  const int64_t N = p.op->N;
  NYS_CHECK_HIP(hipMemcpyAsync(w.g, v0, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL((sumsq_kernel<T>), dim3(kRedBlocks), dim3(256), 0, st, w.g, N, w.part);
  NYS_TRY(launch_check("sumsq_kernel"));
  hipLaunchKernelGGL((scale_by_norm_kernel<T>), dim3(std::min<int64_t>(cdiv(N, 256), 1024)),
                     dim3(256), 0, st, w.g, w.v, N, w.part, kRedBlocks, w.norms);
  NYS_TRY(launch_check("scale_by_norm_kernel"));
  for (int it = 0; it < iters; ++it)
    NYS_TRY(power_step<T>(p, pc, w.v, w.g, w.meas, w.part, w.norms, st));
  return NYS_OK;
}

// WAPG start: x = u = 0, the prox state cleared, and A U formed when it is
// held (the operator's rows of U, for the coefficients (A U)^T psi).
template <class T>
static nys_status wapg_setup(const nys_problem& p, nys_pc pc, T* x, const SolveWs<T>& w,
                             hipStream_t st) {
  nys_op op = p.op;
  const int64_t N = op->N, M = op->M;
  const int nch = SolveWs<T>::nch(p.reg);
  NYS_TRY(fill_zero<T>(x, N, st));
  NYS_TRY(fill_zero<T>(w.u, N, st));
  if (nch) NYS_TRY(fill_zero<T>(static_cast<T*>(w.state), static_cast<size_t>(nch) * N, st));
  else if (w.state) NYS_TRY(fill_zero<double>(static_cast<double*>(w.state), pc->ell, st));
  // the prox's kept warm-start coefficients: those of Q = 0
  if (nch && pc) NYS_TRY(fill_zero<double>(static_cast<double*>(w.prox), PcMeta::kMaxEll, st));
  if (w.au) {
    // A U: U's rows (zero past ell) packed, then the operator on all of them
    NYS_CHECK_HIP(hipMemcpy2DAsync(w.ucopy, sizeof(T) * N, pc->U.p, sizeof(T) * pc->ldu,
                                   sizeof(T) * N, pc->ell_pad, hipMemcpyDeviceToDevice, st));
    NYS_TRY(op_fwd<T>(op, w.ucopy, w.aucont, pc->ell_pad, st));
    NYS_CHECK_HIP(hipMemcpy2DAsync(w.au, sizeof(T) * w.ldau, w.aucont, sizeof(T) * M, sizeof(T) * M,
                                   pc->ell_pad, hipMemcpyDeviceToDevice, st));
  }
  return NYS_OK;
}

// Where a replayed iteration finds its momentum weight and cost slot:
// betas[*ctr + j] and costs[*ctr + j] (null: beta and costs + k from the host).
struct WapgIdx {
  const double* betas = nullptr;
  const int32_t* ctr = nullptr;
  int j = 0;
};

// One WAPG iteration (Alg. 3): s = u - alpha P^{-1} grad f(u), x+ = prox^P(s),
// the momentum step with weight beta, and F(x+) into cost when given.
// Returns NYS_ENOCONV (and goes on) when a semismooth Newton prox ran out of
// trial points.
template <class T>
static nys_status wapg_iter(const nys_problem& p, nys_pc pc, double alpha, int warm_start, T* x,
                            const SolveWs<T>& w, double beta, double* cost, const WapgIdx& ix,
                            hipStream_t st) {
  nys_op op = p.op;
  const int64_t N = op->N, M = op->M;
  const double lam_bar = alpha * p.lambda;
  Scratch::Mark mark(op->scr);   // this iteration's coefficient partials
  nys_status conv = NYS_OK;
  // s = u - alpha P^{-1} grad f(u), grad f(u) = A^T psi(A u - y)
  if (op_fwd_fused_ok<T>(op)) {
    NYS_TRY(op_fwd_psi<T>(op, w.u, static_cast<const T*>(p.y), p.loss, p.delta, w.meas, 1, st));
  } else {
    NYS_TRY(op_fwd<T>(op, w.u, w.meas, 1, st));
    hipLaunchKernelGGL((residual_kernel<T>), dim3(cdiv(M, 256)), dim3(256), 0, st, w.meas,
                       static_cast<const T*>(p.y), M, p.loss, static_cast<T>(p.delta));
    NYS_TRY(launch_check("residual_kernel"));
  }
  // cd = d . U^T grad (eq. (11)): partials of (A U)^T psi where A U is held,
  // else of U^T grad
  CoefPartials cp;
  if (w.au) NYS_TRY(pc_partials_on<T>(pc, w.au, w.ldau, M, w.meas, 1, &cp, st));
  NYS_TRY(op_adj<T>(op, w.meas, w.g, 1, st));
  if (pc && !w.au) NYS_TRY(pc_partials_on<T>(pc, pc->U.as<T>(), pc->ldu, N, w.g, 1, &cp, st));
  if (pc && p.reg.kind == NYS_REG_L1) {
    // the step s = u - alpha (grad + U cd) is formed inside the prox (by
    // its first evaluation pass over U where possible)
    const SsnStep sp{w.u, w.g, alpha, cp, w.part};
    const nys_status ps = ssn_prox<T>(p.reg, lam_bar, pc, w.s, w.xn,
                                      warm_start ? static_cast<double*>(w.state) : nullptr, st,
                                      nullptr, &sp);
    if (ps == NYS_ENOCONV) conv = ps;
    else if (ps != NYS_OK) return ps;
  } else if (pc) {
    NYS_TRY(pc_tail(pc, true, cp, w.part, st));
    NYS_TRY(pc_x_from_pinv<T>(pc, w.u, w.g, w.part, alpha, w.s, st));
  } else {
    hipLaunchKernelGGL((step_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, w.u, w.g,
                       static_cast<T>(alpha), N, w.s);
    NYS_TRY(launch_check("step_kernel"));
  }
  // x+ = prox^P_{alpha lambda g}(s)
  if (!(pc && p.reg.kind == NYS_REG_L1)) {
    const nys_status ps = prox_run<T>(p.reg, lam_bar, pc, w.s, w.xn,
                                      warm_start ? w.state : nullptr, st, w.prox, warm_start);
    if (ps == NYS_ENOCONV) conv = ps;
    else if (ps != NYS_OK) return ps;
  }
  hipLaunchKernelGGL((momentum_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, w.xn, x, w.u,
                     static_cast<T>(beta), N, ix.betas, ix.ctr, ix.j);
  NYS_TRY(launch_check("momentum_kernel"));
  if (cost) NYS_TRY(cost_impl<T>(p, x, cost, w.meas, w.part, st, ix.ctr, ix.j));
  return conv;
}

// The momentum weights of Alg. 3: t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
// beta_k = (t_k - 1) / t_{k+1}.
static std::vector<double> wapg_betas(int n) {
  std::vector<double> b(std::max(n, 0));
  double t_prev = 1.0;
  for (int k = 0; k < n; ++k) {
    const double t = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t_prev * t_prev));
    b[k] = (t_prev - 1.0) / t;
    t_prev = t;
  }
  return b;
}

// WAPG outer iterations with a known step (no host synchronisation for the
// TV / HS priors once pc->pinv_norm_cache is set).
template <class T>
nys_status wapg_enqueue(const nys_problem& p, nys_pc pc, double alpha, int max_iter,
                        int warm_start, T* x, double* costs, void* wsb, hipStream_t st) {
  SolveWs<T> w(p, pc, wsb);
  NYS_TRY(wapg_setup<T>(p, pc, x, w, st));
  const std::vector<double> betas = wapg_betas(max_iter);
  nys_status conv = NYS_OK;   // a prox that ran out of Newton trials (the solve goes on)
  for (int k = 0; k < max_iter; ++k) {
    const nys_status s = wapg_iter<T>(p, pc, alpha, warm_start, x, w, betas[k],
                                      costs ? costs + k : nullptr, WapgIdx{}, st);
    if (s == NYS_ENOCONV) conv = s;
    else if (s != NYS_OK) return s;
  }
  return conv;
}

template nys_status power_enqueue<float>(const nys_problem&, nys_pc, const float*, int, void*, hipStream_t);
template nys_status power_enqueue<double>(const nys_problem&, nys_pc, const double*, int, void*, hipStream_t);
template nys_status wapg_enqueue<float>(const nys_problem&, nys_pc, double, int, int, float*, double*, void*, hipStream_t);
template nys_status wapg_enqueue<double>(const nys_problem&, nys_pc, double, int, int, double*, double*, void*, hipStream_t);


// Workspace of solve: the status word, the iteration's buffers (SolveWs),
// and the scratch of the operator (on one column, or on ell_pad columns when
// A U is formed) and of the preconditioner's applications.
template <class T>
size_t solve_call_ws_bytes(const nys_problem& p, nys_pc pc) {
  const int64_t cols = SolveWs<T>::use_au(p, pc) ? pc->ell_pad : 1;
  // the gradient step's coefficient partials are held while the prox takes
  // its own: two columns' worth of the preconditioner's scratch
  return 256 + ws_round(SolveWs<T>::bytes(p, pc)) + op_ws_bytes(p.op, sizeof(T), cols) +
         (pc ? pc_ws_bytes(pc, 2) : 0);
}

template <class T>
static nys_status solve_impl(const nys_problem& p, nys_pc pc, const nys_solve_opts& o, T* x,
                             double* costs, double* info, void* ws, size_t ws_bytes,
                             hipStream_t st) {
  NYS_TRY(check_workspace(ws, ws_bytes, solve_call_ws_bytes<T>(p, pc), "solve"));
  WsBind bind(ws, ws_bytes, p.op, pc);
  int32_t* status = nullptr;
  char* wsb = nullptr;
  NYS_TAKE(&bind.s, int32_t, status, 64);
  NYS_TAKE(&bind.s, char, wsb, SolveWs<T>::bytes(p, pc));
  SolveWs<T> w(p, pc, wsb);
  hipLaunchKernelGGL(status_clear_kernel, dim3(1), dim3(64), 0, st, status);
  NYS_TRY(launch_check("status_clear_kernel"));
  const double curv = p.loss == NYS_LOSS_HUBER ? 1.0 / p.delta : 1.0;
  double alpha = o.alpha;
  double Lest = 0.0;
  if (!(alpha > 0)) {
    NYS_REQUIRE(o.power_v0 && o.power_iters > 0, "solve: power_v0 / power_iters needed when alpha <= 0");
    NYS_TRY(power_enqueue<T>(p, pc, static_cast<const T*>(o.power_v0), o.power_iters, wsb, st));
    double lam = 0;
    NYS_CHECK_HIP(hipMemcpyAsync(&lam, w.norms, sizeof(double), hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    Lest = curv * lam;
    const double safety = o.safety > 0 ? o.safety : 1.01;
    if (!(Lest > 0 && std::isfinite(Lest))) {
      set_error("solve: the power method gave L = %g (non-finite or non-positive inputs)", Lest);
      return std::isfinite(Lest) ? NYS_EINVAL : NYS_ENOTFINITE;
    }
    alpha = 1.0 / (safety * Lest);
  }
  const nys_status ws_status =
      wapg_enqueue<T>(p, pc, alpha, o.max_iter, o.warm_start, x, costs, wsb, st);
  if (ws_status != NYS_OK && ws_status != NYS_ENOCONV) return ws_status;
  hipLaunchKernelGGL((finite_check_kernel<T>),
                     dim3(std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(p.op->N, 256)))),
                     dim3(256), 0, st, x, p.op->N, status);
  NYS_TRY(launch_check("finite_check_kernel"));
  nys_status result = ws_status;
  if (info) {
    int32_t dev_status = 0;
    NYS_CHECK_HIP(hipMemcpyAsync(&dev_status, status, sizeof dev_status, hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    if (dev_status != NYS_OK) {
      set_error("solve: the iterate holds non-finite values");
      result = static_cast<nys_status>(dev_status);
    }
    info[0] = alpha;
    info[1] = Lest;
    info[2] = result;
    info[3] = 0;
  }
  if (result == NYS_ENOCONV)
    set_error("solve: a semismooth Newton prox ran out of trial points (the iteration went on)");
  return result;
}

}  // namespace nys

using namespace nys;

static nys_status check_problem(const nys_problem* p, nys_dtype dt) {
  NYS_REQUIRE(p && p->op && p->y, "solve: null problem, operator or y");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "solve: dtype must be F64 or F32");
  NYS_REQUIRE(static_cast<int64_t>(p->reg.n1) * p->reg.n2 == p->op->N,
              "solve: regulariser size != number of unknowns");
  NYS_REQUIRE(p->loss == NYS_LOSS_LS || (p->loss == NYS_LOSS_HUBER && p->delta > 0),
              "solve: bad loss / delta");
  NYS_REQUIRE(p->lambda >= 0, "solve: lambda < 0");
  NYS_TRY(check_box(p->reg));
  return NYS_OK;
}

extern "C" nys_status nys_workspace_size(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                         size_t* bytes) {
  NYS_TRY(check_problem(prob, dt));
  NYS_REQUIRE(bytes, "nys_workspace_size: null bytes");
  if (pc) NYS_REQUIRE(pc->N == prob->op->N, "nys_workspace_size: pc size != number of unknowns");
  *bytes = dt == NYS_F64 ? solve_call_ws_bytes<double>(*prob, pc)
                         : solve_call_ws_bytes<float>(*prob, pc);
  return NYS_OK;
}

extern "C" nys_status solve(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                            const nys_solve_opts* opts, void* x_out, double* costs, double* info,
                            void* ws, size_t ws_bytes, void* stream) {
  NYS_TRY(check_problem(prob, dt));
  NYS_REQUIRE(opts && x_out && opts->max_iter >= 0, "solve: bad options or x_out");
  NYS_REQUIRE(prob->lambda > 0, "solve: lambda must be > 0");
  if (pc) {
    NYS_REQUIRE(pc->N == prob->op->N, "solve: pc size != number of unknowns");
    NYS_REQUIRE(pc->u_dtype == static_cast<int32_t>(dt), "solve: pc u_dtype != solver dtype");
  }
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return solve_impl<double>(*prob, pc, *opts, static_cast<double*>(x_out), costs, info, ws,
                              ws_bytes, st);
  return solve_impl<float>(*prob, pc, *opts, static_cast<float*>(x_out), costs, info, ws, ws_bytes,
                           st);
}

extern "C" nys_status nys_cost_workspace_size(const nys_problem* prob, nys_dtype dt, size_t* bytes) {
  NYS_TRY(check_problem(prob, dt));
  NYS_REQUIRE(bytes, "nys_cost_workspace_size: null bytes");
  *bytes = ws_round(sizeof(double) * 2 * kRedBlocks) + ws_round(dtype_size(dt) * prob->op->M) +
           op_ws_bytes(prob->op, dtype_size(dt), 1);
  return NYS_OK;
}

extern "C" nys_status nys_cost(const nys_problem* prob, nys_dtype dt, const void* x, double* cost,
                               void* ws, size_t ws_bytes, void* stream) {
  NYS_TRY(check_problem(prob, dt));
  NYS_REQUIRE(x && cost, "nys_cost: null x / cost");
  size_t need = 0;
  NYS_TRY(nys_cost_workspace_size(prob, dt, &need));
  NYS_TRY(check_workspace(ws, ws_bytes, need, "nys_cost"));
  WsBind bind(ws, ws_bytes, prob->op, nullptr);
  hipStream_t st = as_stream(stream);
  double* part = nullptr;
  char* meas = nullptr;
  NYS_TAKE(&bind.s, double, part, 2 * kRedBlocks);
  NYS_TAKE(&bind.s, char, meas, dtype_size(dt) * prob->op->M);
  if (dt == NYS_F64)
    return cost_impl<double>(*prob, static_cast<const double*>(x), cost,
                             reinterpret_cast<double*>(meas), part, st);
  return cost_impl<float>(*prob, static_cast<const float*>(x), cost, reinterpret_cast<float*>(meas),
                          part, st);
}

// ================================================================ captured solve
// A fixed-count WAPG solve as HIP graphs captured once: the start (status
// word, x = u = 0, prox state, A U), a chunk of G iterations replayed
// max_iter / G times, the remaining iterations, and the final finite check.
// The replays find their momentum weight and cost slot through a device
// counter that the chunk advances; the host only enqueues graph launches.
struct nys_solve_plan_s {
  hipStream_t cs = nullptr;             // the capturing stream (never run on)
  hipGraph_t g[4] = {};                 // start, chunk, remainder, end
  hipGraphExec_t e[4] = {};
  int nchunk = 0;
  double* dev = nullptr;                // betas (max_iter), then the counter
  double alpha = 0, L = 0;
  ~nys_solve_plan_s() {
    for (int i = 0; i < 4; ++i) {
      if (e[i]) (void)hipGraphExecDestroy(e[i]);
      if (g[i]) (void)hipGraphDestroy(g[i]);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (dev) (void)hipFree(dev);
  }
};

namespace nys {

constexpr int kPlanChunk = 16;

// Runs `body` under capture on plan->cs into graph slot i.
template <class F>
static nys_status plan_capture(nys_solve_plan_s* plan, int i, F&& body) {
  NYS_CHECK_HIP(hipStreamBeginCapture(plan->cs, hipStreamCaptureModeThreadLocal));
  const nys_status s = body(plan->cs);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(plan->cs, &g);
  if (s != NYS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (ee != hipSuccess || !g) {
    set_error("nys_solve_plan_create: capture failed: %s", hipGetErrorString(ee));
    return NYS_EHIP;
  }
  plan->g[i] = g;
  if (hipGraphInstantiate(&plan->e[i], g, nullptr, nullptr, 0) != hipSuccess) {
    set_error("nys_solve_plan_create: hipGraphInstantiate failed");
    return NYS_EHIP;
  }
  return NYS_OK;
}

template <class T>
static nys_status plan_create_impl(const nys_problem& p, nys_pc pc, const nys_solve_opts& o,
                                   T* x, double* costs, void* ws, size_t ws_bytes, hipStream_t st,
                                   nys_solve_plan_s* plan) {
  NYS_TRY(check_workspace(ws, ws_bytes, solve_call_ws_bytes<T>(p, pc), "nys_solve_plan_create"));
  WsBind bind(ws, ws_bytes, p.op, pc);
  int32_t* status = nullptr;
  char* wsb = nullptr;
  NYS_TAKE(&bind.s, int32_t, status, 64);
  NYS_TAKE(&bind.s, char, wsb, SolveWs<T>::bytes(p, pc));
  SolveWs<T> w(p, pc, wsb);
  // the step, by the power method on the caller's stream when not given
  double alpha = o.alpha;
  if (!(alpha > 0)) {
    NYS_REQUIRE(o.power_v0 && o.power_iters > 0,
                "nys_solve_plan_create: power_v0 / power_iters needed when alpha <= 0");
    NYS_TRY(power_enqueue<T>(p, pc, static_cast<const T*>(o.power_v0), o.power_iters, wsb, st));
    double lam = 0;
    NYS_CHECK_HIP(hipMemcpyAsync(&lam, w.norms, sizeof(double), hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    const double curv = p.loss == NYS_LOSS_HUBER ? 1.0 / p.delta : 1.0;
    plan->L = curv * lam;
    if (!(plan->L > 0 && std::isfinite(plan->L))) {
      set_error("nys_solve_plan_create: the power method gave L = %g", plan->L);
      return std::isfinite(plan->L) ? NYS_EINVAL : NYS_ENOTFINITE;
    }
    alpha = 1.0 / ((o.safety > 0 ? o.safety : 1.01) * plan->L);
  }
  plan->alpha = alpha;
  // ||P^{-1}||, which the P-weighted dual prox reads on the host, once
  if (pc && pc->pinv_norm_cache < 0) {
    double hm[PcMeta::kTotal];
    NYS_CHECK_HIP(hipMemcpyAsync(hm, pc->meta.p, sizeof hm, hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    pc->pinv_norm_cache = hm[PcMeta::kPinvNorm];
  }
  // the P-weighted l1 prox: its captured trials need stored Jacobian factors
  // of this preconditioner, which one host-driven iteration leaves behind
  const bool l1pc = pc && p.reg.kind == NYS_REG_L1;
  if (l1pc && !pc->ssn_lu_valid) {
    NYS_TRY(wapg_setup<T>(p, pc, x, w, st));
    const nys_status s0 = wapg_iter<T>(p, pc, alpha, o.warm_start, x, w, 0.0, nullptr, WapgIdx{}, st);
    if (s0 != NYS_OK && s0 != NYS_ENOCONV) return s0;
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    NYS_REQUIRE(pc->ssn_lu_valid, "nys_solve_plan_create: no stored Newton factors");
  }
  struct SsnDeviceMode {   // the semismooth Newton calls of the capture decide on the device
    nys_pc pc;
    SsnDeviceMode(nys_pc q, int32_t* status) : pc(q) {
      if (pc) { pc->ssn_device = true; pc->ssn_status = status; }
    }
    ~SsnDeviceMode() {
      if (pc) { pc->ssn_device = false; pc->ssn_status = nullptr; }
    }
  } ssn_mode(l1pc ? pc : nullptr, status);
  const int K = o.max_iter;
  const std::vector<double> betas = wapg_betas(K);
  NYS_CHECK_HIP(hipMalloc(&plan->dev, sizeof(double) * (K + 1)));
  if (K > 0)
    NYS_CHECK_HIP(hipMemcpy(plan->dev, betas.data(), sizeof(double) * K, hipMemcpyHostToDevice));
  int32_t* ctr = reinterpret_cast<int32_t*>(plan->dev + K);
  NYS_CHECK_HIP(hipStreamCreateWithFlags(&plan->cs, hipStreamNonBlocking));
  const int G = std::min(kPlanChunk, std::max(K, 1));
  plan->nchunk = K / G;
  const int rem = K - plan->nchunk * G;
  NYS_TRY(plan_capture(plan, 0, [&](hipStream_t cs) -> nys_status {
    hipLaunchKernelGGL(status_clear_kernel, dim3(1), dim3(64), 0, cs, status);
    NYS_TRY(launch_check("status_clear_kernel"));
    NYS_TRY(wapg_setup<T>(p, pc, x, w, cs));
    hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, cs, ctr, 0, 1);
    return launch_check("counter_kernel");
  }));
  auto iters = [&](int count) {
    return [&, count](hipStream_t cs) -> nys_status {
      for (int j = 0; j < count; ++j)
        NYS_TRY(wapg_iter<T>(p, pc, alpha, o.warm_start, x, w, 0.0, costs,
                             WapgIdx{plan->dev, ctr, j}, cs));
      hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, cs, ctr, count, 0);
      return launch_check("counter_kernel");
    };
  };
  if (plan->nchunk > 0) NYS_TRY(plan_capture(plan, 1, iters(G)));
  if (rem > 0) NYS_TRY(plan_capture(plan, 2, iters(rem)));
  NYS_TRY(plan_capture(plan, 3, [&](hipStream_t cs) -> nys_status {
    hipLaunchKernelGGL((finite_check_kernel<T>),
                       dim3(std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(p.op->N, 256)))),
                       dim3(256), 0, cs, x, p.op->N, status);
    return launch_check("finite_check_kernel");
  }));
  return NYS_OK;
}

}  // namespace nys

extern "C" nys_status nys_solve_plan_create(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                            const nys_solve_opts* opts, void* x_out,
                                            double* costs, void* ws, size_t ws_bytes,
                                            void* stream, double* info, nys_solve_plan* out) {
  NYS_TRY(check_problem(prob, dt));
  NYS_REQUIRE(opts && x_out && out && opts->max_iter >= 0, "nys_solve_plan_create: bad argument");
  NYS_REQUIRE(prob->lambda > 0, "nys_solve_plan_create: lambda must be > 0");
  if (pc) {
    NYS_REQUIRE(pc->N == prob->op->N, "nys_solve_plan_create: pc size != number of unknowns");
    NYS_REQUIRE(pc->u_dtype == static_cast<int32_t>(dt),
                "nys_solve_plan_create: pc u_dtype != solver dtype");
    NYS_REQUIRE(!prob->reg.box, "nys_solve_plan_create: the P-weighted box projection decides "
                "on the host (semismooth Newton); use solve");
    NYS_REQUIRE(prob->reg.kind != NYS_REG_L1 || (dt == NYS_F32 && pc->ell <= 64),
                "nys_solve_plan_create: the P-weighted l1 prox is captured in FP32 with ell <= 64 "
                "only; use solve");
  }
  *out = nullptr;
  auto* plan = new nys_solve_plan_s;
  const hipStream_t st = as_stream(stream);
  const nys_status s =
      dt == NYS_F64
          ? plan_create_impl<double>(*prob, pc, *opts, static_cast<double*>(x_out), costs, ws,
                                     ws_bytes, st, plan)
          : plan_create_impl<float>(*prob, pc, *opts, static_cast<float*>(x_out), costs, ws,
                                    ws_bytes, st, plan);
  if (s != NYS_OK) {
    delete plan;
    return s;
  }
  if (info) {
    info[0] = plan->alpha;
    info[1] = plan->L;
    info[2] = NYS_OK;
    info[3] = 0;
  }
  *out = plan;
  return NYS_OK;
}

extern "C" nys_status nys_solve_plan_run(nys_solve_plan plan, void* stream) {
  NYS_REQUIRE(plan && plan->e[0] && plan->e[3], "nys_solve_plan_run: bad plan");
  const hipStream_t st = as_stream(stream);
  NYS_CHECK_HIP(hipGraphLaunch(plan->e[0], st));
  for (int c = 0; c < plan->nchunk; ++c) NYS_CHECK_HIP(hipGraphLaunch(plan->e[1], st));
  if (plan->e[2]) NYS_CHECK_HIP(hipGraphLaunch(plan->e[2], st));
  NYS_CHECK_HIP(hipGraphLaunch(plan->e[3], st));
  return NYS_OK;
}

extern "C" void nys_solve_plan_destroy(nys_solve_plan plan) { delete plan; }
