// P-weighted proximal maps (definition in Sec. I-D; C = R^N or a box).
//
// TV / TV_ANISO / Hessian Schatten kinds: accelerated projected gradient on the dual variable Q
// (eqs. (21)-(29)): each inner iteration computes t = L^T R, applies P^{-1},
// forms x = s - lam_bar (P^{-1} t), and updates Q, R with the ball
// projection and momentum.  L1: Thm. 1 with a semismooth Newton method whose
// decisions (accept / backtrack / converge) are taken on the device.

#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "fused.hpp"
#include "internal.hpp"
#include "stencil.hpp"

namespace nys {

// t = L^T q  (or x = s - lam t when s != nullptr, the P = I path)
template <class T>
__global__ __launch_bounds__(256) void lt_kernel(const T* __restrict__ q, int reg, int n1, int n2,
                                                 const T* __restrict__ s, T lam, T* __restrict__ out) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  T v = lt_at(q, reg, i, j, n1, n2);
  const size_t o = static_cast<size_t>(i) * n2 + j;
  out[o] = s ? s[o] - lam * v : v;
}

// Q+ = Proj(R + step L x); R = Q+ + beta (Q+ - Q); Q = Q+
template <class T>
__global__ __launch_bounds__(256) void dual_update_kernel(const T* __restrict__ x, T* __restrict__ Q,
                                                          T* __restrict__ R, int reg, int n1, int n2,
                                                          T step, T beta) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  dual_update_at(x, Q, R, reg, i, j, n1, n2, step, beta);
}

// One fused inner iteration over the tiles of one image (see fused.hpp).
// FP32: static LDS; FP64: the same regions in dynamic LDS (over 64 KiB).
template <int KR, int TW>
__global__ __launch_bounds__(kFThreads) __attribute__((amdgpu_waves_per_eu(4)))
void dual_fused_kernel(FusedArgs A, int ntx, int ntiles, int ntl) {
  __shared__ FusedLds<TW> L;
  extern __shared__ float fused_tail[];  // ntl rows of the tile past the kept ones
  const int tile = fused_tile_of(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  fused_tile<KR, TW>(A, tile, ntx, L, fused_tail, ntl);
}
template <int KR, int TW>
__global__ __launch_bounds__(kFThreads) __attribute__((amdgpu_waves_per_eu(4)))
void dual_fused_f64_kernel(FusedArgsT<double> A, int ntx, int ntiles) {
  extern __shared__ __align__(16) char fused_lds[];
  auto& L = *reinterpret_cast<FusedLds<TW, double>*>(fused_lds);
  const int tile = fused_tile_of(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  fused_tile<KR, TW>(A, tile, ntx, L);
}

// x = s - lam_bar (L^T Q + U c): the prox output from the final dual
template <class T>
__global__ __launch_bounds__(256) void x_from_dual_kernel(const T* __restrict__ s,
                                                          const T* __restrict__ Q, int reg, int n1,
                                                          int n2, const T* __restrict__ U,
                                                          int64_t ldu, const double* __restrict__ cd,
                                                          int L, T lam, T* __restrict__ x) {
  __shared__ T cs[PcMeta::kMaxEll];
  for (int k = threadIdx.x; k < L; k += blockDim.x) cs[k] = static_cast<T>(cd[k]);
  __syncthreads();
  const int64_t N = static_cast<int64_t>(n1) * n2;
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  const int i = static_cast<int>(n / n2), j = static_cast<int>(n - static_cast<int64_t>(i) * n2);
  T acc = 0;
  for (int k = 0; k < L; ++k) acc += U[static_cast<size_t>(k) * ldu + n] * cs[k];
  x[n] = s[n] - lam * (lt_at(Q, reg, i, j, n1, n2) + acc);
}

static int fused_keep(int ell_pad) { return ell_pad < kFKeep ? ell_pad : kFKeep; }
// FP64 values take two registers: 32 rows are kept on the Hessian tiles, 16
// on the wider TV tiles (32 would spill there)
template <int TW> constexpr int fused_keep64() { return TW == fused_tw(true) ? 32 : 16; }

template <int TW>
static nys_status fused_launch_tw(const FusedArgs& A, hipStream_t st) {
  const int ntx = cdiv(A.n2, TW), nty = cdiv(A.n1, kFThreads / TW);
  const int ntiles = ntx * nty;
  const dim3 grid(static_cast<unsigned>((ntiles + 7) / 8 * 8));
  switch (fused_keep(A.ell_pad)) {
    case 16: hipLaunchKernelGGL((dual_fused_kernel<16, TW>), grid, dim3(kFThreads), 0, st, A, ntx, ntiles, 0); break;
    case 32: hipLaunchKernelGGL((dual_fused_kernel<32, TW>), grid, dim3(kFThreads), 0, st, A, ntx, ntiles, 0); break;
    case 48: hipLaunchKernelGGL((dual_fused_kernel<48, TW>), grid, dim3(kFThreads), 0, st, A, ntx, ntiles, 0); break;
    case 64: hipLaunchKernelGGL((dual_fused_kernel<64, TW>), grid, dim3(kFThreads), 0, st, A, ntx, ntiles, 0); break;
    default: {
      // rows past the 80 kept ones: as many as fit in LDS next to the
      // tile's regions with two workgroups per CU (160 KiB per CU) stay
      // there, the rest are read again
      constexpr int kPerCu = 160 * 1024, kSlack = 1024;
      constexpr int kRowBytes = kFThreads * static_cast<int>(sizeof(float));
      constexpr int cap = (kPerCu / 2 - static_cast<int>(sizeof(FusedLds<TW>)) - kSlack) / kRowBytes;
      const int ntl = std::max(0, std::min(A.ell - kFKeep, cap));
      const size_t dyn = static_cast<size_t>(ntl) * kRowBytes;
      if (dyn > 0)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dual_fused_kernel<kFKeep, TW>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn));
      hipLaunchKernelGGL((dual_fused_kernel<kFKeep, TW>), grid, dim3(kFThreads), dyn, st, A, ntx,
                         ntiles, ntl);
      break;
    }
  }
  return launch_check("dual_fused_kernel");
}

template <int TW, int KR>
static nys_status fused_launch_f64_kr(const FusedArgsT<double>& A, dim3 grid, int ntx, int ntiles,
                                      hipStream_t st) {
  constexpr size_t lds = sizeof(FusedLds<TW, double>);
  // the device allows up to 160 KiB per workgroup (a launch without the
  // attribute fails and is reported by launch_check)
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dual_fused_f64_kernel<KR, TW>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  hipLaunchKernelGGL((dual_fused_f64_kernel<KR, TW>), grid, dim3(kFThreads), lds, st, A, ntx,
                     ntiles);
  return launch_check("dual_fused_f64_kernel");
}

template <int TW>
static nys_status fused_launch_tw(const FusedArgsT<double>& A, hipStream_t st) {
  const int ntx = cdiv(A.n2, TW), nty = cdiv(A.n1, kFThreads / TW);
  const int ntiles = ntx * nty;
  const dim3 grid(static_cast<unsigned>((ntiles + 7) / 8 * 8));
  return A.ell_pad <= 16 ? fused_launch_f64_kr<TW, 16>(A, grid, ntx, ntiles, st)
                         : fused_launch_f64_kr<TW, fused_keep64<TW>()>(A, grid, ntx, ntiles, st);
}

template <class T>
static nys_status fused_launch(const FusedArgsT<T>& A, hipStream_t st) {
  return reg_hessian(A.reg) ? fused_launch_tw<fused_tw(true)>(A, st)
                            : fused_launch_tw<fused_tw(false)>(A, st);
}

// tiles of the fused iteration for an image and regulariser kind
static size_t fused_tiles(int n1, int n2, int kind) {
  const int tw = fused_tw(reg_hessian(kind));
  return static_cast<size_t>(cdiv(n1, kFThreads / tw)) * static_cast<size_t>(cdiv(n2, tw));
}

template <class T>
__global__ void zero_kernel(T* p, size_t n) {
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[e] = T(0);
}

template <class T>
nys_status fill_zero(T* p, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((zero_kernel<T>), dim3(std::min<size_t>(cdiv(n, 256), 2048)), dim3(256), 0, st, p, n);
  return launch_check("zero_kernel");
}

// x = clip(x, lo, hi)
template <class T>
__global__ void clip_kernel(T* __restrict__ x, T lo, T hi, int64_t N) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  x[n] = fmin(hi, fmax(lo, x[n]));
}

// x <- prox^P_{delta_C}(x) for the box of reg (eq. (26)): the clip for P = I,
// else Thm. 1's semismooth Newton with the clip, warm-started from gbox
template <class T>
static nys_status project_box(const nys_reg_desc& reg, nys_pc pc, T* x, double* gbox,
                              hipStream_t st) {
  const int64_t N = static_cast<int64_t>(reg.n1) * reg.n2;
  if (!pc) {
    hipLaunchKernelGGL((clip_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, x,
                       static_cast<T>(reg.lo), static_cast<T>(reg.hi), N);
    return launch_check("clip_kernel");
  }
  const SsnBox b{reg.lo, reg.hi};
  return ssn_prox<T>(reg, 0.0, pc, x, x, gbox, st, nullptr, nullptr, &b);
}

template <class T>
static nys_status dual_prox(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                            T* Q, T* R, T* tbuf, double* cd, double* gbox, hipStream_t st) {
  const int n1 = reg.n1, n2 = reg.n2;
  const int64_t N = static_cast<int64_t>(n1) * n2;
  const int nch = reg_hessian(reg.kind) ? 3 : 2;
  double lnorm2 = reg.lnorm2 > 0 ? reg.lnorm2 : (reg_hessian(reg.kind) ? 34.0 : 8.0);
  double pinv_norm = 1.0;
  if (pc) {
    if (pc->pinv_norm_cache < 0) {
      double hm[PcMeta::kTotal];
      NYS_CHECK_HIP(hipMemcpyAsync(hm, pc->meta.p, sizeof hm, hipMemcpyDeviceToHost, st));
      NYS_CHECK_HIP(hipStreamSynchronize(st));
      pc->pinv_norm_cache = hm[PcMeta::kPinvNorm];
    }
    pinv_norm = pc->pinv_norm_cache;
  }
  const double step = 1.0 / (lam_bar * lnorm2 * pinv_norm);
  dim3 g2(cdiv(n2, 64), cdiv(n1, 4));
  NYS_CHECK_HIP(hipMemcpyAsync(R, Q, sizeof(T) * nch * N, hipMemcpyDeviceToDevice, st));
  if (reg.box && pc) NYS_TRY(fill_zero<double>(gbox, PcMeta::kMaxEll, st));
  const int L = pc ? static_cast<int>(pc->ell) : 0;
  double tau = 1.0;
  nys_status conv = NYS_OK;   // a box projection that ran out of Newton trials
  for (int it = 0; it <= reg.n_inner; ++it) {
    const bool last = it == reg.n_inner;
    const T* src = last ? Q : R;                 // the output uses Q, not R
    if (!pc) {
      hipLaunchKernelGGL((lt_kernel<T>), g2, dim3(256), 0, st, src, reg.kind, n1, n2, s,
                         static_cast<T>(lam_bar), x);
      NYS_TRY(launch_check("lt_kernel"));
    } else {
      hipLaunchKernelGGL((lt_kernel<T>), g2, dim3(256), 0, st, src, reg.kind, n1, n2,
                         static_cast<const T*>(nullptr), T(0), tbuf);
      NYS_TRY(launch_check("lt_kernel"));
      NYS_TRY(pc_coeffs<T>(pc, true, tbuf, 1, cd, st));
      NYS_TRY(pc_x_from_pinv<T>(pc, s, tbuf, cd, lam_bar, x, st));
    }
    // x(Q) = prox^P_{delta_C}(s - lam_bar P^{-1} L^T Q) for a box C
    if (reg.box) {
      const nys_status bs = project_box<T>(reg, pc, x, gbox, st);
      if (bs == NYS_ENOCONV) conv = bs;
      else NYS_TRY(bs);
    }
    if (last) break;
    double tau_n = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
    double beta = (tau - 1.0) / tau_n;
    hipLaunchKernelGGL((dual_update_kernel<T>), g2, dim3(256), 0, st, x, Q, R, reg.kind, n1, n2,
                       static_cast<T>(step), static_cast<T>(beta));
    NYS_TRY(launch_check("dual_update_kernel"));
    tau = tau_n;
  }
  if (conv != NYS_OK)
    set_error("prox: a P-weighted box projection ran out of semismooth Newton trial points");
  return conv;
}

// The dual iteration of dual_prox with P^{-1} applied inside one fused pass
// per inner iteration (FP32 U, C = R^N).  The duals alternate between the
// caller's Q / the workspace R and the second buffers Q2 / R2; the first
// iteration reads R = Q (the warm start), the last writes the partials of
// L^T Q+ (the output uses Q, not R).  The final Q is left in the caller's Q.
template <class T>
static nys_status dual_prox_fused(const nys_reg_desc& reg, double lam_bar, nys_pc pc,
                                  const T* s, T* x, T* Q, T* R, T* Q2, T* R2, T* tbuf,
                                  double* cd, double* fpart, bool c_kept, hipStream_t st) {
  const int n1 = reg.n1, n2 = reg.n2;
  const int64_t N = static_cast<int64_t>(n1) * n2;
  const int nch = reg_hessian(reg.kind) ? 3 : 2;
  const double lnorm2 = reg.lnorm2 > 0 ? reg.lnorm2 : (reg_hessian(reg.kind) ? 34.0 : 8.0);
  if (pc->pinv_norm_cache < 0) {
    double hm[PcMeta::kTotal];
    NYS_CHECK_HIP(hipMemcpyAsync(hm, pc->meta.p, sizeof hm, hipMemcpyDeviceToHost, st));
    NYS_CHECK_HIP(hipStreamSynchronize(st));
    pc->pinv_norm_cache = hm[PcMeta::kPinvNorm];
  }
  const double step = 1.0 / (lam_bar * lnorm2 * pc->pinv_norm_cache);
  const dim3 g2(cdiv(n2, 64), cdiv(n1, 4));
  // c of the warm start: d . U^T L^T Q (kept in cd by the previous call on
  // the same state: its last iteration forms them for its final Q)
  if (!c_kept) {
    hipLaunchKernelGGL((lt_kernel<T>), g2, dim3(256), 0, st, Q, reg.kind, n1, n2,
                       static_cast<const T*>(nullptr), T(0), tbuf);
    NYS_TRY(launch_check("lt_kernel"));
    NYS_TRY(pc_coeffs<T>(pc, true, tbuf, 1, cd, st));
  }
  FusedArgsT<T> A{};
  A.n1 = n1;
  A.n2 = n2;
  A.reg = reg.kind;
  A.ell = static_cast<int>(pc->ell);
  A.ell_pad = static_cast<int>(pc->ell_pad);
  A.ldu = pc->ldu;
  A.U = pc->U.as<T>();
  A.cd = cd;
  A.s = s;
  A.lam_bar = static_cast<T>(lam_bar);
  A.step = static_cast<T>(step);
  A.part = fpart;
  const CoefPartials cp{fpart, static_cast<int>(fused_tiles(n1, n2, reg.kind)), 1};
  T* qbuf[2] = {Q, Q2};
  T* rbuf[2] = {R, R2};
  const T* qcur = Q;
  const T* rcur = Q;                 // R = Q at the start
  double tau = 1.0;
  for (int it = 0; it < reg.n_inner; ++it) {
    const double tau_n = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
    A.beta = static_cast<T>((tau - 1.0) / tau_n);
    A.Qi = qcur;
    A.Ri = rcur;
    A.Qo = qbuf[(it + 1) & 1];
    A.Ro = rbuf[it & 1];
    A.last = it == reg.n_inner - 1;
    NYS_TRY(fused_launch<T>(A, st));
    NYS_TRY(pc_tail(pc, true, cp, cd, st));
    qcur = A.Qo;
    rcur = A.Ro;
    tau = tau_n;
  }
  if (qcur != Q)
    NYS_CHECK_HIP(hipMemcpyAsync(Q, qcur, sizeof(T) * nch * N, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL((x_from_dual_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, s, Q,
                     reg.kind, n1, n2, pc->U.as<T>(), pc->ldu, cd, static_cast<int>(pc->ell),
                     static_cast<T>(lam_bar), x);
  return launch_check("x_from_dual_kernel");
}

template <class T>
__global__ void soft_kernel(const T* __restrict__ s, T lam, int64_t N, T* __restrict__ x) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T r = s[n];
  T ar = fabs(r);
  x[n] = ar > lam ? (r > 0 ? r - lam : r + lam) : T(0);
}

// [cd, gbox: kMaxEll doubles each | R | Q (when no state) | t | Q', R' (the
//  fused iteration's second buffers) | block partials]
template <class T>
size_t prox_ws_bytes(const nys_reg_desc& reg) {
  const size_t N = static_cast<size_t>(reg.n1) * reg.n2;
  const int nch = reg_hessian(reg.kind) ? 3 : 2;
  size_t b = sizeof(double) * 2 * PcMeta::kMaxEll + sizeof(T) * (static_cast<size_t>(nch) * N * 2 + N);
  b += ws_round(sizeof(T) * static_cast<size_t>(nch) * N * 2) +
       ws_round(sizeof(double) * fused_tiles(reg.n1, reg.n2, reg.kind) * PcMeta::kMaxEll);
  return b + 512;
}

template <class T>
nys_status prox_run(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                    void* state, hipStream_t st, void* work, bool c_kept) {
  const int64_t N = static_cast<int64_t>(reg.n1) * reg.n2;
  if (reg.kind == NYS_REG_L1) {
    if (!pc) {
      hipLaunchKernelGGL((soft_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, s,
                         static_cast<T>(lam_bar), N, x);
      return launch_check("soft_kernel");
    }
    return ssn_prox<T>(reg, lam_bar, pc, s, x, static_cast<double*>(state), st);
  }
  const int nch = reg_hessian(reg.kind) ? 3 : 2;
  // work: the caller's buffer of prox_ws_bytes
  NYS_REQUIRE(work, "prox: no work buffer");
  char* base = static_cast<char*>(work);
  double* cd = reinterpret_cast<double*>(base);
  double* gbox = cd + PcMeta::kMaxEll;
  T* R = reinterpret_cast<T*>(gbox + PcMeta::kMaxEll);
  T* Q = state ? static_cast<T*>(state) : R + static_cast<size_t>(nch) * N;
  T* tbuf = R + static_cast<size_t>(nch) * N * 2;
  if (!state) NYS_TRY(fill_zero<T>(Q, static_cast<size_t>(nch) * N, st));
  const int udt = std::is_same<T, float>::value ? NYS_F32 : NYS_F64;
  if (pc && !reg.box && pc->u_dtype == udt && pc->ell >= 1 && pc->ell_pad <= PcMeta::kMaxEll) {
    char* f = reinterpret_cast<char*>(tbuf + N);
    f = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(f) + 255) / 256 * 256);
    T* Q2 = reinterpret_cast<T*>(f);
    T* R2 = Q2 + static_cast<size_t>(nch) * N;
    double* fpart = reinterpret_cast<double*>(
        f + ws_round(sizeof(T) * static_cast<size_t>(nch) * N * 2));
    return dual_prox_fused<T>(reg, lam_bar, pc, s, x, Q, R, Q2, R2, tbuf, cd, fpart,
                              c_kept && state != nullptr, st);
  }
  return dual_prox<T>(reg, lam_bar, pc, s, x, Q, R, tbuf, cd, gbox, st);
}

template nys_status prox_run<double>(const nys_reg_desc&, double, nys_pc, const double*, double*,
                                     void*, hipStream_t, void*, bool);
template nys_status prox_run<float>(const nys_reg_desc&, double, nys_pc, const float*, float*,
                                    void*, hipStream_t, void*, bool);
template size_t prox_ws_bytes<double>(const nys_reg_desc&);
template size_t prox_ws_bytes<float>(const nys_reg_desc&);
template nys_status fill_zero<double>(double*, size_t, hipStream_t);
template nys_status fill_zero<float>(float*, size_t, hipStream_t);

}  // namespace nys

using namespace nys;

static nys_status check_reg(const nys_reg_desc* reg, nys_pc pc, nys_dtype dt) {
  NYS_REQUIRE(reg, "null regulariser descriptor");
  NYS_REQUIRE(reg->n1 > 0 && reg->n2 > 0, "bad regulariser image size");
  NYS_REQUIRE(reg->kind >= NYS_REG_TV && reg->kind <= NYS_REG_HSINF, "bad regulariser kind");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "prox dtype must be F64 or F32");
  if (pc) {
    NYS_REQUIRE(pc->N == static_cast<int64_t>(reg->n1) * reg->n2, "pc size != image size");
    NYS_REQUIRE(pc->u_dtype == static_cast<int32_t>(dt), "pc u_dtype != prox dtype");
  }
  if (reg->kind != NYS_REG_L1) NYS_REQUIRE(reg->n_inner >= 0, "n_inner must be >= 0");
  NYS_TRY(check_box(*reg));
  return NYS_OK;
}

extern "C" nys_status nys_prox_state_bytes(const nys_reg_desc* reg, nys_pc pc, nys_dtype dt,
                                           size_t* bytes) {
  NYS_TRY(check_reg(reg, pc, dt));
  NYS_REQUIRE(bytes, "null bytes");
  const size_t N = static_cast<size_t>(reg->n1) * reg->n2;
  if (reg->kind == NYS_REG_L1) *bytes = pc ? sizeof(double) * pc->ell : 0;
  else *bytes = dtype_size(dt) * N * (reg_hessian(reg->kind) ? 3 : 2);
  return NYS_OK;
}

// Workspace of prox_weighted: the dual iteration's buffers and, with a
// preconditioner, the scratch of its applications.
template <class T>
static size_t prox_call_ws_bytes(const nys_reg_desc& reg, nys_pc pc) {
  return ws_round(prox_ws_bytes<T>(reg)) + (pc ? pc_ws_bytes(pc, 1) : 0);
}

extern "C" nys_status nys_prox_workspace_size(const nys_reg_desc* reg, nys_pc pc, nys_dtype dt,
                                              size_t* bytes) {
  NYS_TRY(check_reg(reg, pc, dt));
  NYS_REQUIRE(bytes, "null bytes");
  *bytes = dt == NYS_F64 ? prox_call_ws_bytes<double>(*reg, pc) : prox_call_ws_bytes<float>(*reg, pc);
  return NYS_OK;
}

template <class T>
static nys_status prox_call(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                            void* state, void* ws, size_t ws_bytes, hipStream_t st) {
  NYS_TRY(check_workspace(ws, ws_bytes, prox_call_ws_bytes<T>(reg, pc), "prox_weighted"));
  WsBind bind(ws, ws_bytes, nullptr, pc);
  char* work = nullptr;
  NYS_TAKE(&bind.s, char, work, prox_ws_bytes<T>(reg));
  return prox_run<T>(reg, lam_bar, pc, s, x, state, st, work);
}

extern "C" nys_status prox_weighted(const nys_reg_desc* reg, double lambda_bar, nys_pc pc,
                                    nys_dtype dt, const void* s, void* x, void* state, void* ws,
                                    size_t ws_bytes, void* stream) {
  NYS_TRY(check_reg(reg, pc, dt));
  NYS_REQUIRE(s && x && s != x, "prox_weighted: bad s / x");
  NYS_REQUIRE(lambda_bar > 0 && std::isfinite(lambda_bar), "prox_weighted: lambda_bar must be > 0");
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return prox_call<double>(*reg, lambda_bar, pc, static_cast<const double*>(s),
                             static_cast<double*>(x), state, ws, ws_bytes, st);
  return prox_call<float>(*reg, lambda_bar, pc, static_cast<const float*>(s), static_cast<float*>(x),
                          state, ws, ws_bytes, st);
}
