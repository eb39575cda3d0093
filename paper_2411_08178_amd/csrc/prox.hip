// P-weighted proximal maps (definition in Sec. I-D, C = R^N).
//
// TV / TV_ANISO / HS1: accelerated projected gradient on the dual variable Q
// (eqs. (17)-(22)): each inner iteration computes t = L^T R, applies P^{-1},
// forms x = s - lam_bar (P^{-1} t), and updates Q, R with the ball
// projection and momentum.  L1: Thm. 1 with a semismooth Newton method whose
// decisions (accept / backtrack / converge) are taken on the device.

#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace nys {

// ================================================================ stencils
// Regulariser channels: TV (2): d1 = X[i,j]-X[i-1,j] (0 on row 0),
// d2 = X[i,j]-X[i,j-1] (0 on column 0).  HS1 (3): v11, v22, v12 with
// replicate padding, v12 counted twice in the pairing.
template <class T>
__device__ __forceinline__ T ldc(const T* x, int i, int j, int n1, int n2) {
  i = i < 0 ? 0 : (i >= n1 ? n1 - 1 : i);
  j = j < 0 ? 0 : (j >= n2 ? n2 - 1 : j);
  return x[static_cast<size_t>(i) * n2 + j];
}

// Sum of q over {(i, j) : clip(i + di) = ip, clip(j + dj) = jp}.
template <class T>
__device__ __forceinline__ T rep_adj(const T* q, int ip, int jp, int di, int dj, int n1, int n2) {
  int is[2], js[2], ni = 0, nj = 0;
  if (di == 0) { is[ni++] = ip; }
  else if (di < 0) { if (ip + 1 < n1) is[ni++] = ip + 1; if (ip == 0) is[ni++] = 0; }
  else { if (ip >= 1) is[ni++] = ip - 1; if (ip == n1 - 1) is[ni++] = n1 - 1; }
  if (dj == 0) { js[nj++] = jp; }
  else if (dj < 0) { if (jp + 1 < n2) js[nj++] = jp + 1; if (jp == 0) js[nj++] = 0; }
  else { if (jp >= 1) js[nj++] = jp - 1; if (jp == n2 - 1) js[nj++] = n2 - 1; }
  T s = 0;
  for (int a = 0; a < ni; ++a)
    for (int b = 0; b < nj; ++b) s += q[static_cast<size_t>(is[a]) * n2 + js[b]];
  return s;
}

template <class T>
__device__ __forceinline__ T lt_at(const T* q, int reg, int i, int j, int n1, int n2) {
  const size_t N = static_cast<size_t>(n1) * n2;
  const size_t o = static_cast<size_t>(i) * n2 + j;
  if (reg != NYS_REG_HS1) {
    const T* q1 = q;
    const T* q2 = q + N;
    T v = 0;
    if (i >= 1) v += q1[o];
    if (i + 1 < n1) v -= q1[o + n2];
    if (j >= 1) v += q2[o];
    if (j + 1 < n2) v -= q2[o + 1];
    return v;
  }
  const T* q11 = q;
  const T* q22 = q + N;
  const T* q12 = q + 2 * N;
  T v = rep_adj(q11, i, j, -1, 0, n1, n2) - T(2) * q11[o] + rep_adj(q11, i, j, 1, 0, n1, n2);
  v += rep_adj(q22, i, j, 0, -1, n1, n2) - T(2) * q22[o] + rep_adj(q22, i, j, 0, 1, n1, n2);
  v += T(0.5) * (rep_adj(q12, i, j, 1, 1, n1, n2) - rep_adj(q12, i, j, 1, -1, n1, n2) -
                 rep_adj(q12, i, j, -1, 1, n1, n2) + rep_adj(q12, i, j, -1, -1, n1, n2));
  return v;
}

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

// x = s - lam (t + U cd)   (P^{-1} t = t + U (d . U^T t))
template <class T>
__global__ __launch_bounds__(256) void x_from_pinv_kernel(const T* __restrict__ s,
                                                          const T* __restrict__ t,
                                                          const T* __restrict__ U,
                                                          const double* __restrict__ cd,
                                                          int64_t N, int L, T lam,
                                                          T* __restrict__ x) {
  __shared__ T cs[PcMeta::kMaxEll];
  for (int k = threadIdx.x; k < L; k += blockDim.x) cs[k] = static_cast<T>(cd[k]);
  __syncthreads();
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T acc = t[n];
  for (int k = 0; k < L; ++k) acc += U[static_cast<size_t>(k) * N + n] * cs[k];
  x[n] = s[n] - lam * acc;
}

template <class T>
__device__ __forceinline__ void project_group(int reg, T* v) {
  if (reg == NYS_REG_TV) {
    T nrm = sqrt(v[0] * v[0] + v[1] * v[1]);
    if (nrm > T(1)) { v[0] /= nrm; v[1] /= nrm; }
  } else if (reg == NYS_REG_TV_ANISO) {
    v[0] = fmin(T(1), fmax(T(-1), v[0]));
    v[1] = fmin(T(1), fmax(T(-1), v[1]));
  } else {
    // symmetric [[a, b], [b, c]]: clip eigenvalues to [-1, 1]
    T a = v[0], c = v[1], b = v[2];
    T m = T(0.5) * (a + c), h = T(0.5) * (a - c);
    T r = sqrt(h * h + b * b);
    T l1 = m + r, l2 = m - r;
    if (l1 <= T(1) && l2 >= T(-1)) return;
    T u1 = fmin(T(1), fmax(T(-1), l1)), u2 = fmin(T(1), fmax(T(-1), l2));
    T avg = T(0.5) * (u1 + u2);
    if (r > T(0)) {
      T g = (u1 - u2) / (T(2) * r);
      v[0] = avg + g * h;
      v[1] = avg - g * h;
      v[2] = g * b;
    } else {
      v[0] = avg; v[1] = avg; v[2] = 0;
    }
  }
}

// Q+ = Proj(R + step L x); R = Q+ + beta (Q+ - Q); Q = Q+
template <class T>
__global__ __launch_bounds__(256) void dual_update_kernel(const T* __restrict__ x, T* __restrict__ Q,
                                                          T* __restrict__ R, int reg, int n1, int n2,
                                                          T step, T beta) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= n1 || j >= n2) return;
  const size_t N = static_cast<size_t>(n1) * n2;
  const size_t o = static_cast<size_t>(i) * n2 + j;
  T lx[3];
  int nch;
  if (reg != NYS_REG_HS1) {
    T xc = x[o];
    lx[0] = i >= 1 ? xc - x[o - n2] : T(0);
    lx[1] = j >= 1 ? xc - x[o - 1] : T(0);
    nch = 2;
  } else {
    T xc = x[o];
    lx[0] = ldc(x, i - 1, j, n1, n2) - T(2) * xc + ldc(x, i + 1, j, n1, n2);
    lx[1] = ldc(x, i, j - 1, n1, n2) - T(2) * xc + ldc(x, i, j + 1, n1, n2);
    lx[2] = T(0.25) * (ldc(x, i + 1, j + 1, n1, n2) - ldc(x, i + 1, j - 1, n1, n2) -
                       ldc(x, i - 1, j + 1, n1, n2) + ldc(x, i - 1, j - 1, n1, n2));
    nch = 3;
  }
  T v[3], qo[3];
  for (int c = 0; c < nch; ++c) {
    qo[c] = Q[c * N + o];
    v[c] = R[c * N + o] + step * lx[c];
  }
  project_group(reg, v);
  for (int c = 0; c < nch; ++c) {
    Q[c * N + o] = v[c];
    R[c * N + o] = v[c] + beta * (v[c] - qo[c]);
  }
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

template <class T>
static nys_status dual_prox(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                            T* Q, T* R, T* tbuf, double* cd, hipStream_t st) {
  const int n1 = reg.n1, n2 = reg.n2;
  const int64_t N = static_cast<int64_t>(n1) * n2;
  const int nch = reg.kind == NYS_REG_HS1 ? 3 : 2;
  double lnorm2 = reg.lnorm2 > 0 ? reg.lnorm2 : (reg.kind == NYS_REG_HS1 ? 34.0 : 8.0);
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
  const int L = pc ? static_cast<int>(pc->ell) : 0;
  double tau = 1.0;
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
      hipLaunchKernelGGL((x_from_pinv_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, s, tbuf,
                         pc->U.as<T>(), cd, N, L, static_cast<T>(lam_bar), x);
      NYS_TRY(launch_check("x_from_pinv_kernel"));
    }
    if (last) break;
    double tau_n = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
    double beta = (tau - 1.0) / tau_n;
    hipLaunchKernelGGL((dual_update_kernel<T>), g2, dim3(256), 0, st, x, Q, R, reg.kind, n1, n2,
                       static_cast<T>(step), static_cast<T>(beta));
    NYS_TRY(launch_check("dual_update_kernel"));
    tau = tau_n;
  }
  return NYS_OK;
}

// ================================================================ SSN (L1)
// Device state of the Newton iteration (FP64):
struct SsnState {
  static constexpr int kGamma = 0;                       // accepted gamma
  static constexpr int kTry = PcMeta::kMaxEll;           // trial gamma
  static constexpr int kDelta = 2 * PcMeta::kMaxEll;     // Newton direction
  static constexpr int kF = 3 * PcMeta::kMaxEll;         // F at gamma
  static constexpr int kS = 4 * PcMeta::kMaxEll;         // scalars
  static constexpr int kNF = kS + 0, kT = kS + 1, kDone = kS + 2, kHalv = kS + 3,
                       kHave = kS + 4, kNeedGram = kS + 5, kTrials = kS + 6, kSteps = kS + 7;
  static constexpr int kTotal = kS + 16;
};

// r = s - U g_try; x = soft(r); mask = |r| > lam; partial sums of U^T (x - s)
// over a chunk of kSsnChunk entries per block.
constexpr int kSsnChunk = 1024;

template <class T>
__global__ __launch_bounds__(256) void ssn_eval_kernel(const T* __restrict__ U, const T* __restrict__ s,
                                                       const double* __restrict__ state, int64_t N,
                                                       int L, T lam, uint8_t* __restrict__ mask,
                                                       double* __restrict__ part) {
  if (state[SsnState::kDone] != 0.0) return;
  __shared__ T g[PcMeta::kMaxEll];
  __shared__ T dv[kSsnChunk];
  __shared__ double red[4][32];
  for (int k = threadIdx.x; k < L; k += blockDim.x) g[k] = static_cast<T>(state[SsnState::kTry + k]);
  __syncthreads();
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * kSsnChunk;
  for (int e = threadIdx.x; e < kSsnChunk; e += 256) {
    int64_t n = n0 + e;
    T d = 0;
    if (n < N) {
      T r = s[n];
      for (int k = 0; k < L; ++k) r -= U[static_cast<size_t>(k) * N + n] * g[k];
      T ar = fabs(r);
      T xv = ar > lam ? (r > 0 ? r - lam : r + lam) : T(0);
      d = xv - s[n];
      mask[n] = ar > lam ? 1 : 0;
    }
    dv[e] = d;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k0 = 0; k0 < L; k0 += 32) {
    T a[32];
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) a[kk] = 0;
    for (int e = threadIdx.x; e < kSsnChunk; e += 256) {
      int64_t n = n0 + e;
      if (n >= N) break;
      T d = dv[e];
#pragma unroll
      for (int kk = 0; kk < 32; ++kk)
        if (k0 + kk < L) a[kk] += U[static_cast<size_t>(k0 + kk) * N + n] * d;
    }
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
      double v = static_cast<double>(a[kk]);
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wv][kk] = v;
    }
    __syncthreads();
    if (threadIdx.x < 32 && k0 + threadIdx.x < L)
      part[static_cast<size_t>(blockIdx.x) * L + k0 + threadIdx.x] =
          red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    __syncthreads();
  }
}

// Reduce the partials to F(g_try) = g_try - e . U^T(x - s), then accept or
// backtrack; on acceptance test convergence.
__global__ void ssn_decide_kernel(const double* __restrict__ part, int nchunks, int L,
                                  const double* __restrict__ meta, double* __restrict__ state,
                                  double tol, int max_halvings) {
  if (state[SsnState::kDone] != 0.0) return;
  __shared__ double Ft[PcMeta::kMaxEll];
  __shared__ double red[128];
  const int tid = threadIdx.x;
  double sq = 0;
  for (int k = tid; k < L; k += blockDim.x) {
    double u = 0;
    for (int c = 0; c < nchunks; ++c) u += part[static_cast<size_t>(c) * L + k];
    double f = state[SsnState::kTry + k] - meta[PcMeta::kE + k] * u;
    Ft[k] = f;
    sq += f * f;
  }
  red[tid] = sq;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double nFt = sqrt(red[0]);
  __syncthreads();
  if (tid == 0) {
    state[SsnState::kTrials] += 1.0;
    const bool have = state[SsnState::kHave] != 0.0;
    const double nF = state[SsnState::kNF], t = state[SsnState::kT];
    bool accept = !have || nFt <= (1.0 - 1e-4 * t) * nF || state[SsnState::kHalv] >= max_halvings ||
                  !isfinite(nFt);
    state[SsnState::kNeedGram] = 0.0;
    if (accept) {
      state[SsnState::kHave] = 1.0;
      state[SsnState::kNF] = nFt;
      double gn = 0;
      for (int k = 0; k < L; ++k) gn += state[SsnState::kTry + k] * state[SsnState::kTry + k];
      if (nFt <= tol * (1.0 + sqrt(gn)) || !isfinite(nFt)) state[SsnState::kDone] = 1.0;
      else state[SsnState::kNeedGram] = 1.0;
    } else {
      double tn = 0.5 * t;
      state[SsnState::kT] = tn;
      state[SsnState::kHalv] += 1.0;
      for (int k = 0; k < L; ++k)
        state[SsnState::kTry + k] = state[SsnState::kGamma + k] + tn * state[SsnState::kDelta + k];
    }
  }
  __syncthreads();
  const bool accepted_now = state[SsnState::kNeedGram] != 0.0 ||
                            (state[SsnState::kDone] != 0.0);
  if (accepted_now)
    for (int k = tid; k < L; k += blockDim.x) {
      state[SsnState::kGamma + k] = state[SsnState::kTry + k];
      state[SsnState::kF + k] = Ft[k];
    }
}

// Masked Gram partials: sum over active n (mask set by the evaluation of the
// accepted point) of U[:,n] U[:,n]^T; one 64 x 64 output tile per block.
template <class T>
__global__ __launch_bounds__(256) void ssn_gram_kernel(const T* __restrict__ U,
                                                       const uint8_t* __restrict__ mask,
                                                       const double* __restrict__ state, int64_t N,
                                                       int L, double* __restrict__ part) {
  if (state[SsnState::kDone] != 0.0 || state[SsnState::kNeedGram] == 0.0) return;
  const int ti = blockIdx.y, tj = blockIdx.z;
  if (tj < ti) return;
  __shared__ T As[32][65];
  __shared__ T Bs[32][65];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * kSsnChunk;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int64_t nb = n0; nb < n0 + kSsnChunk && nb < N; nb += 32) {
    for (int e = threadIdx.x; e < 32 * 64; e += 256) {
      int c = e / 32, kk = e - c * 32;
      int64_t n = nb + kk;
      int ka = ti * 64 + c, kb = tj * 64 + c;
      bool on = n < N && mask[n];
      As[kk][c] = (on && ka < L) ? U[static_cast<size_t>(ka) * N + n] : T(0);
      Bs[kk][c] = (on && kb < L) ? U[static_cast<size_t>(kb) * N + n] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 32; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty * 4 + q];
        b[q] = Bs[kk][tx * 4 + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
  const size_t LL = static_cast<size_t>(L) * L;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int ia = ti * 64 + ty * 4 + p, ib = tj * 64 + tx * 4 + q;
      if (ia < L && ib < L) {
        part[blockIdx.x * LL + static_cast<size_t>(ia) * L + ib] = static_cast<double>(acc[p][q]);
        part[blockIdx.x * LL + static_cast<size_t>(ib) * L + ia] = static_cast<double>(acc[p][q]);
      }
    }
}

__global__ void ssn_gram_reduce_kernel(const double* __restrict__ part, int nchunks, int L,
                                       const double* __restrict__ state, double* __restrict__ M) {
  if (state[SsnState::kDone] != 0.0 || state[SsnState::kNeedGram] == 0.0) return;
  const size_t LL = static_cast<size_t>(L) * L;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < LL;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += part[c * LL + e];
    M[e] = s;
  }
}

// Newton direction: (I + diag(e) M) delta = -F by Gaussian elimination with
// partial pivoting (one workgroup, FP64); then g_try = gamma + delta.
__global__ __launch_bounds__(256) void ssn_solve_kernel(double* __restrict__ M, int L,
                                                        const double* __restrict__ meta,
                                                        double* __restrict__ state) {
  if (state[SsnState::kDone] != 0.0 || state[SsnState::kNeedGram] == 0.0) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int W = L + 1;   // augmented matrix in M's buffer would alias; use LDS rows
  __shared__ int piv;
  // build J in place: J = I + diag(e) M, augmented column b = -F in a separate array
  extern __shared__ double rhs_s[];
  for (size_t e = tid; e < static_cast<size_t>(L) * L; e += nt) {
    int i = static_cast<int>(e / L), j = static_cast<int>(e % L);
    M[e] = (i == j ? 1.0 : 0.0) + meta[PcMeta::kE + i] * M[e];
  }
  for (int i = tid; i < L; i += nt) rhs_s[i] = -state[SsnState::kF + i];
  __syncthreads();
  (void)W;
  for (int col = 0; col < L; ++col) {
    if (tid == 0) {
      int p = col;
      double best = fabs(M[col * L + col]);
      for (int r = col + 1; r < L; ++r) {
        double v = fabs(M[r * L + col]);
        if (v > best) { best = v; p = r; }
      }
      piv = p;
    }
    __syncthreads();
    const int p = piv;
    if (p != col) {
      for (int j = tid; j < L; j += nt) {
        double t = M[col * L + j]; M[col * L + j] = M[p * L + j]; M[p * L + j] = t;
      }
      if (tid == 0) { double t = rhs_s[col]; rhs_s[col] = rhs_s[p]; rhs_s[p] = t; }
    }
    __syncthreads();
    const double d = M[col * L + col];
    for (int r = col + 1 + tid; r < L; r += nt) {
      double f = M[r * L + col] / d;
      if (f != 0.0) {
        for (int j = col; j < L; ++j) M[r * L + j] -= f * M[col * L + j];
        rhs_s[r] -= f * rhs_s[col];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int i = L - 1; i >= 0; --i) {
      double s = rhs_s[i];
      for (int j = i + 1; j < L; ++j) s -= M[i * L + j] * rhs_s[j];
      rhs_s[i] = s / M[i * L + i];
    }
    state[SsnState::kT] = 1.0;
    state[SsnState::kHalv] = 0.0;
    state[SsnState::kSteps] += 1.0;
  }
  __syncthreads();
  for (int k = tid; k < L; k += nt) {
    state[SsnState::kDelta + k] = rhs_s[k];
    state[SsnState::kTry + k] = state[SsnState::kGamma + k] + rhs_s[k];
  }
}

// x = soft(s - U gamma)
template <class T>
__global__ __launch_bounds__(256) void ssn_final_kernel(const T* __restrict__ U, const T* __restrict__ s,
                                                        const double* __restrict__ state, int64_t N,
                                                        int L, T lam, T* __restrict__ x) {
  __shared__ T g[PcMeta::kMaxEll];
  for (int k = threadIdx.x; k < L; k += blockDim.x) g[k] = static_cast<T>(state[SsnState::kGamma + k]);
  __syncthreads();
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T r = s[n];
  for (int k = 0; k < L; ++k) r -= U[static_cast<size_t>(k) * N + n] * g[k];
  T ar = fabs(r);
  x[n] = ar > lam ? (r > 0 ? r - lam : r + lam) : T(0);
}

template <class T>
__global__ void soft_kernel(const T* __restrict__ s, T lam, int64_t N, T* __restrict__ x) {
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T r = s[n];
  T ar = fabs(r);
  x[n] = ar > lam ? (r > 0 ? r - lam : r + lam) : T(0);
}

// Initialise the Newton state from the warm start gamma (g_try = gamma).
__global__ void ssn_init_kernel(double* __restrict__ state, const double* __restrict__ gamma0, int L) {
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    double g = gamma0 ? gamma0[k] : 0.0;
    state[SsnState::kGamma + k] = g;
    state[SsnState::kTry + k] = g;
    state[SsnState::kDelta + k] = 0.0;
  }
  if (threadIdx.x == 0) {
    state[SsnState::kNF] = 0; state[SsnState::kT] = 1; state[SsnState::kDone] = 0;
    state[SsnState::kHalv] = 0; state[SsnState::kHave] = 0; state[SsnState::kNeedGram] = 0;
    state[SsnState::kTrials] = 0; state[SsnState::kSteps] = 0;
  }
}

__global__ void ssn_store_gamma_kernel(const double* __restrict__ state, double* __restrict__ gamma, int L) {
  for (int k = threadIdx.x; k < L; k += blockDim.x) gamma[k] = state[SsnState::kGamma + k];
}

template <class T>
static nys_status ssn_prox(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                           double* gamma_state, hipStream_t st) {
  const int64_t N = pc->N;
  const int L = static_cast<int>(pc->ell);
  const int nchunks = static_cast<int>(cdiv(N, kSsnChunk));
  const size_t LL = static_cast<size_t>(L) * L;
  size_t need = SsnState::kTotal + static_cast<size_t>(nchunks) * L + nchunks * LL + LL;
  NYS_TRY(pc->work2.ensure(sizeof(double) * need + N + 256));
  double* state = pc->work2.as<double>();
  double* part = state + SsnState::kTotal;
  double* gpart = part + static_cast<size_t>(nchunks) * L;
  double* M = gpart + nchunks * LL;
  uint8_t* mask = reinterpret_cast<uint8_t*>(M + LL);
  const T lam = static_cast<T>(lam_bar);
  const double tol = reg.newton_tol > 0 ? reg.newton_tol : (sizeof(T) == 8 ? 1e-12 : 1e-6);
  const int max_trials = reg.max_newton > 0 ? reg.max_newton : 60;
  hipLaunchKernelGGL(ssn_init_kernel, dim3(1), dim3(128), 0, st, state, gamma_state, L);
  NYS_TRY(launch_check("ssn_init_kernel"));
  const T* U = pc->U.as<T>();
  const double* meta = pc->meta.as<double>();
  const int ntile = static_cast<int>(cdiv(L, 64));
  for (int trial = 0; trial < max_trials; ++trial) {
    hipLaunchKernelGGL((ssn_eval_kernel<T>), dim3(nchunks), dim3(256), 0, st, U, s, state, N, L,
                       lam, mask, part);
    NYS_TRY(launch_check("ssn_eval_kernel"));
    hipLaunchKernelGGL(ssn_decide_kernel, dim3(1), dim3(128), 0, st, part, nchunks, L, meta,
                       state, tol, 30);
    NYS_TRY(launch_check("ssn_decide_kernel"));
    hipLaunchKernelGGL((ssn_gram_kernel<T>), dim3(nchunks, ntile, ntile), dim3(256), 0, st, U,
                       mask, state, N, L, gpart);
    NYS_TRY(launch_check("ssn_gram_kernel"));
    hipLaunchKernelGGL(ssn_gram_reduce_kernel, dim3(cdiv(LL, 256)), dim3(256), 0, st, gpart,
                       nchunks, L, state, M);
    NYS_TRY(launch_check("ssn_gram_reduce_kernel"));
    hipLaunchKernelGGL(ssn_solve_kernel, dim3(1), dim3(256), sizeof(double) * L, st, M, L, meta,
                       state);
    NYS_TRY(launch_check("ssn_solve_kernel"));
    // read the done flag every other trial so a converged solve stops early
    if ((trial & 1) == 1) {
      double done = 0;
      NYS_CHECK_HIP(hipMemcpyAsync(&done, state + SsnState::kDone, sizeof(double),
                                   hipMemcpyDeviceToHost, st));
      NYS_CHECK_HIP(hipStreamSynchronize(st));
      if (done != 0.0) break;
    }
  }
  hipLaunchKernelGGL((ssn_final_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, U, s, state, N,
                     L, lam, x);
  NYS_TRY(launch_check("ssn_final_kernel"));
  if (gamma_state) {
    hipLaunchKernelGGL(ssn_store_gamma_kernel, dim3(1), dim3(128), 0, st, state, gamma_state, L);
    NYS_TRY(launch_check("ssn_store_gamma_kernel"));
  }
  return NYS_OK;
}

template <class T>
nys_status prox_run(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                    void* state, hipStream_t st, double* scratch_dev) {
  const int64_t N = static_cast<int64_t>(reg.n1) * reg.n2;
  if (reg.kind == NYS_REG_L1) {
    if (!pc) {
      hipLaunchKernelGGL((soft_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, s,
                         static_cast<T>(lam_bar), N, x);
      return launch_check("soft_kernel");
    }
    return ssn_prox<T>(reg, lam_bar, pc, s, x, static_cast<double*>(state), st);
  }
  const int nch = reg.kind == NYS_REG_HS1 ? 3 : 2;
  // work: Q (if no state), R, t, cd
  static thread_local DevBuf fallback;
  nys_status r = NYS_OK;
  DevBuf& buf = fallback;
  // layout: [cd: kMaxEll doubles | R | Q (when no state) | t]
  size_t need = sizeof(double) * PcMeta::kMaxEll +
                sizeof(T) * (static_cast<size_t>(nch) * N * (state ? 1 : 2) + N);
  NYS_TRY(buf.ensure(need));
  double* cd = buf.as<double>();
  T* base = reinterpret_cast<T*>(cd + PcMeta::kMaxEll);
  T* Q = state ? static_cast<T*>(state) : base + static_cast<size_t>(nch) * N;
  T* R = base;
  T* tbuf = base + static_cast<size_t>(nch) * N * (state ? 1 : 2);
  if (!state) NYS_TRY(fill_zero<T>(Q, static_cast<size_t>(nch) * N, st));
  r = dual_prox<T>(reg, lam_bar, pc, s, x, Q, R, tbuf, cd, st);
  return r;
}

template nys_status prox_run<double>(const nys_reg_desc&, double, nys_pc, const double*, double*,
                                     void*, hipStream_t, double*);
template nys_status prox_run<float>(const nys_reg_desc&, double, nys_pc, const float*, float*,
                                    void*, hipStream_t, double*);
template nys_status fill_zero<double>(double*, size_t, hipStream_t);
template nys_status fill_zero<float>(float*, size_t, hipStream_t);

}  // namespace nys

using namespace nys;

static nys_status check_reg(const nys_reg_desc* reg, nys_pc pc, nys_dtype dt) {
  NYS_REQUIRE(reg, "null regulariser descriptor");
  NYS_REQUIRE(reg->n1 > 0 && reg->n2 > 0, "bad regulariser image size");
  NYS_REQUIRE(reg->kind >= NYS_REG_TV && reg->kind <= NYS_REG_L1, "bad regulariser kind");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "prox dtype must be F64 or F32");
  if (pc) {
    NYS_REQUIRE(pc->N == static_cast<int64_t>(reg->n1) * reg->n2, "pc size != image size");
    NYS_REQUIRE(pc->u_dtype == static_cast<int32_t>(dt), "pc u_dtype != prox dtype");
  }
  if (reg->kind != NYS_REG_L1) NYS_REQUIRE(reg->n_inner >= 0, "n_inner must be >= 0");
  return NYS_OK;
}

extern "C" nys_status nys_prox_state_bytes(const nys_reg_desc* reg, nys_pc pc, nys_dtype dt,
                                           size_t* bytes) {
  NYS_TRY(check_reg(reg, pc, dt));
  NYS_REQUIRE(bytes, "null bytes");
  const size_t N = static_cast<size_t>(reg->n1) * reg->n2;
  if (reg->kind == NYS_REG_L1) *bytes = pc ? sizeof(double) * pc->ell : 0;
  else *bytes = dtype_size(dt) * N * (reg->kind == NYS_REG_HS1 ? 3 : 2);
  return NYS_OK;
}

extern "C" nys_status prox_weighted(const nys_reg_desc* reg, double lambda_bar, nys_pc pc,
                                    nys_dtype dt, const void* s, void* x, void* state,
                                    void* stream) {
  NYS_TRY(check_reg(reg, pc, dt));
  NYS_REQUIRE(s && x && s != x, "prox_weighted: bad s / x");
  NYS_REQUIRE(lambda_bar > 0 && std::isfinite(lambda_bar), "prox_weighted: lambda_bar must be > 0");
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return prox_run<double>(*reg, lambda_bar, pc, static_cast<const double*>(s), static_cast<double*>(x),
                            state, st);
  return prox_run<float>(*reg, lambda_bar, pc, static_cast<const float*>(s), static_cast<float*>(x),
                         state, st);
}
