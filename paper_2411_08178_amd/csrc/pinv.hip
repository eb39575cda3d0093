// Applications of the Nystrom preconditioner (eq. (11)) and the P-weighted l1
// prox of Thm. 1, the two places where the tall U (N x ell) is streamed.
//
// U is stored column by column with a padded pitch (pc->ldu >= N elements),
// so its ell columns do not sit a power of two apart in memory.
//
// Reductions U^T w: every thread accumulates its pixels for all ell entries,
// a butterfly reduce-scatter across the 64 lanes leaves entry k on lane k,
// the waves of a block are summed in FP64 into one partial per block, and a
// one-block tail kernel adds the partials in a fixed order and finishes the
// step.  Results are therefore bitwise reproducible.

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <chrono>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "batch.hpp"

namespace nys {

// ---------------------------------------------------------------- helpers
// Butterfly reduce-scatter over the 64 lanes of acc[NV] (NV in 16..128).  On
// return lane l holds, in acc[j] for j < max(NV / 64, 1), the wave sum of
// entry k = j + max(NV / 64, 1) * l (NV >= 64), or of entry k = l % NV
// (NV < 64).
template <int CNT, int O, int NV, class A>
__device__ __forceinline__ void butterfly_level(A (&acc)[NV], int lane) {
  if constexpr (O >= 1 && CNT >= 2) {
    constexpr int half = CNT / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      A send = up ? acc[j] : acc[j + half];
      A keep = up ? acc[j + half] : acc[j];
      acc[j] = keep + __shfl_xor(send, O, 64);
    }
    butterfly_level<half, O / 2, NV>(acc, lane);
  }
}

template <int NV, class A>
__device__ __forceinline__ void butterfly_reduce(A (&acc)[NV], int lane) {
  // fold the lane bits that NV does not need (NV < 64)
#pragma unroll
  for (int o = 32; o >= NV && o >= 1; o >>= 1)
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] += __shfl_xor(acc[j], o, 64);
  butterfly_level<NV, (NV >= 64 ? 32 : NV / 2), NV>(acc, lane);
}

// Map of the reduce-scatter: entry held by (lane, j).
template <int NV>
__device__ __forceinline__ int butterfly_entry(int lane, int j) {
  return NV >= 64 ? j + (NV / 64) * lane : (lane % NV);
}

// Sum a block's per-thread acc[NV] into out (FP64, NV entries); all threads
// must call it.  red must hold (blockDim.x / 64) * NV doubles.
template <int NV, class A>
__device__ __forceinline__ void block_reduce(A (&acc)[NV], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  butterfly_reduce<NV>(acc, lane);
  constexpr int PER = NV >= 64 ? NV / 64 : 1;
  if (NV >= 64 || lane < NV) {
#pragma unroll
    for (int j = 0; j < PER; ++j) red[wave * NV + butterfly_entry<NV>(lane, j)] = static_cast<double>(acc[j]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += blockDim.x) {
    double sacc = 0;
    for (int w = 0; w < nw; ++w) sacc += red[w * NV + k];
    out[k] = sacc;
  }
  __syncthreads();
}

// out[k] = sum_{b < nblk} part[b * L + k] for k < L (L <= 128), with all
// threads of the block: blockDim / L slices of the blocks, 32 loads in flight
// and eight accumulators each, combined in a fixed order.  red: blockDim.x
// doubles of LDS.
__device__ __forceinline__ void tail_sum(const double* __restrict__ part, int nblk, int L,
                                         double* red, double* out) {
  const int S = blockDim.x / L;
  const int k = threadIdx.x % L, sl = threadIdx.x / L;
  if (sl < S) {
    // 32 loads in flight per round, added into 8 accumulators
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int b = sl;
    for (; b + 31 * S < nblk; b += 32 * S) {
      double v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) v[i] = part[static_cast<size_t>(b + i * S) * L + k];
#pragma unroll
      for (int i = 0; i < 32; ++i) a[i & 7] += v[i];
    }
    for (; b < nblk; b += S) a[0] += part[static_cast<size_t>(b) * L + k];
    red[sl * L + k] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  __syncthreads();
  for (int kk = threadIdx.x; kk < L; kk += blockDim.x) {
    double sacc = 0;
    for (int q = 0; q < S; ++q) sacc += red[q * L + kk];
    out[kk] = sacc;
  }
  __syncthreads();
}

// ================================================================ U^T v
// Block (b, col): pixels of chunk b, all rows of U in groups of 16 (rows past
// ell are zero padding): part[col][b][k] = sum over the chunk of U[k][n] v[n].
template <class T>
__device__ __forceinline__ void ut_partial_body(const T* __restrict__ U, int64_t ldu,
                                                const T* __restrict__ vc, int64_t N, int Lp,
                                                int64_t n0, int64_t n1, double* __restrict__ dst) {
  __shared__ double red[1024];
  __shared__ double bsum[16];
  const int bs = blockDim.x;
  constexpr int VW = 16 / sizeof(T);       // elements per 16-byte load
  for (int g = 0; g < Lp / 16; ++g) {
    T acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0;
    if ((N % VW) == 0) {
      // 16-byte loads: VW consecutive pixels per thread (chunk is a multiple of 64)
      for (int64_t n = n0 + VW * threadIdx.x; n < n1; n += VW * bs) {
        T x[VW];
        __builtin_memcpy(x, vc + n, 16);
        const T* p = U + static_cast<size_t>(16 * g) * ldu + n;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          T u[VW];
          __builtin_memcpy(u, p, 16);
#pragma unroll
          for (int i = 0; i < VW; ++i) acc[k] += u[i] * x[i];
          p += ldu;
        }
      }
    } else {
      for (int64_t n = n0 + threadIdx.x; n < n1; n += bs) {
        const T x = vc[n];
        const T* p = U + static_cast<size_t>(16 * g) * ldu + n;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          acc[k] += p[0] * x;
          p += ldu;
        }
      }
    }
    block_reduce<16>(acc, red, bsum);
    if (threadIdx.x < 16) dst[16 * g + threadIdx.x] = bsum[threadIdx.x];
  }
}

template <class T>
__global__ __launch_bounds__(1024) void ut_partial_kernel(const T* __restrict__ U, int64_t ldu,
                                                          const T* __restrict__ v, int64_t N,
                                                          int Lp, int64_t chunk,
                                                          double* __restrict__ part) {
  const int nblk = gridDim.x, col = blockIdx.y;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  ut_partial_body<T>(U, ldu, v + static_cast<size_t>(col) * N, N, Lp, n0, n1,
                     part + (static_cast<size_t>(col) * nblk + blockIdx.x) * Lp);
}

// ---------------------------------------------------------------- batched
// U^T v over one pixel chunk with all NV = 16, 32 or 64 rows of U held in
// registers: every thread streams 16-byte runs of v and of each U row, and
// the block reduces once at the end.  red: (blockDim / 64) * 64 doubles.
template <int NV>
__device__ __forceinline__ void ut_rows_body(const float* __restrict__ U, int64_t ldu,
                                             const float* __restrict__ v, int64_t n0, int64_t n1,
                                             double* red, double* bsum,
                                             double* __restrict__ dst) {
  float acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.f;
  for (int64_t n = n0 + 4 * threadIdx.x; n < n1; n += 4 * blockDim.x) {
    const float4 x = *reinterpret_cast<const float4*>(v + n);
    const float* p = U + n;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const float4 u = *reinterpret_cast<const float4*>(p + k * ldu);
      acc[k] = fmaf(u.x, x.x, fmaf(u.y, x.y, fmaf(u.z, x.z, fmaf(u.w, x.w, acc[k]))));
    }
  }
  block_reduce<NV>(acc, red, bsum);
  for (int k = threadIdx.x; k < NV; k += blockDim.x) dst[k] = bsum[k];
}

// Rows [0, Lp) of U (Lp a multiple of 16) in pieces of 64, 32 and 16 rows,
// each a pass over the chunk with all its rows in registers.
__device__ __forceinline__ void ut_rows_any(const float* __restrict__ U, int64_t ldu,
                                            const float* __restrict__ v, int Lp, int64_t n0,
                                            int64_t n1, double* red, double* bsum,
                                            double* __restrict__ dst) {
  int k0 = 0;
  for (; k0 + 64 <= Lp; k0 += 64) {
    ut_rows_body<64>(U + k0 * ldu, ldu, v, n0, n1, red, bsum, dst + k0);
    __syncthreads();
  }
  if (k0 + 32 <= Lp) {
    ut_rows_body<32>(U + k0 * ldu, ldu, v, n0, n1, red, bsum, dst + k0);
    __syncthreads();
    k0 += 32;
  }
  if (k0 + 16 <= Lp) ut_rows_body<16>(U + k0 * ldu, ldu, v, n0, n1, red, bsum, dst + k0);
}

// Single preconditioner, FP32 U, N % 4 == 0: block (chunk, column), all
// rows; or, with gridDim.z > 1 (short vectors, too few chunks to fill the
// chip), block (chunk, column, group of 16 rows).
__global__ __launch_bounds__(256) void ut_rows_kernel(const float* __restrict__ U, int64_t ldu,
                                                      const float* __restrict__ v, int64_t N,
                                                      int Lp, int64_t chunk,
                                                      double* __restrict__ part) {
  __shared__ double red[4 * 64];
  __shared__ double bsum[64];
  const int nblk = gridDim.x, col = blockIdx.y;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  double* dst = part + (static_cast<size_t>(col) * nblk + blockIdx.x) * Lp;
  if (gridDim.z > 1) {
    const int k0 = 16 * blockIdx.z;
    ut_rows_body<16>(U + k0 * ldu, ldu, v + static_cast<size_t>(col) * N, n0, n1, red, bsum,
                     dst + k0);
    return;
  }
  ut_rows_any(U, ldu, v + static_cast<size_t>(col) * N, Lp, n0, n1, red, bsum, dst);
}

// Block (256 threads) -> (instance, chunk): D.part[b][k] = sum U[k][n] v[n].
// Batched instances have ell_pad in {16, 32, 64} and N % 4 == 0.
__global__ __launch_bounds__(256) void but_partial_kernel(const BDesc* __restrict__ d,
                                                          const BSeg* __restrict__ seg, int nseg,
                                                          int fsrc) {
  __shared__ double red[4 * 64];
  __shared__ double bsum[64];
  const BSeg& sg = seg[seg_find(seg, nseg, blockIdx.x)];
  const BDesc& D = d[sg.inst];
  const int64_t lb = blockIdx.x - sg.first;
  const int64_t n0 = lb * sg.chunk;
  const int64_t n1 = (n0 + sg.chunk < D.N) ? n0 + sg.chunk : D.N;
  double* dst = D.part + static_cast<size_t>(lb) * D.ell_pad;
  const float* v = D.f[fsrc];
  switch (D.ell_pad) {
    case 16: ut_rows_body<16>(D.U, D.ldu, v, n0, n1, red, bsum, dst); break;
    case 32: ut_rows_body<32>(D.U, D.ldu, v, n0, n1, red, bsum, dst); break;
    default: ut_rows_body<64>(D.U, D.ldu, v, n0, n1, red, bsum, dst); break;
  }
}

// One block per segment: D.cd[k] = d_k * sum_b D.part[b][k]  (d of eq. (11)).
__global__ __launch_bounds__(1024) void but_tail_kernel(const BDesc* __restrict__ d,
                                                        const BSeg* __restrict__ seg) {
  __shared__ double red[1024];
  __shared__ double bsum[128];
  const BSeg& sg = seg[blockIdx.x];
  const BDesc& D = d[sg.inst];
  tail_sum(D.part, static_cast<int>(sg.nblk), D.ell_pad, red, bsum);
  for (int k = threadIdx.x; k < D.ell; k += blockDim.x) D.cd[k] = D.meta[PcMeta::kD + k] * bsum[k];
}

// out = s + c (t + U cd) over the pixel chunk of a block, c = -scal[sidx]
// (sidx >= 0) or 1; s = 0 when fs < 0; no U term without a preconditioner
// (ell = 0).  P^{-1} t = t + U (d . U^T t) (eq. (11)).  N % 4 == 0.
__global__ __launch_bounds__(256) void bcombine_kernel(const BDesc* __restrict__ d,
                                                       const BSeg* __restrict__ seg, int nseg,
                                                       int fs, int ft, int fout, int sidx) {
  __shared__ float cs[PcMeta::kMaxEll];
  const BSeg& sg = seg[seg_find(seg, nseg, blockIdx.x)];
  const BDesc& D = d[sg.inst];
  const int L = D.ell;
  for (int k = threadIdx.x; k < L; k += blockDim.x) cs[k] = static_cast<float>(D.cd[k]);
  __syncthreads();
  const float c = sidx >= 0 ? -static_cast<float>(D.scal[sidx]) : 1.f;
  const float* t = D.f[ft];            // may alias out
  const float* sv = fs >= 0 ? D.f[fs] : nullptr;
  float* out = D.f[fout];
  const float* __restrict__ U = D.U;
  const int64_t ldu = D.ldu;
  const int64_t n0 = (blockIdx.x - sg.first) * sg.chunk;
  const int64_t n1 = (n0 + sg.chunk < D.N) ? n0 + sg.chunk : D.N;
  for (int64_t n = n0 + 4 * threadIdx.x; n < n1; n += 4 * blockDim.x) {
    float4 a = *reinterpret_cast<const float4*>(t + n);
    const float* p = U + n;
    int k = 0;
    for (; k + 4 <= L; k += 4) {
      const float4 u0 = *reinterpret_cast<const float4*>(p);
      const float4 u1 = *reinterpret_cast<const float4*>(p + ldu);
      const float4 u2 = *reinterpret_cast<const float4*>(p + 2 * ldu);
      const float4 u3 = *reinterpret_cast<const float4*>(p + 3 * ldu);
      const float c0 = cs[k], c1 = cs[k + 1], c2 = cs[k + 2], c3 = cs[k + 3];
      a.x += u0.x * c0 + u1.x * c1 + u2.x * c2 + u3.x * c3;
      a.y += u0.y * c0 + u1.y * c1 + u2.y * c2 + u3.y * c3;
      a.z += u0.z * c0 + u1.z * c1 + u2.z * c2 + u3.z * c3;
      a.w += u0.w * c0 + u1.w * c1 + u2.w * c2 + u3.w * c3;
      p += 4 * ldu;
    }
    for (; k < L; ++k) {
      const float4 u = *reinterpret_cast<const float4*>(p);
      a.x += u.x * cs[k]; a.y += u.y * cs[k]; a.z += u.z * cs[k]; a.w += u.w * cs[k];
      p += ldu;
    }
    float4 r = make_float4(c * a.x, c * a.y, c * a.z, c * a.w);
    if (sv) {
      const float4 s4 = *reinterpret_cast<const float4*>(sv + n);
      r.x += s4.x; r.y += s4.y; r.z += s4.z; r.w += s4.w;
    }
    *reinterpret_cast<float4*>(out + n) = r;
  }
}

nys_status batch_pinv_coeffs(const BDesc* d, const BSeg* rseg, int nrseg, int64_t rblk, int fsrc,
                             hipStream_t st) {
  hipLaunchKernelGGL(but_partial_kernel, dim3(static_cast<unsigned>(rblk)), dim3(256), 0, st, d,
                     rseg, nrseg, fsrc);
  NYS_TRY(launch_check("but_partial_kernel"));
  hipLaunchKernelGGL(but_tail_kernel, dim3(nrseg), dim3(1024), 0, st, d, rseg);
  return launch_check("but_tail_kernel");
}

nys_status batch_combine(const BDesc* d, const BSeg* pseg, int npseg, int64_t pblk, int fs,
                         int ft, int fout, int sidx, hipStream_t st) {
  hipLaunchKernelGGL(bcombine_kernel, dim3(static_cast<unsigned>(pblk)), dim3(256), 0, st, d,
                     pseg, npseg, fs, ft, fout, sidx);
  return launch_check("bcombine_kernel");
}

// cd[col][k] = coef[k] * sum_b part[col][b][k], 16 coefficients per
// workgroup (grid: ceil(L / 16) x ncols): 64 groups of 16 lanes read 128-byte
// runs of 16 partials per block row, then an LDS tree sums the groups.  The
// read of the partials (nblk x Lp FP64 per column) is spread over several CUs
// instead of one.
__global__ __launch_bounds__(1024) void ut_tail_cols_kernel(const double* __restrict__ part,
                                                            int nblk, int L, int Lp,
                                                            const double* __restrict__ coef,
                                                            double* __restrict__ cd) {
  __shared__ double red[64][17];
  const int kk = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int k = blockIdx.x * 16 + kk;
  const double* pc = part + static_cast<size_t>(blockIdx.y) * nblk * Lp;
  double s = 0.0;
  if (k < L) {
    // eight loads in flight, added in block order
    int b = grp;
    for (; b + 7 * 64 < nblk; b += 8 * 64) {
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = pc[static_cast<size_t>(b + 64 * i) * Lp + k];
#pragma unroll
      for (int i = 0; i < 8; ++i) s += v[i];
    }
    for (; b < nblk; b += 64) s += pc[static_cast<size_t>(b) * Lp + k];
  }
  // the four groups of a wave by lane exchange, then the 16 waves in order
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) < 16) red[wave][kk] = s;
  __syncthreads();
  if (threadIdx.x < 16 && k < L) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w][kk];
    cd[static_cast<size_t>(blockIdx.y) * L + k] = coef[k] * t;
  }
}

// out = v + U cd   (one column of cd per image)
template <class T>
__global__ __launch_bounds__(256) void u_update_kernel(const T* __restrict__ U, int64_t ldu,
                                                       const T* __restrict__ v,
                                                       const double* __restrict__ cd, int64_t N,
                                                       int L, T* __restrict__ out) {
  __shared__ T cs[PcMeta::kMaxEll];
  const int col = blockIdx.y;
  for (int k = threadIdx.x; k < L; k += blockDim.x) cs[k] = static_cast<T>(cd[static_cast<size_t>(col) * L + k]);
  __syncthreads();
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T acc = v[static_cast<size_t>(col) * N + n];
  for (int k = 0; k < L; ++k) acc += U[static_cast<size_t>(k) * ldu + n] * cs[k];
  out[static_cast<size_t>(col) * N + n] = acc;
}

// x = s - lam (t + U cd)   (P^{-1} t = t + U (d . U^T t))
template <class T>
__global__ __launch_bounds__(256) void x_from_pinv_kernel(const T* __restrict__ s,
                                                          const T* __restrict__ t,
                                                          const T* __restrict__ U, int64_t ldu,
                                                          const double* __restrict__ cd,
                                                          int64_t N, int L, T lam,
                                                          T* __restrict__ x) {
  __shared__ T cs[PcMeta::kMaxEll];
  for (int k = threadIdx.x; k < L; k += blockDim.x) cs[k] = static_cast<T>(cd[k]);
  __syncthreads();
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T acc = t[n];
  for (int k = 0; k < L; ++k) acc += U[static_cast<size_t>(k) * ldu + n] * cs[k];
  x[n] = s[n] - lam * acc;
}

// launch geometry of the streaming reductions over N
static void red_geometry(int64_t N, int& nblk, int64_t& chunk) {
  int64_t nb = std::min<int64_t>(256, std::max<int64_t>(1, (N + 1023) / 1024));
  chunk = (N + nb - 1) / nb;
  chunk = (chunk + 63) / 64 * 64;
  nblk = static_cast<int>((N + chunk - 1) / chunk);
}

template <class T>
nys_status pc_partials_on(nys_pc pc, const T* B, int64_t ldb, int64_t len, const T* v,
                          int64_t ncols, CoefPartials* out, hipStream_t st) {
  const int Lp = static_cast<int>(pc->ell_pad);
  int nblk;
  int64_t chunk;
  red_geometry(len, nblk, chunk);
  // from the bound workspace, left in place for the caller's tail (its scope
  // releases it)
  double* part = nullptr;
  NYS_TAKE(pc->scr, double, part, static_cast<size_t>(ncols) * nblk * Lp);
  out->part = part;
  out->nblk = nblk;
  out->ncols = static_cast<int>(ncols);
  if constexpr (std::is_same<T, float>::value) {
    if ((len & 3) == 0 && (ldb & 3) == 0) {
      // fewer chunks than compute units: a block per group of 16 rows too
      const unsigned groups = nblk * ncols < 256 ? static_cast<unsigned>(Lp / 16) : 1u;
      hipLaunchKernelGGL(ut_rows_kernel, dim3(nblk, static_cast<unsigned>(ncols), groups),
                         dim3(256), 0, st, B, ldb, v, len, Lp, chunk, part);
      return launch_check("ut_rows_kernel");
    }
  }
  hipLaunchKernelGGL((ut_partial_kernel<T>), dim3(nblk, static_cast<unsigned>(ncols)), dim3(1024),
                     0, st, B, ldb, v, len, Lp, chunk, part);
  return launch_check("ut_partial_kernel");
}

nys_status pc_tail(nys_pc pc, bool inverse, const CoefPartials& cp, double* cd, hipStream_t st) {
  const double* coef = pc->meta.as<double>() + (inverse ? PcMeta::kD : PcMeta::kE);
  hipLaunchKernelGGL(ut_tail_cols_kernel, dim3(cdiv(pc->ell, 16), static_cast<unsigned>(cp.ncols)),
                     dim3(1024), 0, st, cp.part, cp.nblk, static_cast<int>(pc->ell),
                     static_cast<int>(pc->ell_pad), coef, cd);
  return launch_check("ut_tail_cols_kernel");
}

template <class T>
nys_status pc_coeffs_on(nys_pc pc, const T* B, int64_t ldb, int64_t len, bool inverse, const T* v,
                        int64_t ncols, double* cd, hipStream_t st) {
  Scratch::Mark mark(pc->scr);   // the partials live until the tail has read them
  CoefPartials cp;
  NYS_TRY(pc_partials_on<T>(pc, B, ldb, len, v, ncols, &cp, st));
  return pc_tail(pc, inverse, cp, cd, st);
}

template <class T>
nys_status pc_coeffs(nys_pc pc, bool inverse, const T* v, int64_t ncols, double* cd,
                     hipStream_t st) {
  return pc_coeffs_on<T>(pc, pc->U.as<T>(), pc->ldu, pc->N, inverse, v, ncols, cd, st);
}

// Workspace of pc_apply on ncols columns: the coefficients and the block
// partials (at most 256 blocks a column).
size_t pc_ws_bytes(nys_pc pc, int64_t ncols) {
  return ws_round(sizeof(double) * static_cast<size_t>(ncols) * pc->ell) +
         ws_round(sizeof(double) * static_cast<size_t>(ncols) * 256 * pc->ell_pad);
}

template <class T>
nys_status pc_apply(nys_pc pc, bool inverse, const T* v, T* out, int64_t ncols, hipStream_t st) {
  const int64_t N = pc->N;
  const int L = static_cast<int>(pc->ell);
  Scratch::Mark mark(pc->scr);
  double* cd = nullptr;
  NYS_TAKE(pc->scr, double, cd, static_cast<size_t>(ncols) * L);
  NYS_TRY(pc_coeffs<T>(pc, inverse, v, ncols, cd, st));
  hipLaunchKernelGGL((u_update_kernel<T>), dim3(cdiv(N, 256), ncols), dim3(256), 0, st,
                     pc->U.as<T>(), pc->ldu, v, cd, N, L, out);
  return launch_check("u_update_kernel");
}

// s = u - alpha P^{-1} g: the coefficients d . U^T g, then one pass
// s = u - alpha (g + U cd).
template <class T>
nys_status pc_step(nys_pc pc, const T* u, const T* g, double alpha, T* s, hipStream_t st) {
  Scratch::Mark mark(pc->scr);
  double* cd = nullptr;
  NYS_TAKE(pc->scr, double, cd, pc->ell);
  NYS_TRY(pc_coeffs<T>(pc, true, g, 1, cd, st));
  return pc_x_from_pinv<T>(pc, u, g, cd, alpha, s, st);
}

template <class T>
nys_status pc_x_from_pinv(nys_pc pc, const T* s, const T* t, const double* cd, double lam, T* x,
                          hipStream_t st) {
  hipLaunchKernelGGL((x_from_pinv_kernel<T>), dim3(cdiv(pc->N, 256)), dim3(256), 0, st, s, t,
                     pc->U.as<T>(), pc->ldu, cd, pc->N, static_cast<int>(pc->ell),
                     static_cast<T>(lam), x);
  return launch_check("x_from_pinv_kernel");
}

template nys_status pc_partials_on<double>(nys_pc, const double*, int64_t, int64_t, const double*,
                                           int64_t, CoefPartials*, hipStream_t);
template nys_status pc_partials_on<float>(nys_pc, const float*, int64_t, int64_t, const float*,
                                          int64_t, CoefPartials*, hipStream_t);
template nys_status pc_coeffs_on<double>(nys_pc, const double*, int64_t, int64_t, bool,
                                         const double*, int64_t, double*, hipStream_t);
template nys_status pc_coeffs_on<float>(nys_pc, const float*, int64_t, int64_t, bool, const float*,
                                        int64_t, double*, hipStream_t);
template nys_status pc_coeffs<double>(nys_pc, bool, const double*, int64_t, double*, hipStream_t);
template nys_status pc_coeffs<float>(nys_pc, bool, const float*, int64_t, double*, hipStream_t);
template nys_status pc_apply<double>(nys_pc, bool, const double*, double*, int64_t, hipStream_t);
template nys_status pc_apply<float>(nys_pc, bool, const float*, float*, int64_t, hipStream_t);
template nys_status pc_step<double>(nys_pc, const double*, const double*, double, double*,
                                    hipStream_t);
template nys_status pc_step<float>(nys_pc, const float*, const float*, double, float*, hipStream_t);
template nys_status pc_x_from_pinv<double>(nys_pc, const double*, const double*, const double*,
                                           double, double*, hipStream_t);
template nys_status pc_x_from_pinv<float>(nys_pc, const float*, const float*, const double*,
                                          double, float*, hipStream_t);

// ================================================================ SSN (l1)
// prox of lam ||.||_1 in the norm of P = I + U diag(e) U^T (Thm. 1):
// gamma solves F(gamma) = gamma - diag(e) U^T (soft_lam(s - U gamma) - s) = 0;
// semismooth Newton with the Jacobian I + diag(e) U^T D U, D = diag(|s - U
// gamma| > lam), and backtracking on ||F||.  The device holds the state and
// takes every decision; the host only polls the `done` flag.
struct SsnState {
  static constexpr int kGamma = 0;                       // accepted gamma
  static constexpr int kTry = PcMeta::kMaxEll;           // trial gamma
  static constexpr int kDelta = 2 * PcMeta::kMaxEll;     // Newton direction
  static constexpr int kF = 3 * PcMeta::kMaxEll;         // F at gamma
  static constexpr int kS = 4 * PcMeta::kMaxEll;         // scalars
  static constexpr int kNF = kS + 0, kT = kS + 1, kDone = kS + 2, kHalv = kS + 3,
                       kHave = kS + 4, kNeedGram = kS + 5, kTrials = kS + 6, kSteps = kS + 7,
                       kLuOk = kS + 8,   // FP32: inverse of the last Newton Jacobian stored
                       kBad = kS + 9;    // a trial point gave a non-finite ||F||
  static constexpr int kTotal = kS + 16;
};

// Sets of partial Gram sums left by stage 2 for the Newton solve to add.
constexpr int kGramSets = 4;
// Row pitch (floats) of the stored Jacobian inverse (64 x 64).
constexpr int kLuPitch = 64;

// The unweighted prox of Thm. 1's h and its derivative pattern: the soft
// threshold at lam (h = lam ||.||_1; D: |r| > lam) or, with box, the clip to
// [lo, hi] (h the indicator of the box C; D: lo < r < hi).
template <class T>
__device__ __forceinline__ T ssn_h_prox(T r, T lam, int box, T lo, T hi) {
  if (box) return fmin(hi, fmax(lo, r));
  return fabs(r) > lam ? (r > T(0) ? r - lam : r + lam) : T(0);
}
template <class T>
__device__ __forceinline__ bool ssn_h_active(T r, T lam, int box, T lo, T hi) {
  return box ? (r > lo && r < hi) : fabs(r) > lam;
}

// Evaluation at the trial point in one pass over U: r = s - U g, x = soft(r)
// (to xo, if given), mask = |r| > lam (if given), partial U^T (x - s) per
// block.
template <class T, int ROWS, int LP = (ROWS <= 16 ? 16 : ROWS <= 32 ? 32 : ROWS <= 64 ? 64 : 128)>
__global__ __launch_bounds__(512) void ssn_eval_kernel(const T* __restrict__ U, int64_t ldu,
                                                       const T* __restrict__ s, int64_t N, int L,
                                                       int64_t chunk, T lam,
                                                       const double* __restrict__ state,
                                                       uint8_t* __restrict__ mask,
                                                       double* __restrict__ part,
                                                       T* __restrict__ xo, int box, T lo, T hi) {
  __shared__ double red[8 * LP];
  __shared__ double bsum[LP];
  __shared__ T g[LP];
  if (state[SsnState::kDone] != 0.0) return;
  for (int k = threadIdx.x; k < LP; k += blockDim.x) g[k] = k < L ? static_cast<T>(state[SsnState::kTry + k]) : T(0);
  __syncthreads();
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  T acc[LP];
#pragma unroll
  for (int k = 0; k < LP; ++k) acc[k] = 0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    T u[LP];
    // (U g)_n first, then one subtraction from s_n: the sum rounds at the
    // scale of U g, not of s (F is tested near the FP32 rounding level)
    T ug = 0;
    const T* p = U + n;
#pragma unroll
    for (int k = 0; k < LP; ++k) {
      if (k < ROWS) {
        u[k] = p[0];
        p += ldu;
      } else {
        u[k] = T(0);
      }
      ug += u[k] * g[k];
    }
    const T r = s[n] - ug;
    const T xv = ssn_h_prox(r, lam, box, lo, hi);
    const T d = xv - s[n];
    if (mask != nullptr) mask[n] = ssn_h_active(r, lam, box, lo, hi) ? 1 : 0;
    if (xo != nullptr) xo[n] = xv;
#pragma unroll
    for (int k = 0; k < LP; ++k) acc[k] += u[k] * d;
  }
  block_reduce<LP>(acc, red, bsum);
  for (int k = threadIdx.x; k < L; k += blockDim.x) part[static_cast<size_t>(blockIdx.x) * L + k] = bsum[k];
}

// The first trial of a call whose prox centre is the preconditioned gradient
// step s = u - alpha (g + U cd), cd = d . U^T g (eq. (11); FP32, ROWS <= 64),
// in one kernel: every block sums the ncb partials of U^T g (pitch ROWS, in a
// fixed order) into alpha cd itself and takes the trial point from the warm
// start gamma0 (zero if null); block 0 initialises the Newton state as
// ssn_init_kernel does; each pixel then forms s_n from the same loads of U as
// (U g)_n, writes it out for the later trials, and contributes to the partial
// U^T (x - s) as in ssn_eval_kernel.
template <int ROWS, int LP = (ROWS <= 16 ? 16 : ROWS <= 32 ? 32 : 64)>
__global__ __launch_bounds__(512) void ssn_eval_step_kernel(
    const float* __restrict__ U, int64_t ldu, const float* __restrict__ u,
    const float* __restrict__ g, float alpha, const double* __restrict__ cpart, int ncb,
    const double* __restrict__ dcoef, const double* __restrict__ gamma0, int keep_lu,
    float* __restrict__ s_out, int64_t N, int L, int64_t chunk, float lam,
    double* __restrict__ state, double* __restrict__ part, float* __restrict__ xo) {
  __shared__ double red[8 * LP];
  __shared__ double bsum[LP];
  __shared__ float gam[LP], w[LP];
  {
    // alpha cd from the partials: 512 / ROWS slices of the blocks, one
    // predicated round of up to 32 loads per thread
    const int S = 512 / ROWS;
    const int k = threadIdx.x % ROWS, sl = threadIdx.x / ROWS;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (sl < S) {
      for (int b = sl; b < ncb; b += 32 * S) {
        double v[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) {
          const int bb = b + i * S;
          v[i] = bb < ncb ? cpart[static_cast<size_t>(bb) * ROWS + k] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 32; ++i) a[i & 7] += v[i];
      }
    }
    const double g0 = (threadIdx.x < L && gamma0 != nullptr) ? gamma0[threadIdx.x] : 0.0;
    const double dk = threadIdx.x < L ? dcoef[threadIdx.x] : 0.0;
    if (sl < S) red[sl * ROWS + k] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    if (threadIdx.x < LP) {
      double cs = 0;
      if (threadIdx.x < L)
        for (int q = 0; q < S; ++q) cs += red[q * ROWS + threadIdx.x];
      w[threadIdx.x] = threadIdx.x < L ? static_cast<float>(alpha * dk * cs) : 0.f;
      gam[threadIdx.x] = threadIdx.x < L ? static_cast<float>(g0) : 0.f;
    }
    if (blockIdx.x == 0) {
      if (threadIdx.x < L) {
        state[SsnState::kGamma + threadIdx.x] = g0;
        state[SsnState::kTry + threadIdx.x] = g0;
        state[SsnState::kDelta + threadIdx.x] = 0.0;
      }
      if (threadIdx.x == 0) {
        state[SsnState::kNF] = 0; state[SsnState::kT] = 1; state[SsnState::kDone] = 0;
        state[SsnState::kHalv] = 0; state[SsnState::kHave] = 0; state[SsnState::kNeedGram] = 0;
        state[SsnState::kTrials] = 0; state[SsnState::kSteps] = 0; state[SsnState::kBad] = 0;
        if (!keep_lu) state[SsnState::kLuOk] = 0;
      }
    }
    __syncthreads();
  }
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  float acc[LP];
#pragma unroll
  for (int k = 0; k < LP; ++k) acc[k] = 0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    float uk[LP];
    float uw = 0.f, ug = 0.f;
    const float* p = U + n;
#pragma unroll
    for (int k = 0; k < LP; ++k) {
      if (k < ROWS) {
        uk[k] = p[0];
        p += ldu;
      } else {
        uk[k] = 0.f;
      }
      uw += uk[k] * w[k];
      ug += uk[k] * gam[k];
    }
    const float sn = (u[n] - alpha * g[n]) - uw;
    const float r = sn - ug;
    const float ar = fabsf(r);
    const float xv = ar > lam ? (r > 0.f ? r - lam : r + lam) : 0.f;
    const float d = xv - sn;
    s_out[n] = sn;
    if (xo != nullptr) xo[n] = xv;
#pragma unroll
    for (int k = 0; k < LP; ++k) acc[k] += uk[k] * d;
  }
  block_reduce<LP>(acc, red, bsum);
  for (int k = threadIdx.x; k < L; k += blockDim.x) part[static_cast<size_t>(blockIdx.x) * L + k] = bsum[k];
}

// The host learns the outcome from one 64-bit word in pinned host memory,
// hflag = 16 seq + 8 non-finite + 4 done + 2 need_gram + lu_ok, written by a
// single system-scope store (no fence: the host reads nothing else the
// kernel wrote), also when an earlier decision had finished.
__device__ __forceinline__ void ssn_publish(unsigned long long* hflag, unsigned long long seq,
                                            double done, double need_gram, double lu_ok,
                                            double bad) {
  if (hflag == nullptr || threadIdx.x != 0) return;
  const unsigned long long w = (seq << 4) | (bad != 0.0 ? 8ull : 0ull) |
                               (done != 0.0 ? 4ull : 0ull) | (need_gram != 0.0 ? 2ull : 0ull) |
                               (lu_ok != 0.0 ? 1ull : 0ull);
  __hip_atomic_store(hflag, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Value of v on lane `lane` (wave-uniform index) through the scalar unit.
__device__ __forceinline__ float readlane_r(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// The decision on one block of 1024 threads.  Every global value it reads is
// requested before the first wait: the block partials (nblk <= 32 blockDim/L
// of them per thread in one round, FP64 sums in a fixed order), the trial
// point, e, gamma and delta on the threads k < L, the scalars on thread 0.
// When the decision ends the iteration and gout is given, the root goes to
// gout (the caller's warm start).  With LM > 0 (L <= LM <= 64) the stored
// inverse of an earlier Jacobian (lu) is requested with the partials, and a
// decision that accepts without converging is followed by the chord step of
// ssn_chord_kernel (16 threads a row) when the inverse is stored.
template <int LM = 0>
__device__ __forceinline__ void ssn_decide_body(const double* __restrict__ part, int nblk, int L,
                                const double* __restrict__ meta, double* __restrict__ state,
                                double tol, int max_halvings, unsigned long long* hflag,
                                unsigned long long seq, double* __restrict__ gout,
                                const float* __restrict__ lu = nullptr) {
  __shared__ double red[1024];
  __shared__ double Ft[PcMeta::kMaxEll];
  __shared__ double wsum[2][2];
  __shared__ int accepted, finished, chord_go;
  __shared__ double tn_s;
  __shared__ float lus[LM > 0 ? LM * (LM + 1) : 1];
  __shared__ double tkl[LM > 0 ? LM : 1];
  const int tid = threadIdx.x;
  const int S = blockDim.x / L;
  const int k = tid % L, sl = tid / L;
  const double done0 = state[SsnState::kDone];
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (sl < S) {
    for (int b = sl; b < nblk; b += 32 * S) {
      double v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const int bb = b + i * S;
        v[i] = bb < nblk ? part[static_cast<size_t>(bb) * L + k] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 32; ++i) a[i & 7] += v[i];
    }
  }
  double tk = 0, ek = 0, gk = 0, dk = 0;
  if (tid < L) {
    tk = state[SsnState::kTry + tid];
    ek = meta[PcMeta::kE + tid];
    gk = state[SsnState::kGamma + tid];
    dk = state[SsnState::kDelta + tid];
  }
  double have = 0, nF = 0, t = 0, halv = 0, trials = 0, luok = 0, steps = 0, bad0 = 0;
  if (tid == 0) {
    bad0 = state[SsnState::kBad];
    have = state[SsnState::kHave];
    nF = state[SsnState::kNF];
    t = state[SsnState::kT];
    halv = state[SsnState::kHalv];
    trials = state[SsnState::kTrials];
    luok = state[SsnState::kLuOk];
    steps = state[SsnState::kSteps];
  }
  if constexpr (LM > 0) {
    // the buffer always exists; its values are used only if stored
    for (int e = tid; e < L * L; e += blockDim.x) {
      const int rr = e / L, cc = e - rr * L;
      lus[rr * (LM + 1) + cc] = lu[rr * kLuPitch + cc];
    }
  }
  if (done0 != 0.0) {
    ssn_publish(hflag, seq, 1.0, 0.0, luok, bad0);
    return;
  }
  if (sl < S) red[sl * L + k] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  // F = g_try - e . U^T (x - s), ||F||^2 and ||g_try||^2 on waves 0 and 1
  const int lane = tid & 63, wave = tid >> 6;
  if (wave < 2) {
    double sq = 0, gq = 0;
    if (tid < L) {
      double bs = 0;
      for (int q = 0; q < S; ++q) bs += red[q * L + tid];
      const double f = tk - ek * bs;
      Ft[tid] = f;
      if constexpr (LM > 0) tkl[tid] = tk;
      sq = f * f;
      gq = tk * tk;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      sq += __shfl_xor(sq, o, 64);
      gq += __shfl_xor(gq, o, 64);
    }
    if (lane == 0) { wsum[wave][0] = sq; wsum[wave][1] = gq; }
  }
  __syncthreads();
  if (tid == 0) {
    const double nFt = sqrt(wsum[0][0] + wsum[1][0]), gn = sqrt(wsum[0][1] + wsum[1][1]);
    state[SsnState::kTrials] = trials + 1.0;
    // a non-finite ||F|| ends the iteration without accepting the point (the
    // warm start keeps its value) and is reported to the host
    const bool bad = !isfinite(nFt) || !isfinite(gn);
    const bool accept = !bad && (have == 0.0 || nFt <= (1.0 - 1e-4 * t) * nF ||
                                 halv >= max_halvings);
    double done = 0.0, need = 0.0;
    if (bad) {
      done = 1.0;
      state[SsnState::kDone] = 1.0;
      state[SsnState::kBad] = 1.0;
    } else if (accept) {
      state[SsnState::kHave] = 1.0;
      state[SsnState::kNF] = nFt;
      if (nFt <= tol * (1.0 + gn)) done = 1.0;
      else need = 1.0;
      state[SsnState::kDone] = done;
    } else {
      tn_s = 0.5 * t;
      state[SsnState::kT] = tn_s;
      state[SsnState::kHalv] = halv + 1.0;
    }
    state[SsnState::kNeedGram] = need;
    accepted = accept ? 1 : 0;
    finished = done != 0.0 ? 1 : 0;
    chord_go = (LM > 0 && need != 0.0 && luok != 0.0) ? 1 : 0;
    if (LM > 0 && chord_go) {
      state[SsnState::kT] = 1.0;
      state[SsnState::kHalv] = 0.0;
      state[SsnState::kSteps] = steps + 1.0;
    }
    ssn_publish(hflag, seq, done, need, luok, bad ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < L) {
    if (accepted) {
      state[SsnState::kGamma + tid] = tk;
      state[SsnState::kF + tid] = Ft[tid];
      if (finished && gout != nullptr) gout[tid] = tk;
    } else {
      state[SsnState::kTry + tid] = gk + tn_s * dk;
    }
  }
  if constexpr (LM > 0) {
    // chord direction -J0^{-1} F at the accepted point
    if (chord_go) {
      const int i = tid >> 4, j0 = 4 * (tid & 15);
      float sacc = 0.f;
      if (i < L) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (j0 + c < L) sacc += lus[i * (LM + 1) + j0 + c] * static_cast<float>(Ft[j0 + c]);
      }
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) sacc += __shfl_xor(sacc, o, 16);
      if (i < L && (tid & 15) == 0) {
        const double dv = -static_cast<double>(sacc);
        state[SsnState::kDelta + i] = dv;
        state[SsnState::kTry + i] = tkl[i] + dv;
      }
    }
  }
}

// F(g_try) = g_try - e . U^T (x - s) from the partials, its norm, and the
// decision: accept (and stop, or ask for a Newton step) or backtrack.
__global__ __launch_bounds__(1024) void ssn_decide_kernel(const double* __restrict__ part, int nblk,
                                                         int L, const double* __restrict__ meta,
                                                         double* __restrict__ state, double tol,
                                                         int max_halvings, unsigned long long* hflag,
                                                         unsigned long long seq, double* gout) {
  ssn_decide_body(part, nblk, L, meta, state, tol, max_halvings, hflag, seq, gout);
}

// The decision followed by the chord step with the stored factors lu, when it
// accepts without converging (L <= LM).
template <int LM>
__global__ __launch_bounds__(1024) void ssn_decide_chord_kernel(
    const double* __restrict__ part, int nblk, int L, const double* __restrict__ meta,
    double* __restrict__ state, double tol, int max_halvings, unsigned long long* hflag,
    unsigned long long seq, double* gout, const float* __restrict__ lu) {
  ssn_decide_body<LM>(part, nblk, L, meta, state, tol, max_halvings, hflag, seq, gout, lu);
}

// ---- masked Gram on the matrix cores
typedef float floatx16_v __attribute__((ext_vector_type(16)));

// One pass over an FP32 U at the point g (Thm. 1; at state offset gsrc: the
// trial point, or the accepted point for a Newton step there): per pixel
// r = s - U g, x = soft_lam(r) (written to xo: the prox itself if g is the
// accepted final point), d = x - s and D = [|r| > lam]; per block the
// partial U^T d (FP64) for F(g) and the partial masked Gram U^T D U for the
// Newton step that follows if g is accepted.
// Every wave owns stages of 64 pixels: lane p loads the 32 NRG values of
// pixel p (one coalesced row segment per load), evaluates r, and puts the
// stage in its own LDS region (row-major), from which the Gram and U^T d
// (lane = row) read it; the loads of the wave's next stage are issued before
// that.  No block barrier until the final reductions.  The Gram runs on the
// BF16 matrix cores with every masked value split as hi + lo (hi = bf16(v),
// lo = bf16(v - hi)): hi hi^T + hi lo^T + lo hi^T in FP32 accumulation, a
// relative error near 2^-16 -- the Gram only shapes the Newton direction; F
// itself is evaluated in FP32 with FP64 sums.  Rows past L and pixels past the
// block's range read clamped, finite values and contribute nothing (g is zero
// past L; d and D are zero outside the range).
template <int NRG> constexpr int evg_waves() { return NRG <= 2 ? 8 : 4; }
constexpr int kEvgPitch = 68;   // floats per LDS row of a stage: 64 pixels + pad
template <int NRG> constexpr size_t evg_lds_bytes() {
  return sizeof(float) * evg_waves<NRG>() * 32 * NRG * kEvgPitch;
}
typedef __bf16 bf16x8_v __attribute__((ext_vector_type(8)));

template <int NRG>
__global__ __launch_bounds__(64 * evg_waves<NRG>()) void ssn_evalgram_kernel(
    const float* __restrict__ U, int64_t ldu, const float* __restrict__ s, int64_t N, int L,
    int64_t chunk, float lam, const double* __restrict__ state, double* __restrict__ part,
    float* __restrict__ gpart, float* __restrict__ xo, int gsrc, int box, float lo, float hi,
    int need_only) {
  constexpr int W = evg_waves<NRG>();
  constexpr int NTRI = NRG * (NRG + 1) / 2;
  constexpr int ROWS = 32 * NRG;
  constexpr int PP = kEvgPitch;
  constexpr int RPL = (ROWS + 63) / 64;       // rows of U^T d per lane
  extern __shared__ __align__(16) float evg_lds[];
  __shared__ __align__(16) float gs[ROWS];
  __shared__ __align__(16) float dw[W][64];
  __shared__ __align__(16) float mw[W][64];
  __shared__ double udw[W][ROWS];
  // skipped once the iteration has converged, and (need_only) unless the
  // last decision asked for a Newton direction
  if (state[SsnState::kDone] != 0.0 || (need_only && state[SsnState::kNeedGram] == 0.0)) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 31, lh = lane >> 5;
  for (int k = tid; k < ROWS; k += 64 * W) gs[k] = k < L ? static_cast<float>(state[gsrc + k]) : 0.f;
  __syncthreads();
  float* ws = evg_lds + wave * ROWS * PP;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  const int nst = n1 > n0 ? static_cast<int>((n1 - n0 + 63) / 64) : 0;
  floatx16_v acc[NTRI];
#pragma unroll
  for (int t = 0; t < NTRI; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  double udacc[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) udacc[i] = 0.0;
  float u[ROWS];
  float sv = 0.f;
  auto load = [&](int t) {
    int64_t pix = n0 + 64 * static_cast<int64_t>(t) + lane;
    pix = pix < N ? pix : N - 1;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
      const int row = k < L ? k : L - 1;
      u[k] = U[static_cast<size_t>(row) * ldu + pix];
    }
    sv = s[pix];
  };
  int t = wave;
  if (t < nst) load(t);
  for (; t < nst; t += W) {
    const int64_t px = n0 + 64 * static_cast<int64_t>(t) + lane;
    const bool in = px < n1;
    float pr = 0.f;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) pr += u[k] * gs[k];
    const float r = sv - pr;
    const float xv = ssn_h_prox(r, lam, box, lo, hi);
    if (in && xo != nullptr) xo[px] = xv;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) ws[k * PP + lane] = u[k];
    dw[wave][lane] = in ? xv - sv : 0.f;
    mw[wave][lane] = (in && ssn_h_active(r, lam, box, lo, hi)) ? 1.f : 0.f;
    if (t + W < nst) load(t + W);
    // masked Gram: 4 steps of 16 pixels; lane l supplies row 32 g + l % 32,
    // pixels 16 kk + 8 (l / 32) + 0..7
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int p0 = 16 * kk + 8 * lh;
      const float4 m0 = *reinterpret_cast<const float4*>(&mw[wave][p0]);
      const float4 m1 = *reinterpret_cast<const float4*>(&mw[wave][p0 + 4]);
      bf16x8_v hi[NRG], lo[NRG];
#pragma unroll
      for (int g = 0; g < NRG; ++g) {
        const float* src = ws + (32 * g + lr) * PP + p0;
        const float4 a0 = *reinterpret_cast<const float4*>(src);
        const float4 a1 = *reinterpret_cast<const float4*>(src + 4);
        const float v[8] = {a0.x * m0.x, a0.y * m0.y, a0.z * m0.z, a0.w * m0.w,
                            a1.x * m1.x, a1.y * m1.y, a1.z * m1.z, a1.w * m1.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const __bf16 h = static_cast<__bf16>(v[i]);
          hi[g][i] = h;
          lo[g][i] = static_cast<__bf16>(v[i] - static_cast<float>(h));
        }
      }
      int tile = 0;
#pragma unroll
      for (int ti = 0; ti < NRG; ++ti)
#pragma unroll
        for (int tj = ti; tj < NRG; ++tj, ++tile) {
          acc[tile] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[ti], hi[tj], acc[tile], 0, 0, 0);
          acc[tile] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[ti], lo[tj], acc[tile], 0, 0, 0);
          acc[tile] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[ti], hi[tj], acc[tile], 0, 0, 0);
        }
    }
    // U^T d, lane = row: 8 pixels in FP32, then added in FP64
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = lane + 64 * i;
      if (row < ROWS) {
        const float* c = ws + row * PP;
#pragma unroll 2
        for (int p = 0; p < 64; p += 8) {
          const float4 c0 = *reinterpret_cast<const float4*>(c + p);
          const float4 c1 = *reinterpret_cast<const float4*>(c + p + 4);
          const float4 d0 = *reinterpret_cast<const float4*>(&dw[wave][p]);
          const float4 d1 = *reinterpret_cast<const float4*>(&dw[wave][p + 4]);
          const float tsum = c0.x * d0.x + c0.y * d0.y + c0.z * d0.z + c0.w * d0.w +
                             c1.x * d1.x + c1.y * d1.y + c1.z * d1.z + c1.w * d1.w;
          udacc[i] += static_cast<double>(tsum);
        }
      }
    }
  }
  // U^T d: waves summed in a fixed order
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = lane + 64 * i;
    if (row < ROWS) udw[wave][row] = udacc[i];
  }
  __syncthreads();
  for (int k = tid; k < L; k += 64 * W) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) a += udw[w][k];
    part[static_cast<size_t>(blockIdx.x) * L + k] = a;
  }
  // Gram: the waves' tiles summed in LDS in a fixed order
  float* sum = evg_lds;     // NTRI * 1024 floats
  for (int w = 0; w < W; ++w) {
    if (wave == w) {
#pragma unroll
      for (int tt = 0; tt < NTRI; ++tt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int idx = tt * 1024 + (8 * (r / 4) + 4 * lh + (r & 3)) * 32 + lr;
          sum[idx] = (w == 0 ? 0.f : sum[idx]) + acc[tt][r];
        }
    }
    __syncthreads();
  }
  float* dst = gpart + static_cast<size_t>(blockIdx.x) * NTRI * 1024;
  for (int e = tid; e < NTRI * 1024; e += 64 * W) dst[e] = sum[e];
}

// The decision (last block, if with_decide) and the Gram stage-2 reduction
// (NTRI * 4 blocks: entries 256 b .. 256 b + 255, the kGramSets sets on the
// thread quarters) in one launch; the reduction runs whether or not the
// decision asks for a Newton step, the Newton solve checks.
template <int NRG>
__global__ __launch_bounds__(1024) void ssn_decide_gram_kernel(
    const double* __restrict__ part, int nblk, int L, const double* __restrict__ meta,
    double* __restrict__ state, double tol, int max_halvings, unsigned long long* hflag,
    unsigned long long seq, double* gout,
    const float* __restrict__ gpart, double* __restrict__ part2, int with_decide,
    int need_only) {
  static_assert(kGramSets == 4, "four sets on the thread quarters of 1024");
  constexpr int NTRI = NRG * (NRG + 1) / 2;
  if (with_decide && blockIdx.x == gridDim.x - 1) {
    ssn_decide_body(part, nblk, L, meta, state, tol, max_halvings, hflag, seq, gout);
    return;
  }
  // a Newton step at the accepted point only: skipped as its Gram pass was
  if (!with_decide && (state[SsnState::kDone] != 0.0 ||
                       (need_only && state[SsnState::kNeedGram] == 0.0)))
    return;
  const int e = blockIdx.x * 256 + (threadIdx.x & 255), q = threadIdx.x >> 8;
  if (e >= NTRI * 1024) return;
  const size_t stride = static_cast<size_t>(NTRI) * 1024;
  double a[4] = {0, 0, 0, 0};
  int b = q;
  for (; b + 15 * kGramSets < nblk; b += 16 * kGramSets) {
    float v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = gpart[(b + i * kGramSets) * stride + e];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i & 3] += static_cast<double>(v[i]);
  }
  for (; b < nblk; b += kGramSets) a[0] += static_cast<double>(gpart[b * stride + e]);
  part2[q * stride + e] = (a[0] + a[1]) + (a[2] + a[3]);
}

// ---- Newton direction: J delta = -F(gamma), J = I + diag(e) M, by LU with
// partial pivoting (pivot rows left in place, pivot order recorded).  A is
// J in LDS with pitch L + 1.  Sets delta, the trial point gamma + delta and
// resets the line search.
__device__ void ssn_set_direction(const double* __restrict__ sol, int L, double* __restrict__ state) {
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    state[SsnState::kDelta + k] = sol[k];
    state[SsnState::kTry + k] = state[SsnState::kGamma + k] + sol[k];
  }
  if (threadIdx.x == 0) {
    state[SsnState::kT] = 1.0;
    state[SsnState::kHalv] = 0.0;
    state[SsnState::kSteps] += 1.0;
  }
}

// Value of v on lane `lane` (wave-uniform index) through the scalar unit.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffu), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
  return __longlong_as_double((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                              static_cast<unsigned>(lo));
}

// Maximum of v over the 64 lanes through DPP moves (quad permutes, row
// mirrors, then the row broadcasts that carry each row's maximum into the
// next rows); lane 63 ends with the wave maximum.  Lanes outside a row mask
// keep their value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_max(float v) {
  const int o = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK,
                                            0xf, false);
  return fmaxf(v, __int_as_float(o));
}

__device__ __forceinline__ float wave_max_f32(float v) {
  v = dpp_max<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
  v = dpp_max<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
  v = dpp_max<0x141, 0xf>(v);   // row_half_mirror
  v = dpp_max<0x140, 0xf>(v);   // row_mirror
  v = dpp_max<0x142, 0xa>(v);   // row_bcast15 into rows 1 and 3
  v = dpp_max<0x143, 0xc>(v);   // row_bcast31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float wave_max_r(float v) { return wave_max_f32(v); }
__device__ __forceinline__ double wave_max_r(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double readlane_r(double v, int lane) { return readlane_f64(v, lane); }

// L <= LM (16, 32 or 64) on wave 0 alone, arithmetic in R (float for an FP32
// U: the Newton direction only has to resolve F to the FP32 stopping
// tolerance; double otherwise).  Lane r holds row r of J in LM registers and
// the right-hand side; the fully unrolled elimination addresses columns by
// constant register index and reads the pivot row through the scalar unit,
// so there is no barrier and no LDS traffic per column.  Partial pivoting
// (largest |J[r][j]| over the rows not yet used, lowest row on ties) with
// the pivot rows left in place; the back substitution runs in the same wave
// and lane j ends with delta_j.
template <class R, int LM>
__device__ void lu_wave_regs(const double* __restrict__ A, int L, double* __restrict__ state) {
  const int r = threadIdx.x;
  const int LP1 = L + 1;
  R a[LM];
#pragma unroll
  for (int c = 0; c < LM; ++c)
    a[c] = (r < L && c < L) ? static_cast<R>(A[r * LP1 + c]) : (r == c ? R(1) : R(0));
  R rh = (r < L) ? static_cast<R>(-state[SsnState::kF + r]) : R(0);
  bool used = r >= L;
  int piv = 0;   // lane j: the pivot row of column j
#pragma unroll
  for (int j = 0; j < LM; ++j) {
    if (j < L) {
      const R val = used ? R(-1) : static_cast<R>(fabs(a[j]));
      const R m = wave_max_r(val);
      const unsigned long long hit = __ballot(!used && val == m);
      const int p = __builtin_amdgcn_readfirstlane(__ffsll(static_cast<unsigned long long>(hit)) - 1);
      const R inv = R(1) / readlane_r(a[j], p);
      const R f = (used || r == p) ? R(0) : a[j] * inv;
      if (r == p) used = true;
#pragma unroll
      for (int k = j + 1; k < LM; ++k) a[k] -= f * readlane_r(a[k], p);
      rh -= f * readlane_r(rh, p);
      if (r == j) piv = p;
    }
  }
  R sol = 0;
#pragma unroll
  for (int j = LM - 1; j >= 0; --j) {
    if (j < L) {
      const int p = __builtin_amdgcn_readlane(piv, j);
      const R d = readlane_r(rh, p) / readlane_r(a[j], p);
      if (r == j) sol = d;
      rh -= a[j] * d;
    }
  }
  if (r < L) {
    const double dv = static_cast<double>(sol);
    state[SsnState::kDelta + r] = dv;
    state[SsnState::kTry + r] = state[SsnState::kGamma + r] + dv;
  }
  if (r == 0) {
    state[SsnState::kT] = 1.0;
    state[SsnState::kHalv] = 0.0;
    state[SsnState::kSteps] += 1.0;
  }
}

// Any L <= 128: elimination on wave 0 alone (lane r owns rows r and r + 64).
__device__ void lu_wave(double* __restrict__ A, int L, double* __restrict__ state) {
  __shared__ double rhs[PcMeta::kMaxEll], sol[PcMeta::kMaxEll];
  __shared__ int porder[PcMeta::kMaxEll];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int LP1 = L + 1;
  for (int i = tid; i < L; i += blockDim.x) rhs[i] = -state[SsnState::kF + i];
  __syncthreads();
  if (wave == 0) {
    const int r0 = lane, r1 = lane + 64;
    bool used0 = r0 >= L, used1 = r1 >= L;
    for (int j = 0; j < L; ++j) {
      double best = -1.0;
      int bi = -1;
      if (!used0) { best = fabs(A[r0 * LP1 + j]); bi = r0; }
      if (!used1) { const double v = fabs(A[r1 * LP1 + j]); if (v > best) { best = v; bi = r1; } }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi >= 0 && (bi < 0 || oi < bi))) { best = ob; bi = oi; }
      }
      const int p = bi;
      if (lane == 0) porder[j] = p;
      if (p == r0) used0 = true;
      if (p == r1) used1 = true;
      const double idp = 1.0 / A[p * LP1 + j];
      const double rp = rhs[p];
      if (!used0) {
        const double f = A[r0 * LP1 + j] * idp;
        for (int k = j + 1; k < L; ++k) A[r0 * LP1 + k] -= f * A[p * LP1 + k];
        rhs[r0] -= f * rp;
      }
      if (!used1) {
        const double f = A[r1 * LP1 + j] * idp;
        for (int k = j + 1; k < L; ++k) A[r1 * LP1 + k] -= f * A[p * LP1 + k];
        rhs[r1] -= f * rp;
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
    for (int j = L - 1; j >= 0; --j) {
      const int p = porder[j];
      double ps = 0;
      for (int k = j + 1 + lane; k < L; k += 64) ps += A[p * LP1 + k] * sol[k];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) ps += __shfl_xor(ps, o, 64);
      if (lane == 0) sol[j] = (rhs[p] - ps) / A[p * LP1 + j];
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  ssn_set_direction(sol, L, state);
}

// FP32 inverse of J (L <= 64) by Gauss-Jordan elimination in place, on 1024
// threads: thread t holds J[i][4q .. 4q + 3] (i = t / 16, q = t % 16; the
// identity past L) in registers; at step k the holders of row k and of column
// k publish their old values through LDS (two buffers: one barrier a step),
// and every thread updates its four entries.  No row exchanges: every leading
// principal block of J = I + diag(e) M is I + E_k M_k with M_k a principal
// block of U^T D U (0 <= M_k <= I) and e > -1, so E_k M_k (similar to
// M_k^1/2 E_k M_k^1/2) has real eigenvalues above -1 and no pivot vanishes.
// A pivot below 2^-12 max |J| (lost accuracy) or a non-finite entry returns
// false with nothing written, and the caller solves with partial pivoting.
// Otherwise it sets the direction -J^{-1} F, the trial point, and stores
// J^{-1} (row pitch kLuPitch) for the chord steps of later calls.
__device__ bool gj_inverse_1024(const double* __restrict__ A, int L, double* __restrict__ state,
                                float* __restrict__ jinv) {
  __shared__ float rowb[2][64], colb[2][64];
  __shared__ float wmax[16];
  __shared__ float Fs[64];
  const int t = threadIdx.x, i = t >> 4, q = t & 15, j0 = 4 * q;
  const int LP1 = L + 1;
  float a[4];
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + c;
    a[c] = (i < L && j < L) ? static_cast<float>(A[i * LP1 + j]) : (i == j ? 1.f : 0.f);
    if (i < L && j < L) m = fmaxf(m, fabsf(a[c]));
  }
  if (t < 64) Fs[t] = t < L ? static_cast<float>(state[SsnState::kF + t]) : 0.f;
  m = wave_max_f32(m);
  if ((t & 63) == 0) wmax[t >> 6] = m;
  __syncthreads();
  float amax = 0.f;
#pragma unroll
  for (int w = 0; w < 16; ++w) amax = fmaxf(amax, wmax[w]);
  const float thresh = 0x1p-12f * amax;
  bool small = false;
  for (int k = 0; k < L; ++k) {
    const int b = k & 1;
    if (i == k) {
#pragma unroll
      for (int c = 0; c < 4; ++c) rowb[b][j0 + c] = a[c];
    }
    if (q == (k >> 2)) {
      const int c = k & 3;
      colb[b][i] = c == 0 ? a[0] : c == 1 ? a[1] : c == 2 ? a[2] : a[3];
    }
    __syncthreads();
    const float p = rowb[b][k];
    const float f = colb[b][i];
    const float ip = 1.f / p;
    small = small || !(fabsf(p) >= thresh);
    if (i == k) {
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] = (j0 + c == k) ? ip : a[c] * ip;
    } else {
      const float fi = f * ip;
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] = (j0 + c == k) ? -fi : a[c] - fi * rowb[b][j0 + c];
    }
  }
  bool bad = small || !isfinite(a[0]) || !isfinite(a[1]) || !isfinite(a[2]) || !isfinite(a[3]);
  if (__syncthreads_or(bad)) return false;
  // direction -J^{-1} F: the 16 holders of a row reduce their partial sums
  float sacc = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) sacc += a[c] * Fs[j0 + c];
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) sacc += __shfl_xor(sacc, o, 16);
  if (i < L) {
    if (q == 0) {
      const double dv = -static_cast<double>(sacc);
      state[SsnState::kDelta + i] = dv;
      state[SsnState::kTry + i] = state[SsnState::kGamma + i] + dv;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (j0 + c < L) jinv[i * kLuPitch + j0 + c] = a[c];
  }
  if (t == 0) {
    state[SsnState::kT] = 1.0;
    state[SsnState::kHalv] = 0.0;
    state[SsnState::kSteps] += 1.0;
    state[SsnState::kLuOk] = 1.0;
  }
  return true;
}

// Chord step (FP32, L <= 64): the direction -J0^{-1} F(gamma) with the stored
// inverse of an earlier Jacobian J0 of the same preconditioner (the masks of
// consecutive prox centres differ in few pixels); lane r forms row r.
__global__ __launch_bounds__(64) void ssn_chord_kernel(const float* __restrict__ jinv, int L,
                                                       double* __restrict__ state) {
  __shared__ float Fs[64];
  // only after a decision that accepted its point without converging, and
  // with an inverse stored; the inverse, F and gamma are requested together
  // with the flags (the buffer always exists; its values are used only if
  // stored)
  const int r = threadIdx.x;
  const double done = state[SsnState::kDone], need = state[SsnState::kNeedGram],
               luok = state[SsnState::kLuOk];
  float a[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) a[c] = (r < L && c < L) ? jinv[r * kLuPitch + c] : 0.f;
  const double fr = r < L ? state[SsnState::kF + r] : 0.0;
  const double gr = r < L ? state[SsnState::kGamma + r] : 0.0;
  if (done != 0.0 || need == 0.0 || luok == 0.0) return;
  Fs[r] = static_cast<float>(fr);
  __syncthreads();
  float sacc = 0.f;
#pragma unroll
  for (int c = 0; c < 64; ++c) sacc += a[c] * Fs[c];
  if (r < L) {
    const double dv = -static_cast<double>(sacc);
    state[SsnState::kDelta + r] = dv;
    state[SsnState::kTry + r] = gr + dv;
  }
  if (r == 0) {
    state[SsnState::kT] = 1.0;
    state[SsnState::kHalv] = 0.0;
    state[SsnState::kSteps] += 1.0;
  }
}

template <class R, int LM>
__device__ __forceinline__ void lu_wave_any(const double* A, int L, double* state) {
  if (threadIdx.x >= 64) return;
  lu_wave_regs<R, LM>(A, L, state);
}

template <class R>
__device__ __forceinline__ void ssn_lu(double* A, int L, double* state) {
  if (L <= 16) lu_wave_any<R, 16>(A, L, state);
  else if (L <= 32) lu_wave_any<R, 32>(A, L, state);
  else if (L <= 64) lu_wave_any<R, 64>(A, L, state);
  else lu_wave(A, L, state);
}

// One block: J = I + diag(e) M with M = sum of the kGramSets stage-2
// partials, then the LU solve.
template <int NRG>
__global__ __launch_bounds__(1024) void ssn_solve_kernel(const double* __restrict__ part2, int L,
                                                        const double* __restrict__ meta,
                                                        double* __restrict__ state, int force,
                                                        float* __restrict__ lu) {
  constexpr int NTRI = NRG * (NRG + 1) / 2;
  extern __shared__ double A[];
  if (state[SsnState::kDone] != 0.0 || (state[SsnState::kNeedGram] == 0.0 && !force)) return;
  const int LP1 = L + 1;
  const size_t stride = static_cast<size_t>(NTRI) * 1024;
  for (int e = threadIdx.x; e < NTRI * 1024; e += blockDim.x) {
    const int tile = e >> 10, rr = e & 1023;
    int ti = 0, t = tile;
    while (t >= NRG - ti) { t -= NRG - ti; ++ti; }
    const int tj = ti + t;
    const int gi = 32 * ti + (rr >> 5), gj = 32 * tj + (rr & 31);
    if (gi >= L || gj >= L || (ti == tj && gi > gj)) continue;
    double v[kGramSets];
#pragma unroll
    for (int b = 0; b < kGramSets; ++b) v[b] = part2[b * stride + e];
    double sacc = 0;
#pragma unroll
    for (int b = 0; b < kGramSets; ++b) sacc += v[b];
    A[gi * LP1 + gj] = (gi == gj ? 1.0 : 0.0) + meta[PcMeta::kE + gi] * sacc;
    if (gi != gj) A[gj * LP1 + gi] = meta[PcMeta::kE + gj] * sacc;
  }
  __syncthreads();
  // Gauss-Jordan inverse without row exchanges; the compact pivoted
  // elimination of the whole block only if that reports lost accuracy
  bool diag_ok = false;
  if constexpr (NRG <= 2) diag_ok = gj_inverse_1024(A, L, state, lu);
  if (!diag_ok) {
    if (threadIdx.x == 0) state[SsnState::kLuOk] = 0.0;   // no stored factors from this path
    lu_wave(A, L, state);
  }
}

// FP64 U: masked Gram on the vector units, one 64 x 64 output tile per block
// and chunk, then the same reduction + solve in a second small kernel.
__global__ __launch_bounds__(256) void ssn_gram_f64_kernel(const double* __restrict__ U,
                                                           int64_t ldu,
                                                           const uint8_t* __restrict__ mask,
                                                           const double* __restrict__ state,
                                                           int64_t N, int L, int64_t chunk,
                                                           double* __restrict__ part) {
  if (state[SsnState::kDone] != 0.0 || state[SsnState::kNeedGram] == 0.0) return;
  const int ti = blockIdx.y, tj = blockIdx.z;
  if (tj < ti) return;
  __shared__ double As[32][65];
  __shared__ double Bs[32][65];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int64_t nb = n0; nb < n1; nb += 32) {
    for (int e = threadIdx.x; e < 32 * 64; e += 256) {
      int c = e / 32, kk = e - c * 32;
      int64_t n = nb + kk;
      int ka = ti * 64 + c, kb = tj * 64 + c;
      bool on = n < n1 && mask[n];
      As[kk][c] = (on && ka < L) ? U[static_cast<size_t>(ka) * ldu + n] : 0.0;
      Bs[kk][c] = (on && kb < L) ? U[static_cast<size_t>(kb) * ldu + n] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 32; ++kk) {
      double a[4], b[4];
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
        part[blockIdx.x * LL + static_cast<size_t>(ia) * L + ib] = acc[p][q];
        part[blockIdx.x * LL + static_cast<size_t>(ib) * L + ia] = acc[p][q];
      }
    }
}

__global__ __launch_bounds__(256) void ssn_solve_f64_kernel(const double* __restrict__ part,
                                                            int nchunks, int L,
                                                            const double* __restrict__ meta,
                                                            double* __restrict__ state) {
  extern __shared__ double A[];
  if (state[SsnState::kDone] != 0.0 || state[SsnState::kNeedGram] == 0.0) return;
  const size_t LL = static_cast<size_t>(L) * L;
  for (size_t e = threadIdx.x; e < LL; e += blockDim.x) {
    const int i = static_cast<int>(e / L), j = static_cast<int>(e % L);
    double sacc = 0;
    for (int c = 0; c < nchunks; ++c) sacc += part[c * LL + e];
    A[i * (L + 1) + j] = (i == j ? 1.0 : 0.0) + meta[PcMeta::kE + i] * sacc;
  }
  __syncthreads();
  ssn_lu<double>(A, L, state);
}

// x = soft(s - U gamma)
template <class T>
__global__ __launch_bounds__(256) void ssn_final_kernel(const T* __restrict__ U, int64_t ldu,
                                                        const T* __restrict__ s,
                                                        const double* __restrict__ state,
                                                        int64_t N, int L, T lam, T* __restrict__ x,
                                                        int box, T lo, T hi, int unfinished_only) {
  __shared__ T g[PcMeta::kMaxEll];
  // (unfinished_only) the converged trial has written x already
  if (unfinished_only && state[SsnState::kDone] != 0.0 && state[SsnState::kBad] == 0.0) return;
  for (int k = threadIdx.x; k < L; k += blockDim.x) g[k] = static_cast<T>(state[SsnState::kGamma + k]);
  __syncthreads();
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T ug = 0;
  for (int k = 0; k < L; ++k) ug += U[static_cast<size_t>(k) * ldu + n] * g[k];
  const T r = s[n] - ug;
  x[n] = ssn_h_prox(r, lam, box, lo, hi);
}

// Initialise the Newton state from the warm start gamma (g_try = gamma).
// keep_lu = 0 marks the stored LU factors as not belonging to this
// preconditioner.
__global__ void ssn_init_kernel(double* __restrict__ state, const double* __restrict__ gamma0, int L,
                                int keep_lu) {
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    double g = gamma0 ? gamma0[k] : 0.0;
    state[SsnState::kGamma + k] = g;
    state[SsnState::kTry + k] = g;
    state[SsnState::kDelta + k] = 0.0;
  }
  if (threadIdx.x == 0) {
    state[SsnState::kNF] = 0; state[SsnState::kT] = 1; state[SsnState::kDone] = 0;
    state[SsnState::kHalv] = 0; state[SsnState::kHave] = 0; state[SsnState::kNeedGram] = 0;
    state[SsnState::kTrials] = 0; state[SsnState::kSteps] = 0; state[SsnState::kBad] = 0;
    if (!keep_lu) state[SsnState::kLuOk] = 0;
  }
}

__global__ void ssn_store_gamma_kernel(const double* __restrict__ state, double* __restrict__ gamma, int L,
                                       int unfinished_only) {
  if (unfinished_only && state[SsnState::kDone] != 0.0) return;
  for (int k = threadIdx.x; k < L; k += blockDim.x) gamma[k] = state[SsnState::kGamma + k];
}

// The outcome of a device-decided call: a non-finite ||F|| (status[0] =
// NYS_ENOTFINITE) or no convergence within its trials (status[1] = NYS_ENOCONV).
__global__ void ssn_status_kernel(const double* __restrict__ state, int32_t* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (state[SsnState::kBad] != 0.0) status[0] = NYS_ENOTFINITE;
  else if (state[SsnState::kDone] == 0.0) status[1] = NYS_ENOCONV;
}

template <class T, int ROWS>
static void launch_ssn_eval(nys_pc pc, const T* s, T lam, double* state, uint8_t* mask,
                            double* part, int nblk, int64_t chunk, T* xo, hipStream_t st) {
  hipLaunchKernelGGL((ssn_eval_kernel<T, ROWS>), dim3(nblk), dim3(512), 0, st, pc->U.as<T>(),
                     pc->ldu, s, pc->N, static_cast<int>(pc->ell), chunk, lam, state, mask, part, xo,
                     pc->ssn_box, static_cast<T>(pc->ssn_lo), static_cast<T>(pc->ssn_hi));
}

template <class T>
static nys_status launch_eval(nys_pc pc, const T* s, T lam, double* state, uint8_t* mask,
                              double* part, int nblk, int64_t chunk, double tol, hipStream_t st,
                              T* xo = nullptr) {
  switch (pc->ell_pad) {
    case 16: launch_ssn_eval<T, 16>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    case 32: launch_ssn_eval<T, 32>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    case 48: launch_ssn_eval<T, 48>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    case 64: launch_ssn_eval<T, 64>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    case 80: launch_ssn_eval<T, 80>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    case 96: launch_ssn_eval<T, 96>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    case 112: launch_ssn_eval<T, 112>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
    default: launch_ssn_eval<T, 128>(pc, s, lam, state, mask, part, nblk, chunk, xo, st); break;
  }
  NYS_TRY(launch_check("ssn_eval_kernel"));
  hipLaunchKernelGGL(ssn_decide_kernel, dim3(1), dim3(1024), 0, st, part, nblk,
                     static_cast<int>(pc->ell), pc->meta.as<double>(), state, tol, 30, pc->hflag,
                     ++pc->flag_seq, pc->ssn_gout);
  return launch_check("ssn_decide_kernel");
}

template <int ROWS>
static void launch_ssn_eval_step(nys_pc pc, const SsnStep& sp, const double* gamma0, int keep_lu,
                                 float* s_out, float lam, double* state, double* part, int nblk,
                                 int64_t chunk, float* xo, hipStream_t st) {
  hipLaunchKernelGGL((ssn_eval_step_kernel<ROWS>), dim3(nblk), dim3(512), 0, st, pc->U.as<float>(),
                     pc->ldu, static_cast<const float*>(sp.u), static_cast<const float*>(sp.g),
                     static_cast<float>(sp.alpha), sp.cp.part, sp.cp.nblk,
                     pc->meta.as<double>() + PcMeta::kD, gamma0, keep_lu, s_out, pc->N,
                     static_cast<int>(pc->ell), chunk, lam, state, part, xo);
}

// The decision on the partials of an evaluation; with lu, followed by the
// chord step from the stored factors (FP32, L <= 64).
static nys_status launch_decide(nys_pc pc, double* part, int nblk, double* state, double tol,
                                const float* lu, hipStream_t st) {
  const int L = static_cast<int>(pc->ell);
  if (lu == nullptr) {
    hipLaunchKernelGGL(ssn_decide_kernel, dim3(1), dim3(1024), 0, st, part, nblk, L,
                       pc->meta.as<double>(), state, tol, 30, pc->hflag, ++pc->flag_seq,
                       pc->ssn_gout);
    return launch_check("ssn_decide_kernel");
  }
  if (L <= 32)
    hipLaunchKernelGGL(ssn_decide_chord_kernel<32>, dim3(1), dim3(1024), 0, st, part, nblk, L,
                       pc->meta.as<double>(), state, tol, 30, pc->hflag, ++pc->flag_seq,
                       pc->ssn_gout, lu);
  else
    hipLaunchKernelGGL(ssn_decide_chord_kernel<64>, dim3(1), dim3(1024), 0, st, part, nblk, L,
                       pc->meta.as<double>(), state, tol, 30, pc->hflag, ++pc->flag_seq,
                       pc->ssn_gout, lu);
  return launch_check("ssn_decide_chord_kernel");
}

// The first trial with the gradient step and the state initialisation fused
// in, and its decision (with the chord step when lu is given).
static nys_status launch_eval_step(nys_pc pc, const SsnStep& sp, const double* gamma0, int keep_lu,
                                   float* s_out, float lam, double* state, double* part, int nblk,
                                   int64_t chunk, double tol, float* xo, const float* lu,
                                   hipStream_t st) {
  switch (pc->ell_pad) {
    case 16: launch_ssn_eval_step<16>(pc, sp, gamma0, keep_lu, s_out, lam, state, part, nblk, chunk, xo, st); break;
    case 32: launch_ssn_eval_step<32>(pc, sp, gamma0, keep_lu, s_out, lam, state, part, nblk, chunk, xo, st); break;
    case 48: launch_ssn_eval_step<48>(pc, sp, gamma0, keep_lu, s_out, lam, state, part, nblk, chunk, xo, st); break;
    default: launch_ssn_eval_step<64>(pc, sp, gamma0, keep_lu, s_out, lam, state, part, nblk, chunk, xo, st); break;
  }
  NYS_TRY(launch_check("ssn_eval_step_kernel"));
  return launch_decide(pc, part, nblk, state, tol, lu, st);
}

// One trial of the FP32 Newton iteration: the fused evaluation + masked Gram
// at the trial point, the decision, and (if it asks for one) the Newton step;
// or (newton_at_gamma) the Newton step at the accepted point alone.
template <int NRG>
static nys_status launch_ssn_trial(nys_pc pc, const float* s, float lam, double* state,
                                   double* fpart, float* part, int nblk, int64_t chunk, double tol,
                                   float* x, float* lu, hipStream_t st, bool newton_at_gamma = false,
                                   bool need_only = false) {
  constexpr int NTRI = NRG * (NRG + 1) / 2;
  const int L = static_cast<int>(pc->ell);
  constexpr size_t elds = evg_lds_bytes<NRG>();
  static_assert(elds >= sizeof(float) * NTRI * 1024, "LDS of the fused pass holds the Gram sum");
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ssn_evalgram_kernel<NRG>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(elds));
  hipLaunchKernelGGL((ssn_evalgram_kernel<NRG>), dim3(nblk), dim3(64 * evg_waves<NRG>()), elds, st,
                     pc->U.as<float>(), pc->ldu, s, pc->N, L, chunk, lam, state, fpart, part, x,
                     static_cast<int>(newton_at_gamma ? SsnState::kGamma : SsnState::kTry),
                     pc->ssn_box, static_cast<float>(pc->ssn_lo), static_cast<float>(pc->ssn_hi),
                     need_only ? 1 : 0);
  NYS_TRY(launch_check("ssn_evalgram_kernel"));
  double* part2 = reinterpret_cast<double*>(part + static_cast<size_t>(nblk) * NTRI * 1024);
  const int with_decide = newton_at_gamma ? 0 : 1;
  if (with_decide) ++pc->flag_seq;
  hipLaunchKernelGGL((ssn_decide_gram_kernel<NRG>), dim3(NTRI * 4 + with_decide), dim3(1024), 0, st,
                     fpart, nblk, L, pc->meta.as<double>(), state, tol, 30, pc->hflag, pc->flag_seq,
                     pc->ssn_gout, part, part2, with_decide, need_only ? 1 : 0);
  NYS_TRY(launch_check("ssn_decide_gram_kernel"));
  const size_t lds = sizeof(double) * pc->ell * (pc->ell + 1);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ssn_solve_kernel<NRG>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  hipLaunchKernelGGL((ssn_solve_kernel<NRG>), dim3(1), dim3(1024), lds, st, part2,
                     static_cast<int>(pc->ell), pc->meta.as<double>(), state,
                     newton_at_gamma && !need_only ? 1 : 0, lu);
  return launch_check("ssn_solve_kernel");
}

// Waits until the decision kernel last enqueued on st has published its
// outcome (sequence number pc->flag_seq).  Spins on the pinned word for up to
// 2 s, then falls back to a stream synchronisation.
static nys_status ssn_wait_decision(nys_pc pc, hipStream_t st, bool& done, bool& need_gram,
                                    bool& lu_ok, bool& bad) {
  volatile unsigned long long* f = pc->hflag;
  const unsigned long long want = pc->flag_seq;
  const auto t0 = std::chrono::steady_clock::now();
  unsigned long long w = *f;
  while ((w >> 4) != want) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      NYS_CHECK_HIP(hipStreamSynchronize(st));
      w = *f;
      if ((w >> 4) != want) {
        set_error("semismooth Newton decision %llu not published", want);
        return NYS_EHIP;
      }
      break;
    }
    w = *f;
  }
  bad = (w & 8) != 0;
  done = (w & 4) != 0;
  need_gram = (w & 2) != 0;
  lu_ok = (w & 1) != 0;
  return NYS_OK;
}

// Geometry and buffer layout of the semismooth Newton iteration for N pixels,
// L columns and es-byte values: the evaluation blocks, the fused evaluation +
// Gram blocks, the state, block partials, Gram partials, the FP64 Jacobian,
// the active-set mask and the stored FP32 Jacobian inverse.  The buffer is
// allocated with the preconditioner (ssn_ws_bytes).
struct SsnLayout {
  int nblk, ngb, nrg;
  int64_t chunk, gchunk;
  size_t gpart_d, need, mask_b, lu_b;
  SsnLayout(int64_t N, int L, size_t es) {
    red_geometry(N, nblk, chunk);
    // fused pass: one block per CU at most, at least two 64-pixel stages per
    // wave of a block (1024 pixels for 8 waves), chunks a multiple of 64
    const int nrg0 = (L + 31) / 32;
    const int64_t per_blk = 64 * 2 * (nrg0 <= 2 ? 8 : 4);
    const int64_t gblk = std::min<int64_t>(256, std::max<int64_t>(1, (N + per_blk - 1) / per_blk));
    gchunk = (N + gblk - 1) / gblk;
    gchunk = (gchunk + 63) / 64 * 64;
    ngb = static_cast<int>((N + gchunk - 1) / gchunk);
    nrg = (L + 31) / 32;
    const size_t LL = static_cast<size_t>(L) * L;
    const size_t ntri = static_cast<size_t>(nrg) * (nrg + 1) / 2;
    if (es == 4)   // block partials (FP32), then part2 (kGramSets sets)
      gpart_d = (static_cast<size_t>(ngb) * ntri * 1024 + 1) / 2 + kGramSets * ntri * 1024 + 1;
    else gpart_d = static_cast<size_t>(cdiv(N, 4096)) * LL;
    need = SsnState::kTotal + static_cast<size_t>(std::max(nblk, ngb)) * L + gpart_d + LL;
    mask_b = static_cast<size_t>((N + 255) / 256 * 256);
    lu_b = sizeof(float) * kLuPitch * kLuPitch;
  }
  size_t bytes() const { return sizeof(double) * need + mask_b + lu_b + 256; }
};

size_t ssn_ws_bytes(int64_t N, int L, size_t es) { return SsnLayout(N, L, es).bytes(); }

template <class T>
static bool xf_ok(const T* x, const T* s) {
  return x != nullptr && static_cast<const void*>(x) != static_cast<const void*>(s);
}

template <class T>
nys_status ssn_prox(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                    double* gamma_state, hipStream_t st, int* trials_out, const SsnStep* step,
                    const SsnBox* box) {
  NYS_REQUIRE(!(box && step), "ssn_prox: a box projection has no gradient step");
  pc->ssn_box = box ? 1 : 0;   // read by the launchers of this call
  pc->ssn_lo = box ? box->lo : 0.0;
  pc->ssn_hi = box ? box->hi : 0.0;
  const int64_t N = pc->N;
  const int L = static_cast<int>(pc->ell);
  const SsnLayout ly(N, L, sizeof(T));
  const int nblk = ly.nblk, ngb = ly.ngb, nrg = ly.nrg;
  const int64_t chunk = ly.chunk, gchunk = ly.gchunk;
  const size_t LL = static_cast<size_t>(L) * L;
  NYS_REQUIRE(pc->ssn_ws.bytes >= ly.bytes(), "ssn_prox: semismooth Newton buffer too small");
  NYS_REQUIRE(pc->hflag, "ssn_prox: no decision word");
  double* state = pc->ssn_ws.as<double>();
  double* part = state + SsnState::kTotal;
  double* gpart = part + static_cast<size_t>(std::max(nblk, ngb)) * L;
  double* Mj = gpart + ly.gpart_d;
  uint8_t* mask = reinterpret_cast<uint8_t*>(Mj + LL);
  float* lu = reinterpret_cast<float*>(mask + ly.mask_b);
  const T lam = static_cast<T>(lam_bar);
  const double tol = reg.newton_tol > 0 ? reg.newton_tol : (sizeof(T) == 8 ? 1e-12 : 1e-6);
  const int max_trials = reg.max_newton > 0 ? reg.max_newton : 60;
  // stored factors are kept only while they belong to this preconditioner
  const bool fp32_lu = sizeof(T) == 4 && L <= 64;
  const bool have_lu = fp32_lu && pc->ssn_lu_valid;
  // With factors known to be stored, the first trial, its chord step and the
  // second trial are enqueued together (the chord step runs only if the first
  // decision asks for a direction; a converged first trial makes the second
  // one exit at once), and the host waits for the second decision only.
  // With `step` there, the first trial also initialises the state and forms
  // the gradient step from the partials of U^T g; otherwise the step is
  // formed into s first.
  if (pc->ssn_device) {
    // A call being captured: the first two trials as below (the gradient
    // step fused into the first, the chord step after its decision), then
    // ssn_slots rounds of a Newton step at the accepted point and a trial
    // there, every kernel skipping itself on the device state once the
    // iteration has converged (the Newton step of a later round also unless
    // the last decision asked for a direction).  The prox output is the
    // converged trial's, else soft(s - U gamma) at the last accepted point.
    NYS_REQUIRE(sizeof(T) == 4 && fp32_lu && have_lu && step != nullptr && xf_ok(x, s) && !box,
                "ssn_prox: a captured call needs FP32 U with ell <= 64, stored factors, the "
                "gradient step and x apart from s");
    if constexpr (sizeof(T) == 4) {
      pc->ssn_gout = gamma_state;
      float* sw = reinterpret_cast<float*>(const_cast<T*>(s));
      float* xw = reinterpret_cast<float*>(x);
      const float lf = static_cast<float>(lam);
      NYS_TRY(launch_eval_step(pc, *step, gamma_state, 1, sw, lf, state, part, nblk, chunk, tol,
                               xw, lu, st));
      NYS_TRY(launch_eval<float>(pc, sw, lf, state, nullptr, part, nblk, chunk, tol, st, xw));
      for (int r = 0; r < pc->ssn_slots; ++r) {
        float* gp = reinterpret_cast<float*>(gpart);
        nys_status ts;
        switch (nrg) {
          case 1: ts = launch_ssn_trial<1>(pc, sw, lf, state, part, gp, ngb, gchunk, tol, nullptr, lu, st, true, r > 0); break;
          default: ts = launch_ssn_trial<2>(pc, sw, lf, state, part, gp, ngb, gchunk, tol, nullptr, lu, st, true, r > 0); break;
        }
        NYS_TRY(ts);
        NYS_TRY(launch_eval<float>(pc, sw, lf, state, nullptr, part, nblk, chunk, tol, st, xw));
      }
      hipLaunchKernelGGL((ssn_final_kernel<float>), dim3(cdiv(N, 256)), dim3(256), 0, st,
                         pc->U.as<float>(), pc->ldu, sw, state, N, L, lf, xw, 0, 0.f, 0.f, 1);
      NYS_TRY(launch_check("ssn_final_kernel"));
      if (gamma_state) {
        hipLaunchKernelGGL(ssn_store_gamma_kernel, dim3(1), dim3(128), 0, st, state, gamma_state,
                           L, 1);
        NYS_TRY(launch_check("ssn_store_gamma_kernel"));
      }
      if (pc->ssn_status) {
        hipLaunchKernelGGL(ssn_status_kernel, dim3(1), dim3(64), 0, st, state, pc->ssn_status);
        NYS_TRY(launch_check("ssn_status_kernel"));
      }
      pc->ssn_gout = nullptr;
      return NYS_OK;
    }
  }
  const bool prelude = have_lu && pc->ssn_lu_hint && max_trials >= 2;
  const bool step_fused = sizeof(T) == 4 && prelude && step != nullptr;
  if (!step_fused) {
    hipLaunchKernelGGL(ssn_init_kernel, dim3(1), dim3(128), 0, st, state, gamma_state, L,
                       have_lu ? 1 : 0);
    NYS_TRY(launch_check("ssn_init_kernel"));
  }
  pc->ssn_gout = gamma_state;   // the deciding kernel stores the root
  int trial = 0;
  bool done = false, need_gram = false, lu_ok = false, bad = false;
  // FP32: without stored factors the first trial point (nearly always
  // followed by a Newton step) runs the fused evaluation + Gram pass; with
  // them, and at every later trial point, the evaluation runs alone.  A new
  // direction at an accepted point is then a chord step with the stored
  // factors of an earlier Jacobian of this preconditioner (once per call), else
  // a Newton step with its Gram pass at the accepted point (factors stored).
  // A chord direction that is not accepted at once is replaced by a Newton
  // step at the accepted point.
  bool chord_used = false, last_chord = false;
  float* xf = static_cast<const void*>(x) == static_cast<const void*>(s)
                  ? nullptr : reinterpret_cast<float*>(x);   // x aliasing s gets no trial writes
  auto fused = [&](bool at_gamma) -> nys_status {
    float* gp = reinterpret_cast<float*>(gpart);
    const float* sf = reinterpret_cast<const float*>(s);
    const float lf = static_cast<float>(lam);
    float* xo = at_gamma ? nullptr : xf;
    switch (nrg) {
      case 1: return launch_ssn_trial<1>(pc, sf, lf, state, part, gp, ngb, gchunk, tol, xo, lu, st, at_gamma);
      case 2: return launch_ssn_trial<2>(pc, sf, lf, state, part, gp, ngb, gchunk, tol, xo, lu, st, at_gamma);
      case 3: return launch_ssn_trial<3>(pc, sf, lf, state, part, gp, ngb, gchunk, tol, xo, lu, st, at_gamma);
      default: return launch_ssn_trial<4>(pc, sf, lf, state, part, gp, ngb, gchunk, tol, xo, lu, st, at_gamma);
    }
  };
  if (step != nullptr && !step_fused) {
    NYS_TRY(pc_tail(pc, true, step->cp, step->cd, st));
    NYS_TRY(pc_x_from_pinv<T>(pc, static_cast<const T*>(step->u), static_cast<const T*>(step->g),
                              step->cd, step->alpha, const_cast<T*>(s), st));
  }
  if (prelude) {
    const float* sf = reinterpret_cast<const float*>(s);
    const float lf = static_cast<float>(lam);
    if (step_fused) {
      NYS_TRY(launch_eval_step(pc, *step, gamma_state, 1, reinterpret_cast<float*>(const_cast<T*>(s)),
                               lf, state, part, nblk, chunk, tol, xf, lu, st));
    } else {
      NYS_TRY(launch_eval<float>(pc, sf, lf, state, nullptr, part, nblk, chunk, tol, st, xf));
      hipLaunchKernelGGL(ssn_chord_kernel, dim3(1), dim3(64), 0, st, lu, L, state);
      NYS_TRY(launch_check("ssn_chord_kernel"));
    }
    chord_used = last_chord = true;
    trial = 1;
  }
  for (; trial < max_trials; ++trial) {
    if constexpr (sizeof(T) == 4) {
      if (trial == 0 && !have_lu) {
        NYS_TRY(fused(false));
      } else {
        NYS_TRY(launch_eval<float>(pc, reinterpret_cast<const float*>(s), static_cast<float>(lam),
                                   state, nullptr, part, nblk, chunk, tol, st, xf));
      }
    } else {
      NYS_TRY(launch_eval<T>(pc, s, lam, state, mask, part, nblk, chunk, tol, st));
      const int ntile = static_cast<int>(cdiv(L, 64));
      const int nch = static_cast<int>(cdiv(N, 4096));
      hipLaunchKernelGGL(ssn_gram_f64_kernel, dim3(nch, ntile, ntile), dim3(256), 0, st,
                         reinterpret_cast<const double*>(pc->U.p), pc->ldu, mask, state, N, L,
                         static_cast<int64_t>(4096), gpart);
      NYS_TRY(launch_check("ssn_gram_f64_kernel"));
      const size_t lds = sizeof(double) * (LL + L);
      if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ssn_solve_f64_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
      hipLaunchKernelGGL(ssn_solve_f64_kernel, dim3(1), dim3(256), lds, st, gpart, nch, L,
                         pc->meta.as<double>(), state);
      NYS_TRY(launch_check("ssn_solve_f64_kernel"));
    }
    // the decision of this trial, read from pinned host memory while the
    // device goes on; the next trial is enqueued only if it is needed
    NYS_TRY(ssn_wait_decision(pc, st, done, need_gram, lu_ok, bad));
    if (fp32_lu) pc->ssn_lu_hint = lu_ok;
    if (done) break;
    if constexpr (sizeof(T) == 4) {
      const bool fused_here = trial == 0 && !have_lu;   // its Newton step is already enqueued
      if (!fused_here) {
        if (need_gram && fp32_lu && lu_ok && !chord_used) {
          hipLaunchKernelGGL(ssn_chord_kernel, dim3(1), dim3(64), 0, st, lu, L, state);
          NYS_TRY(launch_check("ssn_chord_kernel"));
          chord_used = last_chord = true;
        } else if (need_gram || last_chord) {
          NYS_TRY(fused(true));
          last_chord = false;
        }
        // else: a Newton direction being backtracked; the decision has set
        // the next trial point
      }
    }
  }
  if (fp32_lu && !bad) pc->ssn_lu_valid = true;
  if (trials_out) *trials_out = done ? trial + 1 : trial;
  // the FP32 pass has written soft(s - U g) of its trial point g to x: when
  // the iteration stopped there (accepted and converged), x is the prox
  if (!(sizeof(T) == 4 && done && xf != nullptr)) {
    hipLaunchKernelGGL((ssn_final_kernel<T>), dim3(cdiv(N, 256)), dim3(256), 0, st, pc->U.as<T>(),
                       pc->ldu, s, state, N, L, lam, x, pc->ssn_box, static_cast<T>(pc->ssn_lo),
                       static_cast<T>(pc->ssn_hi), 0);
    NYS_TRY(launch_check("ssn_final_kernel"));
  }
  pc->ssn_gout = nullptr;
  if (gamma_state && !done) {   // the trials ran out: the last accepted point
    hipLaunchKernelGGL(ssn_store_gamma_kernel, dim3(1), dim3(128), 0, st, state, gamma_state, L, 0);
    NYS_TRY(launch_check("ssn_store_gamma_kernel"));
  }
  if (bad) {
    set_error("semismooth Newton: non-finite ||F|| (NaN or infinity in the prox centre or U)");
    return NYS_ENOTFINITE;
  }
  if (!done) {
    set_error("semismooth Newton: no convergence within %d trial points", max_trials);
    return NYS_ENOCONV;
  }
  return NYS_OK;
}

template nys_status ssn_prox<double>(const nys_reg_desc&, double, nys_pc, const double*, double*,
                                     double*, hipStream_t, int*, const SsnStep*, const SsnBox*);
template nys_status ssn_prox<float>(const nys_reg_desc&, double, nys_pc, const float*, float*,
                                    double*, hipStream_t, int*, const SsnStep*, const SsnBox*);

}  // namespace nys

// ================================================================ no-allocation P^{-1}
// nys_apply for callers that cannot allocate: the coefficients and the block
// partials of U^T v live in one file-scope device array instead of a caller
// workspace.  Each device holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns on that device (the array's
// name is a host-side stand-in there).
namespace {

constexpr int kStaticApplyCols = 8;
// per column: ell coefficients and at most 256 blocks x 128 rows of partials,
// each part rounded to 256 bytes as the workspace stack hands them out
constexpr size_t kStaticApplyBytes =
    kStaticApplyCols * (((sizeof(double) * nys::PcMeta::kMaxEll + 255) / 256 * 256) +
                        ((sizeof(double) * 256 * nys::PcMeta::kMaxEll + 255) / 256 * 256));

__device__ __align__(256) char scratch[kStaticApplyBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices] = {};

// The device address of this device's array (looked up once per device, with
// the device current).
nys_status static_scratch(void** out) {
  int dev = 0;
  NYS_CHECK_HIP(hipGetDevice(&dev));
  NYS_REQUIRE(dev >= 0 && dev < kMaxDevices, "nys_apply_static: device %d out of range", dev);
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g_scratch_err[dev] == hipSuccess) g_scratch_ptr[dev] = p;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev]) {
    nys::set_error("nys_apply_static: hipGetSymbolAddress failed: %s",
                   hipGetErrorString(g_scratch_err[dev]));
    return NYS_EHIP;
  }
  *out = g_scratch_ptr[dev];
  return NYS_OK;
}

}  // namespace

extern "C" nys_status nys_apply_static(nys_pc pc, int32_t inverse, nys_dtype dt, const void* v,
                                       void* out, int64_t ncols, void* stream) {
  using namespace nys;
  NYS_REQUIRE(pc && v && out && ncols > 0, "nys_apply_static: bad argument");
  NYS_REQUIRE(ncols <= kStaticApplyCols, "nys_apply_static: ncols = %lld exceeds the maximum %d",
              static_cast<long long>(ncols), kStaticApplyCols);
  NYS_REQUIRE(static_cast<int32_t>(dt) == pc->u_dtype,
              "nys_apply_static: dtype must equal the pc's u_dtype");
  const size_t need = pc_ws_bytes(pc, ncols);
  NYS_REQUIRE(need <= kStaticApplyBytes, "nys_apply_static: needs %zu bytes of scratch > %zu", need,
              kStaticApplyBytes);
  void* ptr = nullptr;
  NYS_TRY(static_scratch(&ptr));
  WsBind bind(ptr, kStaticApplyBytes, nullptr, pc);
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return pc_apply<double>(pc, inverse != 0, static_cast<const double*>(v),
                            static_cast<double*>(out), ncols, st);
  return pc_apply<float>(pc, inverse != 0, static_cast<const float*>(v), static_cast<float*>(out),
                         ncols, st);
}
