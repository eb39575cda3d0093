// Shifted Nystrom factorisation (Alg. 1 steps 3-8) and the preconditioner of
// eq. (11): Gram of [Omega Y], ell x ell FP64 algebra on one workgroup,
// U = Y_nu R in one pass, and P^{-1} / P applications.

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "batch.hpp"

namespace nys {

// ================================================================ Gram
// G = Z^T Z for Z = [Omega | Y] (N x 2 ell, column-major).  Each block
// accumulates one 64 x 64 tile (upper triangle of tiles only) over a chunk
// of rows in the compute type C, then writes it in FP64; a second kernel sums
// the chunk partials in FP64 in a fixed order.
constexpr int kGT = 64, kGK = 32;

__host__ __device__ inline void tri_pair(int t, int ntiles, int& ti, int& tj) {
  ti = 0;
  while (t >= ntiles - ti) { t -= ntiles - ti; ++ti; }
  tj = ti + t;
}

template <class S, class C>
__device__ __forceinline__ void gram_partial_body(const S* __restrict__ omega,
                                                  const S* __restrict__ Y, int64_t N, int ell,
                                                  int64_t n0, int64_t n1, int ti, int tj,
                                                  double* __restrict__ dst) {
  const int m = 2 * ell;
  __shared__ C As[kGK][kGT + 1];
  __shared__ C Bs[kGK][kGT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  C acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int64_t nb = n0; nb < n1; nb += kGK) {
    for (int e = threadIdx.x; e < kGK * kGT; e += 256) {
      int col = e / kGK, kk = e - col * kGK;
      int64_t n = nb + kk;
      int ca = ti * kGT + col, cb = tj * kGT + col;
      C va = 0, vb = 0;
      if (n < n1) {
        if (ca < m) va = ca < ell ? Io<S>::ld(omega, static_cast<size_t>(ca) * N + n)
                                  : Io<S>::ld(Y, static_cast<size_t>(ca - ell) * N + n);
        if (cb < m) vb = cb < ell ? Io<S>::ld(omega, static_cast<size_t>(cb) * N + n)
                                  : Io<S>::ld(Y, static_cast<size_t>(cb - ell) * N + n);
      }
      As[kk][col] = va;
      Bs[kk][col] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kGK; ++kk) {
      C a[4], b[4];
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
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      dst[(ty * 4 + p) * kGT + tx * 4 + q] = static_cast<double>(acc[p][q]);
}

template <class S, class C>
__global__ __launch_bounds__(256) void gram_partial_kernel(
    const S* __restrict__ omega, const S* __restrict__ Y, int64_t N, int ell, int64_t chunk,
    int ntiles, double* __restrict__ part) {
  // blockIdx.y -> upper-triangular tile pair (ti <= tj)
  int ti, tj;
  tri_pair(blockIdx.y, ntiles, ti, tj);
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  const int ntri = ntiles * (ntiles + 1) / 2;
  gram_partial_body<S, C>(omega, Y, N, ell, n0, n1, ti, tj,
                          part + (static_cast<size_t>(blockIdx.x) * ntri + blockIdx.y) * kGT * kGT);
}

// Batched FP32 columns with FP64 accumulation: block -> (instance, chunk),
// blockIdx.y = tile pair (blocks past the instance's pairs exit).
__global__ __launch_bounds__(256) void bgram_kernel(const BDesc* __restrict__ d,
                                                    const BSeg* __restrict__ seg, int nseg) {
  const BSeg& sg = seg[seg_find(seg, nseg, blockIdx.x)];
  const BDesc& D = d[sg.inst];
  const int ntiles = (2 * D.ell + kGT - 1) / kGT;
  const int ntri = ntiles * (ntiles + 1) / 2;
  if (static_cast<int>(blockIdx.y) >= ntri) return;
  int ti, tj;
  tri_pair(blockIdx.y, ntiles, ti, tj);
  const int64_t lb = blockIdx.x - sg.first;
  const int64_t n0 = lb * sg.chunk;
  const int64_t n1 = (n0 + sg.chunk < D.N) ? n0 + sg.chunk : D.N;
  gram_partial_body<float, double>(D.omega, D.Y, D.N, D.ell, n0, n1, ti, tj,
                                   D.gpart + (static_cast<size_t>(lb) * ntri + blockIdx.y) * kGT * kGT);
}

__device__ __forceinline__ void gram_reduce_body(const double* __restrict__ part, int nchunks,
                                                 int ntiles, int ell, double* __restrict__ G,
                                                 int64_t e0, int64_t estride) {
  const int ntri = ntiles * (ntiles + 1) / 2;
  const int m = 2 * ell;
  const int64_t total = static_cast<int64_t>(ntri) * kGT * kGT;
  for (int64_t e = e0; e < total; e += estride) {
    int tri = static_cast<int>(e / (kGT * kGT));
    int r = static_cast<int>(e % (kGT * kGT));
    int i = r / kGT, j = r - i * kGT;
    int t = tri, ti = 0;
    while (t >= ntiles - ti) { t -= ntiles - ti; ++ti; }
    int tj = ti + t;
    int gi = ti * kGT + i, gj = tj * kGT + j;
    if (gi >= m || gj >= m) continue;
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += part[(static_cast<size_t>(c) * ntri + tri) * kGT * kGT + r];
    G[gi * m + gj] = s;
    G[gj * m + gi] = s;
  }
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, int nchunks, int ntiles,
                                   int ell, double* __restrict__ G) {
  gram_reduce_body(part, nchunks, ntiles, ell, G,
                   blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x,
                   static_cast<int64_t>(gridDim.x) * blockDim.x);
}

// Batched: blockIdx.y = segment of the Gram launch.
__global__ void bgram_reduce(const BDesc* __restrict__ d, const BSeg* __restrict__ seg) {
  const BSeg& sg = seg[blockIdx.y];
  const BDesc& D = d[sg.inst];
  gram_reduce_body(D.gpart, static_cast<int>(sg.nblk), (2 * D.ell + kGT - 1) / kGT, D.ell, D.G,
                   blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x,
                   static_cast<int64_t>(gridDim.x) * blockDim.x);
}

// ---------------------------------------------------------------- MFMA Gram
// BF16 / FP32 columns: G = Z Z^T with Z = [Omega; Y] (2 ell rows of N), on
// the matrix cores.  Rows are split in groups of 32; the upper-triangular
// 32 x 32 tiles are spread over the 4 waves of a block, and each block sums
// one chunk of N.  The reduction index n is handed to the lanes in runs of 8
// consecutive pixels (lane l takes n0 + 8 (l / 32) + i), the same for both
// operands, so every product pairs equal n.  Output tile layout of the
// 32 x 32 MFMA: register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.  Partials are FP32 per block; gram_mfma_reduce sums them in
// FP64 in a fixed order.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));

template <int NRG>
struct GramTiles {
  static constexpr int NTRI = NRG * (NRG + 1) / 2;
  static constexpr int TPW = (NTRI + 3) / 4;
  // tile index -> (ti, tj), ti <= tj, row-major over the upper triangle
  static __device__ __forceinline__ void ij(int t, int& ti, int& tj) {
    ti = 0;
    while (t >= NRG - ti) { t -= NRG - ti; ++ti; }
    tj = ti + t;
  }
};

// One 16-byte chunk (8 bf16 / 4 float) of row `a` of Z starting at element n,
// zero past N or past row 2 ell.  N is a multiple of the chunk length here.
template <class S>
__device__ __forceinline__ uint4 gram_chunk(const S* __restrict__ omega, const S* __restrict__ Y,
                                            int64_t N, int ell, int a, int64_t n) {
  if (a >= 2 * ell || n >= N) return make_uint4(0, 0, 0, 0);
  const S* row = a < ell ? omega + static_cast<size_t>(a) * N : Y + static_cast<size_t>(a - ell) * N;
  return *reinterpret_cast<const uint4*>(row + n);
}

// Stage = 128 bytes of every row of Z (64 bf16 or 32 float pixels), staged
// through LDS so that global loads are 128-byte runs of one row (8 lanes per
// row) instead of 32 rows per instruction; the row pitch is padded by 16 B.
template <class S, int NRG>
__device__ __forceinline__ void gram_mfma_body(const S* __restrict__ omega,
                                               const S* __restrict__ Y, int64_t N, int ell,
                                               int64_t n0, int64_t n1, float* __restrict__ dst) {
  using Tl = GramTiles<NRG>;
  constexpr int ROWS = 32 * NRG;
  constexpr int EPC = 16 / sizeof(S);      // elements per 16-byte chunk
  constexpr int KT = 8 * EPC;              // pixels per stage
  constexpr int PITCH = 144;               // bytes per LDS row
  __shared__ __align__(16) unsigned char lds[ROWS * PITCH];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 31, lh = lane >> 5;
  // loader mapping: thread t handles chunk (row 32 g + t / 8, column t % 8)
  const int ld_row = tid >> 3, ld_col = tid & 7;
  floatx16_t acc[Tl::TPW];
#pragma unroll
  for (int t = 0; t < Tl::TPW; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  uint4 pre[NRG];
#pragma unroll
  for (int g = 0; g < NRG; ++g)
    pre[g] = gram_chunk<S>(omega, Y, N, ell, 32 * g + ld_row, n0 + ld_col * EPC);
  for (int64_t n = n0; n < n1; n += KT) {
#pragma unroll
    for (int g = 0; g < NRG; ++g)
      *reinterpret_cast<uint4*>(lds + (32 * g + ld_row) * PITCH + ld_col * 16) = pre[g];
    __syncthreads();
    if (n + KT < n1) {
#pragma unroll
      for (int g = 0; g < NRG; ++g)
        pre[g] = gram_chunk<S>(omega, Y, N, ell, 32 * g + ld_row, n + KT + ld_col * EPC);
    }
    if constexpr (sizeof(S) == 2) {
      // 4 MFMA steps of 16 pixels; lane l supplies pixels 16 kk + 8 (l / 32) + 0..7
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        bf16x8_t fr[NRG];
#pragma unroll
        for (int g = 0; g < NRG; ++g) {
          uint4 u = *reinterpret_cast<const uint4*>(lds + (32 * g + lr) * PITCH + 32 * kk + 16 * lh);
          __builtin_memcpy(&fr[g], &u, 16);
        }
        int tile = 0;
#pragma unroll
        for (int ti = 0; ti < NRG; ++ti)
#pragma unroll
          for (int tj = ti; tj < NRG; ++tj, ++tile)
            if ((tile & 3) == wave)
              acc[tile >> 2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fr[ti], fr[tj], acc[tile >> 2], 0, 0, 0);
      }
    } else {
      // 2 sub-steps of 16 pixels; lane l holds pixels 16 sb + 8 (l / 32) + 0..7
      // and feeds element i to the i-th 32x32x2 MFMA
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) {
        float fr[NRG][8];
#pragma unroll
        for (int g = 0; g < NRG; ++g) {
          const unsigned char* src = lds + (32 * g + lr) * PITCH + 64 * sb + 32 * lh;
          float4 u = *reinterpret_cast<const float4*>(src);
          float4 v = *reinterpret_cast<const float4*>(src + 16);
          fr[g][0] = u.x; fr[g][1] = u.y; fr[g][2] = u.z; fr[g][3] = u.w;
          fr[g][4] = v.x; fr[g][5] = v.y; fr[g][6] = v.z; fr[g][7] = v.w;
        }
        int tile = 0;
#pragma unroll
        for (int ti = 0; ti < NRG; ++ti)
#pragma unroll
          for (int tj = ti; tj < NRG; ++tj, ++tile)
            if ((tile & 3) == wave) {
#pragma unroll
              for (int i = 0; i < 8; ++i)
                acc[tile >> 2] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[ti][i], fr[tj][i], acc[tile >> 2], 0, 0, 0);
            }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < Tl::TPW; ++t) {
    const int tile = wave + 4 * t;
    if (tile < Tl::NTRI) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * lh + (r & 3);
        dst[tile * 1024 + row * 32 + lr] = acc[t][r];
      }
    }
  }
}

template <class S, int NRG>
__global__ __launch_bounds__(256) void gram_mfma_kernel(const S* __restrict__ omega,
                                                        const S* __restrict__ Y, int64_t N,
                                                        int ell, int64_t chunk,
                                                        float* __restrict__ part) {
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  gram_mfma_body<S, NRG>(omega, Y, N, ell, n0, n1,
                         part + static_cast<size_t>(blockIdx.x) * GramTiles<NRG>::NTRI * 1024);
}

template <int NRG>
__device__ __forceinline__ void gram_mfma_reduce_body(const float* __restrict__ part, int nblk,
                                                 int ell, double* __restrict__ G, int e0,
                                                 int estride) {
  using Tl = GramTiles<NRG>;
  const int m = 2 * ell;
  const int total = Tl::NTRI * 1024;
  for (int e = e0; e < total; e += estride) {
    const int tile = e >> 10, r = e & 1023;
    int ti, tj;
    Tl::ij(tile, ti, tj);
    const int gi = 32 * ti + (r >> 5), gj = 32 * tj + (r & 31);
    if (gi >= m || gj >= m) continue;
    double acc8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int b = 0;
    for (; b + 8 <= nblk; b += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        acc8[u] += static_cast<double>(part[static_cast<size_t>(b + u) * total + e]);
    for (; b < nblk; ++b) acc8[0] += static_cast<double>(part[static_cast<size_t>(b) * total + e]);
    const double sacc = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) +
                        ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
    G[gi * m + gj] = sacc;
    G[gj * m + gi] = sacc;
  }
}

template <int NRG>
__global__ __launch_bounds__(256) void gram_mfma_reduce(const float* __restrict__ part, int nblk,
                                                        int ell, double* __restrict__ G) {
  gram_mfma_reduce_body<NRG>(part, nblk, ell, G, blockIdx.x * blockDim.x + threadIdx.x,
                        gridDim.x * blockDim.x);
}

template <class S, int NRG>
static nys_status gram_mfma_launch(const S* omega, const S* Y, int64_t N, int ell, float* part,
                                   int nblk, int64_t chunk, double* G, hipStream_t st) {
  hipLaunchKernelGGL((gram_mfma_kernel<S, NRG>), dim3(nblk), dim3(256), 0, st, omega, Y, N, ell,
                     chunk, part);
  NYS_TRY(launch_check("gram_mfma_kernel"));
  hipLaunchKernelGGL((gram_mfma_reduce<NRG>), dim3(cdiv(GramTiles<NRG>::NTRI * 1024, 256)),
                     dim3(256), 0, st, part, nblk, ell, G);
  return launch_check("gram_mfma_reduce");
}

template <class S>
static nys_status gram_mfma(const S* omega, const S* Y, int64_t N, int ell, float* part, int nblk,
                            int64_t chunk, double* G, hipStream_t st) {
  switch ((2 * ell + 31) / 32) {
    case 1: return gram_mfma_launch<S, 1>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 2: return gram_mfma_launch<S, 2>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 3: return gram_mfma_launch<S, 3>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 4: return gram_mfma_launch<S, 4>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 5: return gram_mfma_launch<S, 5>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 6: return gram_mfma_launch<S, 6>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 7: return gram_mfma_launch<S, 7>(omega, Y, N, ell, part, nblk, chunk, G, st);
    case 8: return gram_mfma_launch<S, 8>(omega, Y, N, ell, part, nblk, chunk, G, st);
    default: break;
  }
  set_error("gram: ell out of range");
  return NYS_EINVAL;
}

// ================================================================ FP64 factor
// One workgroup of kFT threads.  The matrix being worked on (L x L FP64)
// lives in LDS (dynamic shared memory); the eigenvector matrix V, the
// Cholesky factor copy and the triangular-solve outputs live in the global
// work buffer.  G is the 2L x 2L Gram: OO = G[0:L, 0:L], OY = G[0:L, L:2L],
// YY = G[L:2L, L:2L].
constexpr int kFT = 512;

struct FactorWork {
  double *Cg, *X, *Mg, *V, *R, *ev;
};

// Cyclic Jacobi for a symmetric L x L matrix M (full storage) with the
// round-robin ordering: each round rotates L/2 disjoint index pairs, and
// M <- J^T M J is applied as independent 2 x 2 block updates (one barrier per
// round).  Accumulates V <- V J when V != nullptr.  On exit ev = diag(M).
__device__ int jacobi_sym(double* M, double* V, int L, double* ev, int max_sweeps) {
  __shared__ double rc[64], rs[64];
  __shared__ int rp[64], rq[64];
  __shared__ int nrot;
  __shared__ double dmax;
  int sweeps = 0;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = (L + 1) & ~1;      // slot L (odd L) is a dummy
  const int np = m / 2;
  if (V)
    for (int e = tid; e < L * L; e += nt) V[e] = (e / L == e % L) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) {
      nrot = 0;
      double d = 0;
      for (int i = 0; i < L; ++i) d = fmax(d, fabs(M[i * L + i]));
      dmax = d;
    }
    __syncthreads();
    sweeps = sweep + 1;
    for (int r = 0; r < m - 1; ++r) {
      // rotation of pair p; an off-diagonal entry below
      // max(1e-15 sqrt(|a_ii a_jj|), 1e-17 max_k |a_kk|) is set to zero instead
      // (the floor sits above the rounding left by the two-sided updates); the
      // sweep loop ends after a sweep without rotations
      for (int p = tid; p < np; p += nt) {
        int a = (p == 0) ? 0 : ((p - 1 + r) % (m - 1)) + 1;
        int b = ((m - 2 - p + r) % (m - 1)) + 1;
        int i = a < b ? a : b, j = a < b ? b : a;
        double c = 1.0, sn = 0.0;
        if (j < L) {
          const double apq = M[i * L + j];
          const double app = M[i * L + i], aqq = M[j * L + j];
          if (fabs(apq) > fmax(1e-15 * sqrt(fabs(app) * fabs(aqq)), 1e-17 * dmax)) {
            double tau = (aqq - app) / (2.0 * apq);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            atomicAdd(&nrot, 1);
          } else if (apq != 0.0) {
            M[i * L + j] = 0.0;
            M[j * L + i] = 0.0;
          }
        }
        rc[p] = c; rs[p] = sn; rp[p] = i; rq[p] = j;
      }
      __syncthreads();
      // ordered block (P, Q): rows {i1, j1} x cols {i2, j2}; B' = R_P^T B R_Q
      for (int e = tid; e < np * np; e += nt) {
        const int P = e / np, Q = e - P * np;
        const double c1 = rc[P], s1 = rs[P], c2 = rc[Q], s2 = rs[Q];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int i1 = rp[P], j1 = rq[P], i2 = rp[Q], j2 = rq[Q];
        const bool r1 = j1 < L, r2 = j2 < L;
        double b00 = M[i1 * L + i2];
        double b01 = r2 ? M[i1 * L + j2] : 0.0;
        double b10 = r1 ? M[j1 * L + i2] : 0.0;
        double b11 = (r1 && r2) ? M[j1 * L + j2] : 0.0;
        // left: rows
        double t00 = c1 * b00 - s1 * b10, t01 = c1 * b01 - s1 * b11;
        double t10 = s1 * b00 + c1 * b10, t11 = s1 * b01 + c1 * b11;
        // right: columns
        double u00 = c2 * t00 - s2 * t01, u01 = s2 * t00 + c2 * t01;
        double u10 = c2 * t10 - s2 * t11, u11 = s2 * t10 + c2 * t11;
        if (P == Q) { u01 = 0.0; u10 = 0.0; }   // the rotation annihilates the pair
        M[i1 * L + i2] = u00;
        if (r2) M[i1 * L + j2] = u01;
        if (r1) M[j1 * L + i2] = u10;
        if (r1 && r2) M[j1 * L + j2] = u11;
      }
      if (V) {
        for (int e = tid; e < np * L; e += nt) {
          const int row = e / np, P = e - row * np;   // consecutive threads: one row
          const int i = rp[P], j = rq[P];
          if (j >= L || rs[P] == 0.0) continue;
          const double c = rc[P], sn = rs[P];
          double vi = V[row * L + i], vj = V[row * L + j];
          V[row * L + i] = c * vi - sn * vj;
          V[row * L + j] = sn * vi + c * vj;
        }
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  for (int e = tid; e < L; e += nt) ev[e] = M[e * L + e];
  __syncthreads();
  return sweeps;
}

__device__ void factor_body(const double* __restrict__ G, int L, int64_t N, int nu_mode,
                            int tail, double mu_in, int max_esc, FactorWork w, int nlds,
                            double* __restrict__ meta) {
  // L x L matrices: the working matrix S, the Cholesky factor C, the
  // eigenvectors V and the solve output X; the first `nlds` of them live in
  // dynamic LDS, the rest in the global work buffer.
  extern __shared__ double lds_mat[];
  __shared__ double sh_nu, ev_s[PcMeta::kMaxEll];
  __shared__ int sh_fail;
  __shared__ int order[PcMeta::kMaxEll];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = 2 * L;
  const size_t LL = static_cast<size_t>(L) * L;
  double* S = nlds >= 1 ? lds_mat : w.Mg;
  double* Cm = nlds >= 2 ? lds_mat + LL : w.Cg;
  double* Vm = nlds >= 3 ? lds_mat + 2 * LL : w.V;
  double* Xm = nlds >= 4 ? lds_mat + 3 * LL : w.X;
  const double eps = 2.220446049250313e-16;
  if (tid == 0) meta[PcMeta::kScalars + 8 + 7] = static_cast<double>(wall_clock64());
  // ---- shift nu
  if (nu_mode == 0) {
    for (int e = tid; e < L * L; e += nt) S[e] = G[(L + e / L) * m + L + e % L];
    __syncthreads();
    const int sw = jacobi_sym(S, nullptr, L, ev_s, 40);
    if (tid == 0) meta[PcMeta::kSweeps0] = sw;
    if (tid == 0) {
      double mx = 0;
      for (int i = 0; i < L; ++i) mx = fmax(mx, ev_s[i]);
      sh_nu = sqrt(static_cast<double>(N)) * eps * sqrt(fmax(mx, 0.0));
    }
  } else if (tid == 0) {
    double tr = 0;
    for (int i = 0; i < L; ++i) tr += G[i * m + i];
    sh_nu = eps * sqrt(tr);
  }
  __syncthreads();
  double nu = sh_nu;
  if (tid == 0) meta[PcMeta::kScalars + 9] = static_cast<double>(wall_clock64());
  // ---- shifted Cholesky (right-looking, in place in S) with escalation
  int esc = 0;
  for (;; ++esc) {
    for (int e = tid; e < L * L; e += nt) {
      int i = e / L, j = e - i * L;
      double oy = 0.5 * (G[i * m + L + j] + G[j * m + L + i]);
      double oo = 0.5 * (G[i * m + j] + G[j * m + i]);
      S[e] = oy + nu * oo;
    }
    if (tid == 0) sh_fail = 0;
    __syncthreads();
    for (int j = 0; j < L; ++j) {
      if (tid == 0) {
        double d = S[j * L + j];
        if (!(d > 0.0) || !isfinite(d)) { sh_fail = 1; d = 1.0; }
        S[j * L + j] = sqrt(d);
      }
      __syncthreads();
      if (sh_fail) break;
      const double djj = S[j * L + j];
      for (int i = j + 1 + tid; i < L; i += nt) S[i * L + j] /= djj;
      __syncthreads();
      const int rem = L - j - 1;
      for (int e = tid; e < rem * rem; e += nt) {
        int i = j + 1 + e / rem, k = j + 1 + e % rem;
        if (k <= i) S[i * L + k] -= S[i * L + j] * S[k * L + j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (!sh_fail) break;
    if (esc >= max_esc) break;
    nu *= 10.0;
    __syncthreads();
  }
  if (sh_fail) {
    if (tid == 0) {
      meta[PcMeta::kStatus] = NYS_ENOTPD;
      meta[PcMeta::kNu] = nu;
      meta[PcMeta::kKeff] = 0;
      meta[PcMeta::kEscal] = esc;
      for (int i = 0; i < L; ++i) { meta[PcMeta::kShat + i] = 0; meta[PcMeta::kD + i] = 0; meta[PcMeta::kE + i] = 0; }
    }
    for (int e = tid; e < L * L; e += nt) w.R[e] = 0.0;
    return;
  }
  if (tid == 0) meta[PcMeta::kScalars + 10] = static_cast<double>(wall_clock64());
  // lower factor C (the upper part of S is stale)
  for (int e = tid; e < L * L; e += nt) {
    int i = e / L, j = e - i * L;
    Cm[e] = j <= i ? S[e] : 0.0;
  }
  __syncthreads();
  // ---- X = C^{-1} Mv with Mv = Y_nu^T Y_nu = YY + nu (OY + OY^T) + nu^2 OO,
  // one right-hand side column per thread
  for (int j = tid; j < L; j += nt)
    for (int i = 0; i < L; ++i) {
      double sacc = G[(L + i) * m + L + j] + nu * (G[i * m + L + j] + G[j * m + L + i]) +
                    nu * nu * G[i * m + j];
      for (int k = 0; k < i; ++k) sacc -= Cm[i * L + k] * Xm[k * L + j];
      Xm[i * L + j] = sacc / Cm[i * L + i];
    }
  __syncthreads();
  if (tid == 0) meta[PcMeta::kScalars + 11] = static_cast<double>(wall_clock64());
  // ---- M = C^{-1} X^T, into S
  for (int j = tid; j < L; j += nt)
    for (int i = 0; i < L; ++i) {
      double sacc = Xm[j * L + i];
      for (int k = 0; k < i; ++k) sacc -= Cm[i * L + k] * S[k * L + j];
      S[i * L + j] = sacc / Cm[i * L + i];
    }
  __syncthreads();
  for (int e = tid; e < L * L; e += nt) {
    int i = e / L, j = e - i * L;
    if (i < j) {
      double a = 0.5 * (S[i * L + j] + S[j * L + i]);
      S[i * L + j] = a;
      S[j * L + i] = a;
    }
  }
  __syncthreads();
  if (tid == 0) meta[PcMeta::kScalars + 12] = static_cast<double>(wall_clock64());
  // ---- eigen-decomposition M = V diag(S^2) V^T, descending order
  {
    const int sw = jacobi_sym(S, Vm, L, ev_s, 60);
    if (tid == 0) meta[PcMeta::kSweeps1] = sw;
  }
  if (tid == 0) {
    for (int i = 0; i < L; ++i) order[i] = i;
    for (int i = 0; i < L; ++i) {           // selection sort, descending
      int best = i;
      for (int k = i + 1; k < L; ++k)
        if (ev_s[order[k]] > ev_s[order[best]]) best = k;
      int t = order[i]; order[i] = order[best]; order[best] = t;
    }
  }
  __syncthreads();
  if (tid == 0) meta[PcMeta::kScalars + 13] = static_cast<double>(wall_clock64());
  // ---- R = C^{-T} V S^{-1} (column k per thread, back substitution)
  for (int k = tid; k < L; k += nt) {
    const int src = order[k];
    const double s2 = ev_s[src];
    const double inv = s2 > 0 ? 1.0 / sqrt(s2) : 0.0;
    for (int i = L - 1; i >= 0; --i) {
      double sacc = Vm[i * L + src];
      for (int q = i + 1; q < L; ++q) sacc -= Cm[q * L + i] * w.R[q * L + k];
      w.R[i * L + k] = sacc / Cm[i * L + i];
    }
    for (int i = 0; i < L; ++i) w.R[i * L + k] *= inv;
  }
  __syncthreads();
  if (tid == 0) meta[PcMeta::kScalars + 14] = static_cast<double>(wall_clock64());
  // ---- spectrum and preconditioner coefficients
  if (tid == 0) {
    int keff = 0;
    for (int k = 0; k < L; ++k) {
      double sh = fmax(0.0, ev_s[order[k]] - nu);
      meta[PcMeta::kShat + k] = sh;
      if (sh > 0) keff = k + 1;
    }
    double sK = keff > 0 ? meta[PcMeta::kShat + keff - 1] : 0.0;
    double st = tail == 0 ? sqrt(sK) : sK;
    double mu = mu_in < 0 ? nu : mu_in;
    double pn = 1.0;
    for (int k = 0; k < L; ++k) {
      double sh = meta[PcMeta::kShat + k];
      if (k < keff && sh > 0) {
        meta[PcMeta::kD + k] = (st + mu) / (sh + mu) - 1.0;
        meta[PcMeta::kE + k] = (sh + mu) / (st + mu) - 1.0;
        pn = fmax(pn, (st + mu) / (sh + mu));
      } else {
        meta[PcMeta::kD + k] = 0.0;
        meta[PcMeta::kE + k] = 0.0;
      }
    }
    meta[PcMeta::kNu] = nu;
    meta[PcMeta::kSK] = st;
    meta[PcMeta::kMu] = mu;
    meta[PcMeta::kPinvNorm] = pn;
    meta[PcMeta::kKeff] = keff;
    meta[PcMeta::kEscal] = esc;
    bool finite = isfinite(nu) && isfinite(pn);
    meta[PcMeta::kStatus] = finite ? NYS_OK : NYS_ENOTFINITE;
  }
}

__global__ __launch_bounds__(kFT) void factor_kernel(const double* __restrict__ G, int L,
                                                     int64_t N, int nu_mode, int tail,
                                                     double mu_in, int max_esc, FactorWork w,
                                                     int nlds, double* __restrict__ meta) {
  factor_body(G, L, N, nu_mode, tail, mu_in, max_esc, w, nlds, meta);
}

static __host__ __device__ FactorWork factor_work(double* wb, int L) {
  const size_t LL = static_cast<size_t>(L) * L;
  FactorWork w;
  w.Cg = wb; w.X = wb + LL; w.Mg = wb + 2 * LL; w.V = wb + 3 * LL; w.R = wb + 4 * LL;
  w.ev = wb + 5 * LL;
  return w;
}

// L x L matrices that fit in `lds_doubles` of dynamic LDS (at most 4)
static __host__ __device__ int factor_nlds(int L, size_t lds_doubles) {
  const size_t LL = static_cast<size_t>(L) * L;
  const size_t k = lds_doubles / LL;
  return static_cast<int>(k < 4 ? k : 4);
}

// Batched: one workgroup per instance (blockIdx.x = segment).
__global__ __launch_bounds__(kFT) void bfactor_kernel(const BDesc* __restrict__ d,
                                                      const BSeg* __restrict__ seg, int nu_mode,
                                                      int tail, double mu_in, int max_esc,
                                                      int64_t lds_doubles) {
  const BDesc& D = d[seg[blockIdx.x].inst];
  factor_body(D.G, D.ell, D.N, nu_mode, tail, mu_in, max_esc, factor_work(D.fwork, D.ell),
              factor_nlds(D.ell, static_cast<size_t>(lds_doubles)), D.meta);
}

// ================================================================ U
// U[k][n] = sum_j (Y[j][n] + nu Omega[j][n]) R[j][k]; KC outputs per thread.
// The sum runs in FP64 for every storage type: R = C^{-T} V S^{-1} has entries
// up to 1 / S_min, so an FP32 sum of its products cancels by cond(B) (at
// cond(B) ~ 1e3 the FP32 sum moved P^{-1} by 3e-5); FP64 FMAs cost the same
// issue rate as non-packed FP32 ones on this device.
constexpr int kUK = 32;

template <class S, class T, class C>
__device__ __forceinline__ void form_u_body(const S* __restrict__ omega, const S* __restrict__ Y,
                                            const double* __restrict__ R,
                                            const double* __restrict__ meta, int64_t N, int L,
                                            int64_t ldu, T* __restrict__ U, int k0, int64_t n) {
  __shared__ C Rs[PcMeta::kMaxEll][kUK];
  for (int e = threadIdx.x; e < L * kUK; e += blockDim.x) {
    int j = e / kUK, kk = e - j * kUK;
    Rs[j][kk] = (k0 + kk < L) ? static_cast<C>(R[j * L + k0 + kk]) : C(0);
  }
  __syncthreads();
  const C nu = static_cast<C>(meta[PcMeta::kNu]);
  if (n >= N) return;
  C acc[kUK];
#pragma unroll
  for (int kk = 0; kk < kUK; ++kk) acc[kk] = 0;
  for (int j = 0; j < L; ++j) {
    C z = Io<S>::ld(Y, static_cast<size_t>(j) * N + n) + nu * Io<S>::ld(omega, static_cast<size_t>(j) * N + n);
#pragma unroll
    for (int kk = 0; kk < kUK; ++kk) acc[kk] += z * Rs[j][kk];
  }
#pragma unroll
  for (int kk = 0; kk < kUK; ++kk)
    if (k0 + kk < L) U[static_cast<size_t>(k0 + kk) * ldu + n] = static_cast<T>(acc[kk]);
}

template <class S, class T, class C>
__global__ __launch_bounds__(256) void form_u_kernel(const S* __restrict__ omega,
                                                     const S* __restrict__ Y,
                                                     const double* __restrict__ R,
                                                     const double* __restrict__ meta, int64_t N,
                                                     int L, int64_t ldu, T* __restrict__ U) {
  form_u_body<S, T, C>(omega, Y, R, meta, N, L, ldu, U, blockIdx.y * kUK,
                       blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x);
}

// Batched: block -> (instance, 256 pixels), blockIdx.y = group of kUK columns.
// A failed factorisation leaves R = 0 and therefore U = 0.
__global__ __launch_bounds__(256) void bform_u_kernel(const BDesc* __restrict__ d,
                                                      const BSeg* __restrict__ seg, int nseg) {
  const BSeg& sg = seg[seg_find(seg, nseg, blockIdx.x)];
  const BDesc& D = d[sg.inst];
  const int k0 = blockIdx.y * kUK;
  if (k0 >= D.ell) return;
  const int64_t n = (blockIdx.x - sg.first) * 256 + threadIdx.x;
  form_u_body<float, float, double>(D.omega, D.Y, factor_work(D.fwork, D.ell).R, D.meta, D.N,
                                   D.ell, D.ldu, D.U, k0, n);
}

// Launch geometry and scratch of Alg. 1 steps 3-8 for N pixels and L
// columns: the VALU Gram's pixel chunks and 32 x 32 tiles, the MFMA Gram's
// blocks, and the FP64 scratch (Gram partials, the 2L x 2L Gram, the factor's
// L x L matrices).
struct FactorGeom {
  int ntiles, ntri;
  int64_t nchunks, chunk, mfma_blocks, mfma_chunk;
  size_t part_d, G_d, w_d;
  FactorGeom(int64_t N, int L) {
    const int m = 2 * L;
    ntiles = static_cast<int>(cdiv(m, kGT));
    ntri = ntiles * (ntiles + 1) / 2;
    nchunks = std::min<int64_t>(256, std::max<int64_t>(1, N / 4096));
    chunk = (N + nchunks - 1) / nchunks;
    chunk = (chunk + kGK - 1) / kGK * kGK;
    nchunks = (N + chunk - 1) / chunk;
    part_d = static_cast<size_t>(nchunks) * ntri * kGT * kGT;
    // MFMA Gram (BF16): one block per chunk of at least 256 pixels
    mfma_blocks = std::min<int64_t>(256, std::max<int64_t>(1, N / 256));
    mfma_chunk = (N + mfma_blocks - 1) / mfma_blocks;
    mfma_chunk = (mfma_chunk + 63) / 64 * 64;
    mfma_blocks = (N + mfma_chunk - 1) / mfma_chunk;
    const int nrg = (2 * L + 31) / 32;
    const size_t mfma_d = (static_cast<size_t>(mfma_blocks) * nrg * (nrg + 1) / 2 * 1024 + 1) / 2;
    part_d = std::max(part_d, mfma_d);
    G_d = static_cast<size_t>(m) * m;
    w_d = 5 * static_cast<size_t>(L) * L + L;
  }
  size_t bytes() const { return ws_round(sizeof(double) * (part_d + G_d + w_d)); }
};

size_t factor_ws_bytes(int64_t N, int L) { return FactorGeom(N, L).bytes(); }

template <class S>
static nys_status factor_impl(const S* omega, const S* Y, int64_t N, int L,
                              const nys_factor_opts& o, nys_pc pc, hipStream_t st) {
  const FactorGeom g(N, L);
  const int ntiles = g.ntiles, ntri = g.ntri;
  const int64_t nchunks = g.nchunks, chunk = g.chunk, mfma_blocks = g.mfma_blocks,
                mfma_chunk = g.mfma_chunk;
  const size_t part_d = g.part_d, G_d = g.G_d;
  Scratch::Mark mark(pc->scr);
  double* part = nullptr;
  NYS_TAKE(pc->scr, double, part, part_d + G_d + g.w_d);
  double* G = part + part_d;
  double* wb = G + G_d;
  FactorWork w;
  size_t LL = static_cast<size_t>(L) * L;
  w.Cg = wb; w.X = wb + LL; w.Mg = wb + 2 * LL; w.V = wb + 3 * LL; w.R = wb + 4 * LL;
  w.ev = wb + 5 * LL;
  using C = typename Io<S>::C;
  // BF16 columns: MFMA with FP32 accumulation when every column is a whole
  // number of 16-byte chunks.  FP32 and FP64 columns: the VALU tile kernel
  // with FP64 accumulation (products of FP32 values are exact in FP64), since
  // the Gram route squares the condition number of the sketch.
  bool use_mfma = false;
  if constexpr (std::is_same<S, uint16_t>::value) use_mfma = (N % (16 / sizeof(S))) == 0;
  using Acc = typename std::conditional<std::is_same<S, uint16_t>::value, float, double>::type;
  if (!use_mfma) {
    hipLaunchKernelGGL((gram_partial_kernel<S, Acc>), dim3(static_cast<unsigned>(nchunks), ntri),
                       dim3(256), 0, st, omega, Y, N, L, chunk, ntiles, part);
    NYS_TRY(launch_check("gram_partial_kernel"));
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(64), dim3(256), 0, st, part,
                       static_cast<int>(nchunks), ntiles, L, G);
    NYS_TRY(launch_check("gram_reduce_kernel"));
  } else {
    if constexpr (!std::is_same<S, double>::value)
      NYS_TRY(gram_mfma<S>(omega, Y, N, L, reinterpret_cast<float*>(part), mfma_blocks, mfma_chunk,
                           G, st));
  }
  // as many L x L matrices in LDS as the device allows per workgroup
  int dev = 0, maxsh = 0;
  NYS_CHECK_HIP(hipGetDevice(&dev));
  NYS_CHECK_HIP(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const size_t avail = maxsh > 8192 ? static_cast<size_t>(maxsh) - 8192 : 0;
  const int nlds = static_cast<int>(std::min<size_t>(4, avail / (sizeof(double) * LL)));
  const size_t lds = sizeof(double) * LL * nlds;
  if (lds > 64 * 1024) {
    NYS_CHECK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(factor_kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(lds)));
  }
  hipLaunchKernelGGL(factor_kernel, dim3(1), dim3(kFT), lds, st, G, L, N, o.nu_mode, o.tail, o.mu,
                     o.max_escalations < 0 ? 6 : o.max_escalations, w, nlds, pc->meta.as<double>());
  NYS_TRY(launch_check("factor_kernel"));
  dim3 ug(cdiv(N, 256), cdiv(L, kUK));
  if (pc->u_dtype == NYS_F64) {
    hipLaunchKernelGGL((form_u_kernel<S, double, double>), ug, dim3(256), 0, st, omega, Y, w.R,
                       pc->meta.as<double>(), N, L, pc->ldu, pc->U.as<double>());
  } else {
    hipLaunchKernelGGL((form_u_kernel<S, float, double>), ug, dim3(256), 0, st, omega, Y, w.R,
                       pc->meta.as<double>(), N, L, pc->ldu, pc->U.as<float>());
  }
  return launch_check("form_u_kernel");
}

nys_status batch_factor_prepare(int64_t lds_bytes) {
  if (lds_bytes > 64 * 1024)
    NYS_CHECK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(bfactor_kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(lds_bytes)));
  return NYS_OK;
}

nys_status batch_factor_enqueue(const BDesc* d, const BLaunch& gram, const BLaunch& fac,
                                const BLaunch& upix, int kgroups, int max_ell, int64_t lds_doubles,
                                int nu_mode, int tail, double mu, int max_esc, hipStream_t st) {
  const int ntiles = (2 * max_ell + kGT - 1) / kGT;
  const int ntri = ntiles * (ntiles + 1) / 2;
  hipLaunchKernelGGL(bgram_kernel, dim3(static_cast<unsigned>(gram.nblk), ntri), dim3(256), 0, st,
                     d, gram.seg, gram.nseg);
  NYS_TRY(launch_check("bgram_kernel"));
  hipLaunchKernelGGL(bgram_reduce, dim3(cdiv(ntri * kGT * kGT, 256), gram.nseg), dim3(256), 0, st,
                     d, gram.seg);
  NYS_TRY(launch_check("bgram_reduce"));
  hipLaunchKernelGGL(bfactor_kernel, dim3(fac.nseg), dim3(kFT),
                     static_cast<size_t>(lds_doubles) * sizeof(double), st, d, fac.seg, nu_mode,
                     tail, mu, max_esc, lds_doubles);
  NYS_TRY(launch_check("bfactor_kernel"));
  hipLaunchKernelGGL(bform_u_kernel, dim3(static_cast<unsigned>(upix.nblk), kgroups), dim3(256), 0,
                     st, d, upix.seg, upix.nseg);
  return launch_check("bform_u_kernel");
}

// Alg. 1 steps 3-8 again on a handle made by nys_factor for the same N, ell
// and storage type, reusing its buffers (U's padding rows stay zero).
nys_status factor_refresh(nys_pc pc, const void* omega, const void* Y, nys_dtype in_dt,
                          const nys_factor_opts& o, hipStream_t st) {
  pc->pinv_norm_cache = -1.0;
  pc->tail = o.tail;
  pc->ssn_lu_valid = false;
  const int L = static_cast<int>(pc->ell);
  switch (in_dt) {
    case NYS_F64:
      return factor_impl<double>(static_cast<const double*>(omega), static_cast<const double*>(Y),
                                 pc->N, L, o, pc, st);
    case NYS_F32:
      return factor_impl<float>(static_cast<const float*>(omega), static_cast<const float*>(Y),
                                pc->N, L, o, pc, st);
    default:
      set_error("factor_refresh: dtype must be F64 or F32");
      return NYS_EINVAL;
  }
}

// A preconditioner handle for N pixels and ell columns with its own buffers,
// allocated once here: U (padding rows zeroed on the stream), the FP64
// metadata, the semismooth Newton buffer and the pinned decision word.
nys_status pc_create(int64_t N, int64_t ell, const nys_factor_opts& o, nys_pc* out,
                     hipStream_t st) {
  auto* pc = new nys_pc_s();
  pc->N = N;
  pc->ell = ell;
  pc->u_dtype = o.u_dtype;
  pc->tail = o.tail;
  // column pitch: a multiple of 64 elements, plus 96 for large images so the
  // ell columns are not a power of two apart
  pc->ldu = (N + 63) / 64 * 64 + (N >= 16384 ? 96 : 0);
  pc->ell_pad = (ell + 15) / 16 * 16;
  const size_t ues = dtype_size(static_cast<nys_dtype>(o.u_dtype));
  const size_t ucount = static_cast<size_t>(pc->ldu) * pc->ell_pad;
  nys_status s = pc->U.ensure(ues * ucount);
  if (s == NYS_OK) s = pc->meta.ensure(sizeof(double) * PcMeta::kTotal);
  if (s == NYS_OK) s = pc->ssn_ws.ensure(ssn_ws_bytes(N, static_cast<int>(ell), ues));
  if (s == NYS_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(unsigned long long), hipHostMallocCoherent) != hipSuccess) {
      set_error("hipHostMalloc of the decision word failed");
      s = NYS_ENOMEM;
    } else {
      pc->hflag = static_cast<unsigned long long*>(h);
      *pc->hflag = 0;
      pc->flag_seq = 0;
    }
  }
  if (s == NYS_OK)
    s = o.u_dtype == NYS_F64 ? fill_zero<double>(pc->U.as<double>(), ucount, st)
                             : fill_zero<float>(pc->U.as<float>(), ucount, st);
  if (s != NYS_OK) {
    nys_pc_destroy(pc);
    return s;
  }
  *out = pc;
  return NYS_OK;
}

}  // namespace nys

using namespace nys;

extern "C" nys_status nys_factor_workspace_size(int64_t N, int64_t ell, size_t* bytes) {
  NYS_REQUIRE(bytes && N > 0 && ell >= 1 && ell <= PcMeta::kMaxEll,
              "nys_factor_workspace_size: bad argument");
  *bytes = factor_ws_bytes(N, static_cast<int>(ell));
  return NYS_OK;
}

extern "C" nys_status nys_factor(const void* omega, const void* Y, nys_dtype in_dt, int64_t N,
                                 int64_t ell, const nys_factor_opts* opts, void* ws,
                                 size_t ws_bytes, nys_pc* out, void* stream) {
  NYS_REQUIRE(omega && Y && out && N > 0, "nys_factor: bad argument");
  NYS_REQUIRE(ell >= 1 && ell <= PcMeta::kMaxEll, "nys_factor: ell must be in [1, %d]", PcMeta::kMaxEll);
  NYS_REQUIRE(ell <= N, "nys_factor: ell > N");
  NYS_REQUIRE(in_dt == NYS_F64 || in_dt == NYS_F32 || in_dt == NYS_BF16, "nys_factor: bad dtype");
  nys_factor_opts o{0, 0, -1.0, 6, NYS_F32};
  if (opts) o = *opts;
  NYS_REQUIRE(o.u_dtype == NYS_F64 || o.u_dtype == NYS_F32, "nys_factor: u_dtype must be F64/F32");
  NYS_REQUIRE(o.nu_mode == 0 || o.nu_mode == 1, "nys_factor: nu_mode must be 0 or 1");
  NYS_REQUIRE(o.tail == 0 || o.tail == 1, "nys_factor: tail must be 0 or 1");
  NYS_TRY(check_workspace(ws, ws_bytes, factor_ws_bytes(N, static_cast<int>(ell)), "nys_factor"));
  hipStream_t st = as_stream(stream);
  nys_pc pc = nullptr;
  nys_status s = pc_create(N, ell, o, &pc, st);
  if (s != NYS_OK) return s;
  if (s == NYS_OK) {
    WsBind bind(ws, ws_bytes, nullptr, pc);
    switch (in_dt) {
      case NYS_F64:
        s = factor_impl<double>(static_cast<const double*>(omega), static_cast<const double*>(Y), N,
                                static_cast<int>(ell), o, pc, st);
        break;
      case NYS_F32:
        s = factor_impl<float>(static_cast<const float*>(omega), static_cast<const float*>(Y), N,
                               static_cast<int>(ell), o, pc, st);
        break;
      default:
        s = factor_impl<uint16_t>(static_cast<const uint16_t*>(omega),
                                  static_cast<const uint16_t*>(Y), N, static_cast<int>(ell), o, pc, st);
    }
  }
  if (s != NYS_OK) {
    nys_pc_destroy(pc);
    return s;
  }
  *out = pc;
  return NYS_OK;
}

extern "C" void nys_pc_destroy(nys_pc pc) {
  if (!pc) return;
  // the factorisation may still be running on its stream
  (void)hipDeviceSynchronize();
  pc->U.release();
  pc->meta.release();
  pc->ssn_ws.release();
  if (pc->hflag) (void)hipHostFree(pc->hflag);
  delete pc;
}

extern "C" nys_status nys_pc_info(nys_pc pc, double* shat, double* nu, int32_t* k_eff,
                                  int32_t* status, void* stream) {
  NYS_REQUIRE(pc, "nys_pc_info: null pc");
  std::vector<double> meta(PcMeta::kTotal);
  NYS_CHECK_HIP(hipStreamSynchronize(as_stream(stream)));
  NYS_CHECK_HIP(hipMemcpy(meta.data(), pc->meta.p, sizeof(double) * PcMeta::kTotal,
                          hipMemcpyDeviceToHost));
  if (shat)
    for (int k = 0; k < pc->ell; ++k) shat[k] = meta[PcMeta::kShat + k];
  if (nu) *nu = meta[PcMeta::kNu];
  if (k_eff) *k_eff = static_cast<int32_t>(meta[PcMeta::kKeff]);
  if (status) *status = static_cast<int32_t>(meta[PcMeta::kStatus]);
  return NYS_OK;
}

extern "C" nys_status nys_pc_u(nys_pc pc, const void** u, int64_t* N, int64_t* ell,
                               int64_t* ldu, int32_t* u_dtype) {
  NYS_REQUIRE(pc, "nys_pc_u: null pc");
  if (u) *u = pc->U.p;
  if (ldu) *ldu = pc->ldu;
  if (N) *N = pc->N;
  if (ell) *ell = pc->ell;
  if (u_dtype) *u_dtype = pc->u_dtype;
  return NYS_OK;
}

extern "C" nys_status nys_pc_copy_u(nys_pc pc, void* dst, void* stream) {
  NYS_REQUIRE(pc && dst, "nys_pc_copy_u: bad argument");
  const size_t es = dtype_size(static_cast<nys_dtype>(pc->u_dtype));
  NYS_CHECK_HIP(hipMemcpy2DAsync(dst, es * pc->N, pc->U.p, es * pc->ldu, es * pc->N, pc->ell,
                                 hipMemcpyDeviceToDevice, as_stream(stream)));
  return NYS_OK;
}

extern "C" nys_status nys_apply_workspace_size(nys_pc pc, int64_t ncols, size_t* bytes) {
  NYS_REQUIRE(pc && bytes && ncols > 0, "nys_apply_workspace_size: bad argument");
  *bytes = pc_ws_bytes(pc, ncols);
  return NYS_OK;
}

extern "C" nys_status nys_apply(nys_pc pc, int32_t inverse, nys_dtype dt, const void* v, void* out,
                                int64_t ncols, void* ws, size_t ws_bytes, void* stream) {
  NYS_REQUIRE(pc && v && out && ncols > 0 && ncols <= 65535, "nys_apply: bad argument");
  NYS_REQUIRE(static_cast<int32_t>(dt) == pc->u_dtype, "nys_apply: dtype must equal the pc's u_dtype");
  NYS_TRY(check_workspace(ws, ws_bytes, pc_ws_bytes(pc, ncols), "nys_apply"));
  WsBind bind(ws, ws_bytes, nullptr, pc);
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return pc_apply<double>(pc, inverse != 0, static_cast<const double*>(v), static_cast<double*>(out),
                            ncols, st);
  return pc_apply<float>(pc, inverse != 0, static_cast<const float*>(v), static_cast<float*>(out),
                         ncols, st);
}

// ---------------------------------------------------------------- P-norm
// (a - b)^T P (a - b): the difference, P (or P^{-1}) applied to it by the
// regular two-pass application, then an FP64 dot product (block partials and
// one summing block).
template <class T>
__global__ __launch_bounds__(256) void pdiff_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                    T* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    d[i] = b ? static_cast<T>(a[i] - b[i]) : a[i];
}

__device__ __forceinline__ double block_sum_256(double s) {
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

template <class T>
__global__ __launch_bounds__(256) void pdot_partial_kernel(const T* __restrict__ d,
                                                           const T* __restrict__ w, int64_t n,
                                                           double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s += static_cast<double>(d[i]) * static_cast<double>(w[i]);
  s = block_sum_256(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// P = I: block sums of (a - b)^2 (b may be null).
template <class T>
__global__ __launch_bounds__(256) void pdot_plain_kernel(const T* __restrict__ a,
                                                         const T* __restrict__ b, int64_t n,
                                                         double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double di = static_cast<double>(a[i]) - (b ? static_cast<double>(b[i]) : 0.0);
    s += di * di;
  }
  s = block_sum_256(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void pdot_final_kernel(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum_256(s);
  if (threadIdx.x == 0) out[0] = s;
}

constexpr int kPnParts = 1024;

// Workspace of nys_pnorm2: the difference and P (or P^{-1}) times it, the
// dot product's block partials, the application's scratch.
static size_t pnorm2_ws_bytes(nys_pc pc, int64_t n, size_t es) {
  if (!pc) return ws_round(sizeof(double) * kPnParts);
  return 2 * ws_round(es * static_cast<size_t>(n)) + ws_round(sizeof(double) * kPnParts) +
         pc_ws_bytes(pc, 1);
}

template <class T>
static nys_status pnorm2_impl(nys_pc pc, Scratch* scr, int64_t n, bool inverse, const T* a,
                              const T* b, double* out, hipStream_t st) {
  double* part = nullptr;
  NYS_TAKE(scr, double, part, kPnParts);
  const unsigned nb = std::min<unsigned>(cdiv(n, 256), kPnParts);
  if (!pc) {
    hipLaunchKernelGGL((pdot_plain_kernel<T>), dim3(nb), dim3(256), 0, st, a, b, n, part);
    NYS_TRY(launch_check("pdot_plain_kernel"));
  } else {
    T* d = nullptr;
    T* w = nullptr;
    NYS_TAKE(scr, T, d, n);
    NYS_TAKE(scr, T, w, n);
    hipLaunchKernelGGL((pdiff_kernel<T>), dim3(std::min<unsigned>(cdiv(n, 256), 4096)), dim3(256), 0,
                       st, a, b, d, n);
    NYS_TRY(launch_check("pdiff_kernel"));
    NYS_TRY(pc_apply<T>(pc, inverse, d, w, 1, st));
    hipLaunchKernelGGL((pdot_partial_kernel<T>), dim3(nb), dim3(256), 0, st, d, w, n, part);
    NYS_TRY(launch_check("pdot_partial_kernel"));
  }
  hipLaunchKernelGGL(pdot_final_kernel, dim3(1), dim3(256), 0, st, part, static_cast<int>(nb), out);
  return launch_check("pdot_final_kernel");
}

extern "C" nys_status nys_pnorm2_workspace_size(nys_pc pc, int64_t n, nys_dtype dt, size_t* bytes) {
  NYS_REQUIRE(bytes && n > 0 && (dt == NYS_F64 || dt == NYS_F32),
              "nys_pnorm2_workspace_size: bad argument");
  *bytes = pnorm2_ws_bytes(pc, n, dtype_size(dt));
  return NYS_OK;
}

extern "C" nys_status nys_pnorm2(nys_pc pc, int64_t n, int32_t inverse, nys_dtype dt,
                                 const void* a, const void* b, double* out, void* ws,
                                 size_t ws_bytes, void* stream) {
  NYS_REQUIRE(a && out && n > 0, "nys_pnorm2: bad argument");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "nys_pnorm2: dtype must be F64 or F32");
  if (pc) {
    NYS_REQUIRE(n == pc->N, "nys_pnorm2: n must equal the pc's N");
    NYS_REQUIRE(static_cast<int32_t>(dt) == pc->u_dtype,
                "nys_pnorm2: dtype must equal the pc's u_dtype");
  }
  NYS_TRY(check_workspace(ws, ws_bytes, pnorm2_ws_bytes(pc, n, dtype_size(dt)), "nys_pnorm2"));
  WsBind bind(ws, ws_bytes, nullptr, pc);
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return pnorm2_impl<double>(pc, &bind.s, n, inverse != 0, static_cast<const double*>(a),
                               static_cast<const double*>(b), out, st);
  return pnorm2_impl<float>(pc, &bind.s, n, inverse != 0, static_cast<const float*>(a),
                            static_cast<const float*>(b), out, st);
}

extern "C" nys_status nys_pc_diag(nys_pc pc, double* out, int32_t n, void* stream) {
  NYS_REQUIRE(pc && out && n > 0, "nys_pc_diag: bad argument");
  std::vector<double> meta(PcMeta::kTotal);
  NYS_CHECK_HIP(hipStreamSynchronize(as_stream(stream)));
  NYS_CHECK_HIP(hipMemcpy(meta.data(), pc->meta.p, sizeof(double) * PcMeta::kTotal,
                          hipMemcpyDeviceToHost));
  for (int i = 0; i < n && i < 16; ++i) out[i] = meta[PcMeta::kScalars + i];
  return NYS_OK;
}
