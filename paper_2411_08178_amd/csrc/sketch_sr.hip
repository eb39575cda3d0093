// Fused sketch for the wavelet-reparametrised blur + 2x decimation operator:
//   Y = W H^T S^T S H W^T Omega        (Alg. 1 step 2 with the Phi of the
//                                        invertible-L reparametrisation)
// One workgroup produces a 64 x 64 tile of coefficients of one column.  It
// reads the tile plus an 8-pixel halo (whole 8 x 8 Haar blocks) once from
// HBM and keeps every intermediate in LDS: Haar synthesis, blur sampled on
// the decimated grid, zero-filled upsampling + correlation, Haar analysis.
// PSF size <= 9 (two half-widths fit in the 8-pixel halo).
//
// Two kernels:
//  - sketch_sr_sep_kernel: rank-1 PSF (psf = u v^T, e.g. Gaussian).  Loads are
//    16-byte vectors of whole Haar block rows, Haar levels run in registers,
//    the blur is two 1-D passes evaluated only where S keeps samples, and the
//    polyphase up-correlation is fused with the Haar analysis and the store.
//  - sketch_sr_kernel: any PSF, 2-D taps (general fallback).

#include <hip/hip_bf16.h>

#include "common.hpp"
#include "internal.hpp"

namespace nys {

namespace {
constexpr int kT = 64;             // output tile (coefficients)
constexpr int kH = 8;              // halo = one Haar block
constexpr int kR = kT + 2 * kH;    // 80: input region side
constexpr int kRP = kR + 1;        // padded LDS row (general kernel)
constexpr int kZ = kT / 2 + 6;     // low-resolution region side bound (k <= 9)
constexpr int kZP = kZ + 1;
}  // namespace

// ------------------------------------------------------------------ helpers
// 3-level 2-D orthonormal Haar butterflies on an 8 x 8 register block, in the
// in-place layout.  Synthesis runs the coarsest level first, analysis the
// finest first; the 2 x 2 butterfly is its own inverse.
template <bool kAnalysis>
__device__ __forceinline__ void haar8_regs(float (&v)[8][8]) {
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    const int s = kAnalysis ? (1 << it) : (4 >> it);
#pragma unroll
    for (int r = 0; r < 8; r += 2 * s)
#pragma unroll
      for (int q = 0; q < 8; q += 2 * s) {
        float a = v[r][q], b = v[r][q + s], c = v[r + s][q], d = v[r + s][q + s];
        v[r][q] = 0.5f * (a + b + c + d);
        v[r][q + s] = 0.5f * (a - b + c - d);
        v[r + s][q] = 0.5f * (a + b - c - d);
        v[r + s][q + s] = 0.5f * (a - b - c + d);
      }
  }
}

// Load / store 8 consecutive elements as 16-byte vectors.
__device__ __forceinline__ void ld_row8(const uint16_t* p, float (&o)[8]) {
  uint4 u = *reinterpret_cast<const uint4*>(p);
  uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __uint_as_float(w[i] << 16);
    o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}
__device__ __forceinline__ void ld_row8(const float* p, float (&o)[8]) {
  float4 a = *reinterpret_cast<const float4*>(p);
  float4 b = *reinterpret_cast<const float4*>(p + 4);
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
  o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}
// two floats -> packed bfloat16 pair, round to nearest even (hardware convert)
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  __hip_bfloat162 h = __float22bfloat162_rn(make_float2(a, b));
  uint32_t u;
  __builtin_memcpy(&u, &h, 4);
  return u;
}
__device__ __forceinline__ void st_row8(uint16_t* p, const float (&v)[8]) {
  *reinterpret_cast<uint4*>(p) = make_uint4(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]),
                                            pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7]));
}
__device__ __forceinline__ void st_row8(float* p, const float (&v)[8]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}

// 1-D factors of a rank-1 PSF: h[a][b] = hu[a] hv[b]; g* are the flips.
struct SepPsf {
  float gu[9], gv[9], hu[9], hv[9];
};

// Tile geometry for PSF size K (compile time).  Decimated samples needed by
// a tile starting at even P0: indices P0/2 + QA .. P0/2 + QB; the HR rows
// they read start at region row TR0 (region = tile - 8).  Every LDS index
// below stays inside the buffers for K in {1, 3, 5, 7, 9}; outputs past NQ
// that the grouped passes compute are padding and never read.
template <int K>
struct SrGeom {
  static constexpr int C = (K - 1) / 2;
  static constexpr int QA = -(C / 2);
  static constexpr int QB = (63 + C) / 2;
  static constexpr int NQ = QB - QA + 1;        // <= 36
  static constexpr int TR0 = 2 * QA - C + 8;    // >= 0
  static constexpr int NTR = 2 * (NQ - 1) + K;  // TR0 + NTR <= 80
  static constexpr int NL = (7 + C) / 2 - QA + 1;        // samples per 8 outputs
  static constexpr int NLR = (1 + C) / 2 - QA + 1;       // samples per 2 outputs
  static constexpr int G = K == 9 ? 4 : K == 7 ? 5 : K == 5 ? 6 : K == 3 ? 3 : 4;
  static constexpr int NG = (NQ + G - 1) / G;
};

constexpr int kXP = 84;   // region pitch (floats)
constexpr int kTP = 37;   // pitch of the horizontally filtered rows
constexpr int kZP2 = 40;  // pitch of the decimated samples
constexpr int kT2P = 68;  // pitch of the horizontally up-correlated rows

template <class S, int K>
__global__ __launch_bounds__(256) void sketch_sr_sep_kernel(const S* __restrict__ omega,
                                                            S* __restrict__ Y, SepPsf f,
                                                            int n1, int n2, int64_t ncols) {
  using Gm = SrGeom<K>;
  static_assert(Gm::TR0 >= 0 && Gm::TR0 + Gm::NTR <= kR, "region too small");
  static_assert(Gm::TR0 + 2 * (Gm::NG * Gm::G - 1) + K <= kR, "phase 1 reads past the region");
  static_assert(2 * Gm::G * Gm::NG + K - 2 <= kR, "phase 2 reads past the filtered rows");
  static_assert(Gm::NG * Gm::G <= kTP && Gm::NG * Gm::G <= kZP2, "padding columns");
  static_assert(28 + Gm::NL <= kZP2 && 31 + Gm::NLR <= Gm::NQ, "phase 3/4 reads");
  __shared__ __align__(16) float A[kR * kXP];   // region; later the decimated samples Z
  __shared__ __align__(16) float B[kR * kTP];   // row-filtered T; later T2
  const int tid = threadIdx.x;
  // XCD-aware tile order: workgroups are dispatched round-robin over the 8
  // XCDs, so workgroup id i runs on XCD i % 8.  Each XCD takes a contiguous
  // run of (column, tile row, tile column) work items, so neighbouring tiles,
  // whose halos overlap, share one L2.
  const int tiles_x = n2 / kT, tiles_y = n1 / kT;
  const int total = tiles_x * tiles_y * static_cast<int>(ncols);
  const int per_xcd = (total + 7) / 8;
  const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (w >= total) return;
  const int col = w / (tiles_x * tiles_y), t = w - col * tiles_x * tiles_y;
  const int P0 = (t / tiles_x) * kT, Q0 = (t % tiles_x) * kT;
  const size_t colbase = static_cast<size_t>(col) * n1 * n2;
  const S* src = omega + colbase;

  // ---- phase 0: 10 x 10 Haar blocks of the region, synthesised in registers
  if (tid < 100) {
    const int bi = tid / 10, bj = tid - bi * 10;
    int gr = P0 - kH + 8 * bi; gr += (gr < 0) ? n1 : 0; gr -= (gr >= n1) ? n1 : 0;
    int gq = Q0 - kH + 8 * bj; gq += (gq < 0) ? n2 : 0; gq -= (gq >= n2) ? n2 : 0;
    float v[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r) ld_row8(src + static_cast<size_t>(gr + r) * n2 + gq, v[r]);
    haar8_regs<false>(v);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float* d = A + (8 * bi + r) * kXP + 8 * bj;
      *reinterpret_cast<float4*>(d) = make_float4(v[r][0], v[r][1], v[r][2], v[r][3]);
      *reinterpret_cast<float4*>(d + 4) = make_float4(v[r][4], v[r][5], v[r][6], v[r][7]);
    }
  }
  __syncthreads();

  // ---- phase 1: T[tr][j] = sum_b gv[b] X[TR0 + tr][TR0 + 2 j + b], G outputs per item
  for (int item = tid; item < Gm::NTR * Gm::NG; item += 256) {
    const int tr = item / Gm::NG, g = item - tr * Gm::NG;
    const int j0 = g * Gm::G;
    const float* row = A + (Gm::TR0 + tr) * kXP + Gm::TR0 + 2 * j0;
    constexpr int NIN = 2 * Gm::G - 2 + K;
    float x[NIN];
#pragma unroll
    for (int m = 0; m < NIN; ++m) x[m] = row[m];
#pragma unroll
    for (int o = 0; o < Gm::G; ++o) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < K; ++b) acc = fmaf(f.gv[b], x[2 * o + b], acc);
      B[tr * kTP + j0 + o] = acc;
    }
  }
  __syncthreads();

  // ---- phase 2: Z[i][j] = sum_a gu[a] T[2 i + a][j]   (into A)
  for (int item = tid; item < Gm::NQ * Gm::NG; item += 256) {
    const int g = item / Gm::NQ, j = item - g * Gm::NQ;
    const int i0 = g * Gm::G;
    constexpr int NIN = 2 * Gm::G - 2 + K;
    float t[NIN];
#pragma unroll
    for (int m = 0; m < NIN; ++m) t[m] = B[(2 * i0 + m) * kTP + j];
#pragma unroll
    for (int o = 0; o < Gm::G; ++o) {
      float acc = 0.f;
#pragma unroll
      for (int a = 0; a < K; ++a) acc = fmaf(f.gu[a], t[2 * o + a], acc);
      A[(i0 + o) * kZP2 + j] = acc;
    }
  }
  __syncthreads();

  // ---- phase 3: T2[i][q] = sum_{b: q - C + b even} hv[b] Z[i][(q - C + b)/2 - QA]
  // eight consecutive q per item; their samples start at Z[i][q0 / 2]
  for (int item = tid; item < Gm::NQ * 8; item += 256) {
    const int i = item >> 3, q0 = (item & 7) * 8;
    const float* zr = A + i * kZP2 + q0 / 2;
    float z[Gm::NL];
#pragma unroll
    for (int m = 0; m < Gm::NL; ++m) z[m] = zr[m];
    float o8[8];
#pragma unroll
    for (int dq = 0; dq < 8; ++dq) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < K; ++b)
        if (((dq - Gm::C + b) & 1) == 0) acc = fmaf(f.hv[b], z[(dq - Gm::C + b) / 2 - Gm::QA], acc);
      o8[dq] = acc;
    }
    float* d = B + i * kT2P + q0;
    *reinterpret_cast<float4*>(d) = make_float4(o8[0], o8[1], o8[2], o8[3]);
    *reinterpret_cast<float4*>(d + 4) = make_float4(o8[4], o8[5], o8[6], o8[7]);
  }
  __syncthreads();

  // ---- phase 4: out[p][q] = sum_{a: p - C + a even} hu[a] T2[(p - C + a)/2 - QA][q],
  // then the Haar analysis and the stores.  Four lanes share an 8 x 8 output
  // block, lane w holding rows 2w and 2w + 1: level 1 is lane-local, levels
  // 2 and 3 exchange the low-pass values with the partner lanes w^1 and w^2.
  {
    const int blk = tid >> 2, w = tid & 3;
    const int bi = blk >> 3, bj = blk & 7;
    float t2[Gm::NLR][8];
#pragma unroll
    for (int m = 0; m < Gm::NLR; ++m) {
      const float* s2 = B + (4 * bi + w + m) * kT2P + 8 * bj;
      float4 a = *reinterpret_cast<const float4*>(s2);
      float4 b = *reinterpret_cast<const float4*>(s2 + 4);
      t2[m][0] = a.x; t2[m][1] = a.y; t2[m][2] = a.z; t2[m][3] = a.w;
      t2[m][4] = b.x; t2[m][5] = b.y; t2[m][6] = b.z; t2[m][7] = b.w;
    }
    float v[2][8];
#pragma unroll
    for (int dd = 0; dd < 2; ++dd)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < K; ++a)
          if (((dd - Gm::C + a) & 1) == 0)
            acc = fmaf(f.hu[a], t2[(dd - Gm::C + a) / 2 - Gm::QA][q], acc);
        v[dd][q] = acc;
      }
    // level 1 (stride 1): lane-local 2 x 2 groups
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      float a = v[0][q], b = v[0][q + 1], c = v[1][q], d = v[1][q + 1];
      v[0][q] = 0.5f * (a + b + c + d);
      v[0][q + 1] = 0.5f * (a - b + c - d);
      v[1][q] = 0.5f * (a + b - c - d);
      v[1][q + 1] = 0.5f * (a - b - c + d);
    }
    // level 2 (stride 2): low-pass values at row 2w, columns 0, 2, 4, 6;
    // rows 4r and 4r + 2 sit in lanes w and w ^ 1
    {
      const float sg = (w & 1) ? -1.f : 1.f;
#pragma unroll
      for (int q = 0; q < 8; q += 4) {
        float x0 = v[0][q], x1 = v[0][q + 2];
        float y0 = __shfl_xor(x0, 1, 64), y1 = __shfl_xor(x1, 1, 64);
        v[0][q] = 0.5f * ((y0 + y1) + sg * (x0 + x1));
        v[0][q + 2] = 0.5f * ((y0 - y1) + sg * (x0 - x1));
      }
    }
    // level 3 (stride 4): rows 0 and 4 sit in lanes 0 and 2
    {
      const float sg = (w & 2) ? -1.f : 1.f;
      float x0 = v[0][0], x1 = v[0][4];
      float y0 = __shfl_xor(x0, 2, 64), y1 = __shfl_xor(x1, 2, 64);
      if ((w & 1) == 0) {
        v[0][0] = 0.5f * ((y0 + y1) + sg * (x0 + x1));
        v[0][4] = 0.5f * ((y0 - y1) + sg * (x0 - x1));
      }
    }
    S* dst = Y + colbase + static_cast<size_t>(P0 + 8 * bi + 2 * w) * n2 + Q0 + 8 * bj;
    st_row8(dst, v[0]);
    st_row8(dst + n2, v[1]);
  }
}

// One level of the 2 x 2 orthonormal Haar butterfly on the stride-s grid of a
// region of nb x nb blocks of 8 x 8 stored in `buf` (row pitch `pitch`).
__device__ __forceinline__ void haar_level_lds(float* buf, int pitch, int nb, int s) {
  const int per_blk = (8 / (2 * s)) * (8 / (2 * s));    // groups per block
  const int g_side = 8 / (2 * s);
  const int total = nb * nb * per_blk;
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    int blk = g / per_blk, w = g - blk * per_blk;
    int bi = blk / nb, bj = blk - bi * nb;
    int gi = w / g_side, gj = w - gi * g_side;
    int r = bi * 8 + gi * 2 * s, q = bj * 8 + gj * 2 * s;
    float a = buf[r * pitch + q], b = buf[r * pitch + q + s];
    float c = buf[(r + s) * pitch + q], d = buf[(r + s) * pitch + q + s];
    buf[r * pitch + q] = 0.5f * (a + b + c + d);
    buf[r * pitch + q + s] = 0.5f * (a - b + c - d);
    buf[(r + s) * pitch + q] = 0.5f * (a + b - c - d);
    buf[(r + s) * pitch + q + s] = 0.5f * (a - b - c + d);
  }
}

template <class S>
__global__ __launch_bounds__(256) void sketch_sr_kernel(const S* __restrict__ omega,
                                                        S* __restrict__ Y,
                                                        const float* __restrict__ psf_flip,
                                                        const float* __restrict__ psf, int k,
                                                        int n1, int n2) {
  __shared__ float X[kR * kRP];      // input region; reused for the output tile
  __shared__ float Z[kZ * kZP];      // S H x on the low-resolution grid
  __shared__ float G[81], Hh[81];
  const int c = (k - 1) / 2;
  const int P0 = blockIdx.y * kT, Q0 = blockIdx.x * kT;
  const size_t colbase = static_cast<size_t>(blockIdx.z) * n1 * n2;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    G[t] = psf_flip[t];
    Hh[t] = psf[t];
  }
  // ---- load coefficients of the tile + halo (periodic)
  for (int t = threadIdx.x; t < kR * kR; t += blockDim.x) {
    int r = t / kR, q = t - r * kR;
    int gr = P0 - kH + r; gr += (gr < 0) ? n1 : 0; gr -= (gr >= n1) ? n1 : 0;
    int gq = Q0 - kH + q; gq += (gq < 0) ? n2 : 0; gq -= (gq >= n2) ? n2 : 0;
    X[r * kRP + q] = Io<S>::ld(omega, colbase + static_cast<size_t>(gr) * n2 + gq);
  }
  __syncthreads();
  // ---- Haar synthesis (coarsest level first) on the 10 x 10 blocks
  haar_level_lds(X, kRP, kR / 8, 4);
  __syncthreads();
  haar_level_lds(X, kRP, kR / 8, 2);
  __syncthreads();
  haar_level_lds(X, kRP, kR / 8, 1);
  __syncthreads();
  // ---- z[q] = (H x)[2q] for the low-resolution samples the tile needs:
  // 2q in [P0 - c, P0 + kT - 1 + c]
  const int qa = (P0 - c + 1) >> 1;                 // ceil((P0 - c)/2), P0 even
  const int qb = (P0 + kT - 1 + c) >> 1;
  const int nq = qb - qa + 1;
  const int pa = (Q0 - c + 1) >> 1;
  const int pb = (Q0 + kT - 1 + c) >> 1;
  const int np = pb - pa + 1;
  for (int t = threadIdx.x; t < nq * np; t += blockDim.x) {
    int zi = t / np, zj = t - zi * np;
    // HR row 2(qa+zi) - c + a lives at region row 2(qa+zi) - c + a - (P0 - kH)
    int r0 = 2 * (qa + zi) - c - (P0 - kH);
    int q0 = 2 * (pa + zj) - c - (Q0 - kH);
    float acc = 0.f;
    for (int a = 0; a < k; ++a) {
      const float* row = X + (r0 + a) * kRP + q0;
      const float* g = G + a * k;
      for (int b = 0; b < k; ++b) acc += g[b] * row[b];
    }
    Z[zi * kZP + zj] = acc;
  }
  __syncthreads();
  // ---- out[p] = sum_a h[a] Z[(p - c + a) / 2] over even p - c + a; write into X
  for (int t = threadIdx.x; t < kT * kT; t += blockDim.x) {
    int i = t / kT, j = t - i * kT;
    int p = P0 + i, q = Q0 + j;
    int as = (c - p) & 1, bs = (c - q) & 1;
    float acc = 0.f;
    for (int a = as; a < k; a += 2) {
      int zi = ((p - c + a) >> 1) - qa;
      const float* zr = Z + zi * kZP;
      const float* hr = Hh + a * k;
      for (int b = bs; b < k; b += 2) acc += hr[b] * zr[((q - c + b) >> 1) - pa];
    }
    X[i * kRP + j] = acc;
  }
  __syncthreads();
  // ---- Haar analysis (finest level first) on the 8 x 8 output blocks
  haar_level_lds(X, kRP, kT / 8, 1);
  __syncthreads();
  haar_level_lds(X, kRP, kT / 8, 2);
  __syncthreads();
  haar_level_lds(X, kRP, kT / 8, 4);
  __syncthreads();
  for (int t = threadIdx.x; t < kT * kT; t += blockDim.x) {
    int i = t / kT, j = t - i * kT;
    Io<S>::st(Y, colbase + static_cast<size_t>(P0 + i) * n2 + Q0 + j, X[i * kRP + j]);
  }
}

template <class S, int K>
static void launch_sep(const nys_op_s* op, const S* omega, S* Y, int64_t ell, hipStream_t st) {
  const auto& d = op->d;
  SepPsf f;
  for (int a = 0; a < 9; ++a) {
    f.hu[a] = a < K ? static_cast<float>(op->sep_u[a]) : 0.f;
    f.hv[a] = a < K ? static_cast<float>(op->sep_v[a]) : 0.f;
    f.gu[a] = a < K ? static_cast<float>(op->sep_u[K - 1 - a]) : 0.f;
    f.gv[a] = a < K ? static_cast<float>(op->sep_v[K - 1 - a]) : 0.f;
  }
  const int64_t total = static_cast<int64_t>(d.n2 / kT) * (d.n1 / kT) * ell;
  const unsigned blocks = static_cast<unsigned>((total + 7) / 8 * 8);
  hipLaunchKernelGGL((sketch_sr_sep_kernel<S, K>), dim3(blocks), dim3(256), 0, st, omega, Y, f,
                     d.n1, d.n2, ell);
}

template <class S>
nys_status sketch_sr_fused(nys_op op, const S* omega, S* Y, int64_t ell, hipStream_t st) {
  const auto& d = op->d;
  const int k = d.psf_size;
  if (k > 9 || d.n1 % kT != 0 || d.n2 % kT != 0) {
    if constexpr (sizeof(S) == 2) return sketch_sr_chain_bf16(op, omega, Y, ell, st);
    else return sketch_sr_chain_f32(op, omega, Y, ell, st);
  }
  if (op->sep) {
    switch (k) {
      case 3: launch_sep<S, 3>(op, omega, Y, ell, st); break;
      case 5: launch_sep<S, 5>(op, omega, Y, ell, st); break;
      case 7: launch_sep<S, 7>(op, omega, Y, ell, st); break;
      case 9: launch_sep<S, 9>(op, omega, Y, ell, st); break;
      default: launch_sep<S, 1>(op, omega, Y, ell, st); break;
    }
    return launch_check("sketch_sr_sep_kernel");
  }
  const float* base = reinterpret_cast<const float*>(op->psf_dev.as<double>() + 2 * k * k);
  dim3 grid(d.n2 / kT, d.n1 / kT, static_cast<unsigned>(ell));
  hipLaunchKernelGGL((sketch_sr_kernel<S>), grid, dim3(256), 0, st, omega, Y, base, base + k * k,
                     k, d.n1, d.n2);
  return launch_check("sketch_sr_kernel");
}

template nys_status sketch_sr_fused<float>(nys_op, const float*, float*, int64_t, hipStream_t);
template nys_status sketch_sr_fused<uint16_t>(nys_op, const uint16_t*, uint16_t*, int64_t,
                                              hipStream_t);

}  // namespace nys
