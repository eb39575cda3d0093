// Fused sketch for the wavelet-reparametrised blur + 2x decimation operator:
//   Y = W H^T S^T S H W^T Omega        (Alg. 1 step 2 with eq. (23)'s Phi)
// One workgroup produces a 64 x 64 tile of coefficients of one column.  It
// reads the tile plus an 8-pixel halo (whole 8 x 8 Haar blocks) once from
// HBM, and keeps every intermediate in LDS: Haar synthesis, blur sampled at
// the decimated grid, zero-filled upsampling + correlation, Haar analysis.
// Requires PSF size <= 9 (two half-widths fit in the 8-pixel halo).

#include "common.hpp"
#include "internal.hpp"

namespace nys {

namespace {
constexpr int kT = 64;             // output tile (coefficients)
constexpr int kH = 8;              // halo = one Haar block
constexpr int kR = kT + 2 * kH;    // 80: input region side
constexpr int kRP = kR + 1;        // padded LDS row
constexpr int kZ = kT / 2 + 6;     // low-resolution region side bound (k <= 9)
constexpr int kZP = kZ + 1;
}  // namespace

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

template <class S>
nys_status sketch_sr_fused(nys_op op, const S* omega, S* Y, int64_t ell, hipStream_t st) {
  const auto& d = op->d;
  const int k = d.psf_size;
  if (k > 9 || d.n1 % kT != 0 || d.n2 % kT != 0) {
    if constexpr (sizeof(S) == 2) return sketch_sr_chain_bf16(op, omega, Y, ell, st);
    else return sketch_sr_chain_f32(op, omega, Y, ell, st);
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
