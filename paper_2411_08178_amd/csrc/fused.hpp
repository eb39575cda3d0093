// One inner iteration of the P-weighted TV / Hessian-Schatten prox (the
// accelerated dual gradient method of eqs. (21)-(29) with C = R^N) fused
// into one pass over U.
//
// With P^{-1} = I + U diag(d) U^T (eq. (11)), the iteration on the dual pair
// (Q, R) is
//   x   = s - lam_bar (L^T R + U c),      c = d . U^T L^T R,
//   Q+  = Proj(R + step L x),             R+ = Q+ + beta (Q+ - Q),
// and the next iteration needs c+ = d . U^T L^T R+.  A workgroup owns a tile
// of 512 pixels (two per CU resident, so one's loads overlap the other's
// stencil phases): it stages R and Q around the tile in LDS, reads the U
// row of each pixel of the tile and of a ring of HR pixels around it (HR =
// 1 for the TV kinds, 2 for the Hessian kinds), forms x there (into LDS),
// the dual update on the tile and the ring of one pixel that L^T needs (into
// LDS; the tile's values also to the output buffers), L^T R+ on the tile,
// and the products u_p (L^T R+)_p with the U rows kept in registers.  Their
// sum over the tile is written as the tile's FP64 block partial; the
// coefficient tail (a separate small launch) sums the partials in a fixed
// order, so the result is deterministic.  U is read
// once per inner iteration (plus the ring) instead of twice, and the
// iteration is two launches instead of five.
#pragma once

#include "common.hpp"
#include "internal.hpp"
#include "stencil.hpp"

namespace nys {

constexpr int kFThreads = 512;          // one pixel per thread
constexpr int kFWaves = kFThreads / 64;
constexpr int kFKeep = 80;              // rows of U a thread keeps in registers at most (no spills)
// Tile width: 64 x 8 tiles for the TV kinds (ring of 1: longer contiguous
// runs of U per row, 29 % ring), 32 x 16 for the Hessian kinds (ring of 2:
// 41 % instead of 59 %).
__host__ __device__ constexpr int fused_tw(bool hess) { return hess ? 32 : 64; }

// One tile's operands (a single reconstruction or one instance of a batch),
// in the compute type T of U and the images (float or double).
template <class T>
struct FusedArgsT {
  int n1, n2, reg;
  int ell, ell_pad;
  int64_t ldu;
  const T* U;                      // column-major, ell_pad rows, zero padded
  const double* cd;                // c = d . U^T L^T R (ell values)
  const T* s;                      // prox centre
  const T* Qi;                     // duals read (nch channels, N apart)
  const T* Ri;
  T* Qo;                           // duals written (tile pixels only)
  T* Ro;
  T lam_bar, step, beta;
  int last;                        // partials of L^T Q+ instead of L^T R+
  double* part;                    // [tiles][ell_pad] block partials
};
using FusedArgs = FusedArgsT<float>;

// LDS of a tile TW wide (regions for a ring of up to 2): R (ring 3), Q and
// R+ (ring 1), x (ring 2)
template <int TW, class T = float>
struct FusedLds {
  static constexpr int TH = kFThreads / TW;
  T r[3][(TH + 6) * (TW + 6)];
  T q[3][(TH + 2) * (TW + 2)];
  T x[(TH + 4) * (TW + 4)];
  T p[3][(TH + 2) * (TW + 2)];
  T c[PcMeta::kMaxEll];
  double red[kFWaves][PcMeta::kMaxEll];
};

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }

// Butterfly reduce-scatter of CNT values over the lanes of a wave: at each
// offset OFF (32, 16, ...) a lane keeps one half of its values, sends the
// other half to lane ^ OFF and adds what it receives, while CNT stays even;
// the rest is summed over the remaining offsets.  On return the lane holds
// the wave sums of components base .. base + cnt_left - 1; every lane with
// the same base holds the same sums.
template <int CNT, int OFF>
struct Bfly {
  static constexpr bool kHalve = OFF >= 1 && CNT % 2 == 0 && CNT >= 2;
  static constexpr int kLeft = kHalve ? Bfly<CNT / 2, OFF / 2>::kLeft : CNT;
  // lanes below this mask hold duplicates of one another's sums
  static constexpr int kDupMask = kHalve ? Bfly<CNT / 2, OFF / 2>::kDupMask : (OFF * 2 - 1);
  template <class T>
  __device__ __forceinline__ static void run(T* v, int lane, int& base) {
    if constexpr (kHalve) {
      const bool up = (lane & OFF) != 0;
#pragma unroll
      for (int i = 0; i < CNT / 2; ++i) {
        const T keep = up ? v[i + CNT / 2] : v[i];
        const T send = up ? v[i] : v[i + CNT / 2];
        v[i] = keep + __shfl_xor(send, OFF);
      }
      if (up) base += CNT / 2;
      Bfly<CNT / 2, OFF / 2>::run(v, lane, base);
    } else {
#pragma unroll
      for (int o = OFF; o >= 1; o >>= 1) {
#pragma unroll
        for (int i = 0; i < CNT; ++i) v[i] += __shfl_xor(v[i], o);
      }
    }
  }
};
template <int CNT>
struct Bfly<CNT, 0> {
  static constexpr int kLeft = CNT;
  static constexpr int kDupMask = 0;
  template <class T>
  __device__ __forceinline__ static void run(T*, int, int&) {}
};

// Pixel h (0 <= h < 2 hr (TW + 2 hr) + 2 hr TH) of the ring of hr pixels
// around a TW-wide tile -> coordinates in the x region (origin: tile - (hr, hr)).
template <int TW>
__device__ __forceinline__ void fused_ring(int h, int hr, int& ey, int& ex) {
  constexpr int kFW = TW, kFH = kFThreads / TW;
  const int ew = kFW + 2 * hr;
  const int band = hr * ew;
  if (h < band) { ey = h / ew; ex = h - ey * ew; return; }
  h -= band;
  if (h < band) { ey = kFH + hr + h / ew; ex = h % ew; return; }
  h -= band;
  const int side = kFH * hr;
  if (h < side) { ey = hr + h / hr; ex = h % hr; return; }
  h -= side;
  ey = hr + h / hr;
  ex = kFW + hr + h % hr;
}

// KR (a multiple of 16, <= min(ell_pad, kFKeep)) rows of U stay in registers;
// the next ntl rows (at most ell - KR) stay in LDS (Lt, one column per
// thread, written and read back by the same thread), and rows from KR + ntl
// on are read a second time for the partials.
template <int KR, int TW, class T>
__device__ __forceinline__ void fused_tile(const FusedArgsT<T>& A, int tile, int ntx,
                                           FusedLds<TW, T>& L, T* Lt = nullptr, int ntl = 0) {
  constexpr int kFW = TW, kFH = kFThreads / TW;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int n1 = A.n1, n2 = A.n2, reg = A.reg;
  const bool hess = reg_hessian(reg);
  const int nch = hess ? 3 : 2;
  const int hr = hess ? 2 : 1;
  const int64_t N = static_cast<int64_t>(n1) * n2;
  const int ty0 = (tile / ntx) * kFH, tx0 = (tile % ntx) * kFW;
  const int Lp = A.ell_pad;
  const int64_t ldu = A.ldu;
  const T* __restrict__ U = A.U;
  // region geometry: R (ring hr + 1), x (ring hr), duals (ring 1)
  const int rw = kFW + 2 * hr + 2, rh = kFH + 2 * hr + 2;
  const int ry0 = ty0 - hr - 1, rx0 = tx0 - hr - 1;
  const int xw = kFW + 2 * hr;
  const int xy0 = ty0 - hr, xx0 = tx0 - hr;
  constexpr int dw = kFW + 2, dh = kFH + 2;
  const int dy0 = ty0 - 1, dx0 = tx0 - 1;

  // ---- c, R and Q into LDS
  for (int k = t; k < Lp; k += kFThreads) L.c[k] = k < A.ell ? static_cast<T>(A.cd[k]) : T(0);
  for (int r = t; r < rw * rh; r += kFThreads) {
    const int yy = r / rw, xx = r - yy * rw;
    const int gi = ry0 + yy, gj = rx0 + xx;
    if (gi >= 0 && gi < n1 && gj >= 0 && gj < n2) {
      const int64_t o = static_cast<int64_t>(gi) * n2 + gj;
      for (int c = 0; c < nch; ++c) L.r[c][r] = A.Ri[c * N + o];
    }
  }
  for (int r = t; r < dw * dh; r += kFThreads) {
    const int yy = r / dw, xx = r - yy * dw;
    const int gi = dy0 + yy, gj = dx0 + xx;
    if (gi >= 0 && gi < n1 && gj >= 0 && gj < n2) {
      const int64_t o = static_cast<int64_t>(gi) * n2 + gj;
      for (int c = 0; c < nch; ++c) L.q[c][r] = A.Qi[c * N + o];
    }
  }
  __syncthreads();
  auto ra = [&](int c, int ii, int jj) { return L.r[c][(ii - ry0) * rw + (jj - rx0)]; };
  // (U c)_o: the first KR rows with every load issued before the sum, the
  // rest in runs of 16.  Rows from ell on are U's zero padding: they are not
  // loaded (a zero in their place gives the same sums).
  const int ell = A.ell;
  auto uc = [&](int64_t o, T* v, int keep) {
#pragma unroll
    for (int k = 0; k < KR; ++k) v[k] = k < ell ? U[k * ldu + o] : T(0);
    T y = 0;
#pragma unroll
    for (int k = 0; k < KR; ++k) y = fma_t(v[k], L.c[k], y);
    for (int k0 = KR; k0 < Lp; k0 += 16) {
      T w[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) w[j] = k0 + j < ell ? U[(k0 + j) * ldu + o] : T(0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        y = fma_t(w[j], L.c[k0 + j], y);
        if (k0 + j - KR < keep) Lt[(k0 + j - KR) * kFThreads + t] = w[j];
      }
    }
    return y;
  };

  // ---- x = s - lam_bar (L^T R + U c) on the ring of hr (first, so that
  // its loads do not hold registers next to the tile's kept rows) and the
  // tile
  T u[KR];
  const int nring = 2 * hr * xw + 2 * hr * kFH;
  for (int h = t; h < nring; h += kFThreads) {
    int ey, ex;
    fused_ring<TW>(h, hr, ey, ex);
    const int gi = xy0 + ey, gj = xx0 + ex;
    if (gi >= 0 && gi < n1 && gj >= 0 && gj < n2) {
      const int64_t o = static_cast<int64_t>(gi) * n2 + gj;
      const T y = uc(o, u, 0);
      const T tr = lt_with<T>(ra, reg, gi, gj, n1, n2);
      L.x[ey * xw + ex] = A.s[o] - A.lam_bar * (tr + y);
    }
  }
  const int iy = t / kFW, ix = t % kFW;
  const int pi = ty0 + iy, pj = tx0 + ix;
  const bool pin = pi < n1 && pj < n2;
  const int64_t po = pin ? static_cast<int64_t>(pi) * n2 + pj : 0;
  {
    const T y = uc(po, u, ntl);
    if (pin) {
      const T tr = lt_with<T>(ra, reg, pi, pj, n1, n2);
      L.x[(iy + hr) * xw + ix + hr] = A.s[po] - A.lam_bar * (tr + y);
    }
  }
  __syncthreads();

  // ---- dual step on the tile and the ring of one pixel (TV: only the
  // bottom row and right column of the ring feed L^T)
  auto xa = [&](int ii, int jj) { return L.x[(ii - xy0) * xw + (jj - xx0)]; };
  for (int r = t; r < dw * dh; r += kFThreads) {
    const int yy = r / dw, xx = r - yy * dw;
    const int gi = dy0 + yy, gj = dx0 + xx;
    if (gi < 0 || gi >= n1 || gj < 0 || gj >= n2) continue;
    if (!hess && (yy == 0 || xx == 0)) continue;
    const int64_t o = static_cast<int64_t>(gi) * n2 + gj;
    const int rl = (gi - ry0) * rw + (gj - rx0);
    T l0, l1, l2, v[3];
    lx_with<T>(xa, reg, gi, gj, n1, n2, l0, l1, l2);
    v[0] = L.r[0][rl] + A.step * l0;
    v[1] = L.r[1][rl] + A.step * l1;
    v[2] = hess ? L.r[2][rl] + A.step * l2 : T(0);
    project_group(reg, v);
    const bool own = yy >= 1 && yy <= kFH && xx >= 1 && xx <= kFW;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < nch) {
        const T rn = v[c] + A.beta * (v[c] - L.q[c][r]);
        L.p[c][r] = A.last ? v[c] : rn;
        if (own) {
          A.Qo[c * N + o] = v[c];
          A.Ro[c * N + o] = rn;
        }
      }
    }
  }
  __syncthreads();

  // ---- (L^T R+)_p and the tile's partial of U^T L^T R+
  T tp = 0;
  if (pin) {
    auto pa = [&](int c, int ii, int jj) { return L.p[c][(ii - dy0) * dw + (jj - dx0)]; };
    tp = lt_with<T>(pa, reg, pi, pj, n1, n2);
  }
#pragma unroll
  for (int k = 0; k < KR; ++k) u[k] *= tp;
  int base = 0;
  using B = Bfly<KR, 32>;
  B::run(u, lane, base);
  if ((lane & B::kDupMask) == 0) {
#pragma unroll
    for (int i = 0; i < B::kLeft; ++i) L.red[wave][base + i] = static_cast<double>(u[i]);
  }
  for (int k0 = KR; k0 < Lp; k0 += 16) {
    T w[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = k0 + j;
      w[j] = k < ell ? (k - KR < ntl ? Lt[(k - KR) * kFThreads + t] : U[k * ldu + po]) * tp : T(0);
    }
    int b2 = 0;
    using B2 = Bfly<16, 32>;
    B2::run(w, lane, b2);
    if ((lane & B2::kDupMask) == 0) {
#pragma unroll
      for (int i = 0; i < B2::kLeft; ++i) L.red[wave][k0 + b2 + i] = static_cast<double>(w[i]);
    }
  }
  __syncthreads();
  if (t < Lp) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kFWaves; ++w) sum += L.red[w][t];
    A.part[static_cast<size_t>(tile) * Lp + t] = sum;
  }
}

// Tile of block b: every XCD (b mod 8) takes a contiguous run of tiles, so
// the rings a tile reads were mostly read as neighbouring tiles' pixels by
// the same L2.
__device__ __forceinline__ int fused_tile_of(int b, int ntiles) {
  const int per = (ntiles + 7) / 8;
  return (b % 8) * per + b / 8;
}

}  // namespace nys
