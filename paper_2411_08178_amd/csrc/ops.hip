// Operators A, A^T (periodic blur, blur + decimation, parallel-beam Joseph
// pair, Haar pyramid) and the batched sketch Y = Phi Omega (Alg. 1 step 2).
//
// Images are row-major; a batch of columns is indexed by blockIdx.z.
// Every kernel is templated on its input storage type SI, output storage
// type SO and compute type C, so BF16 sketches accumulate in FP32.

#include <cmath>
#include <complex>
#include <type_traits>
#include <vector>
#include <cstdarg>

#include "common.hpp"
#include "internal.hpp"

namespace nys {

// ---------------------------------------------------------------- errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

// ================================================================ blur
// out[i, j] = sum_{a,b} g[a, b] in[(f i - c + a) mod n1, (f j - c + b) mod n2]
// on an output grid o1 x o2.  g = flipped PSF gives H (f = 1) or S H (f > 1);
// g = PSF gives H^T.
constexpr int kCorTW = 64;

// TH output rows per workgroup (16, or 4 when the grid would be small)
template <class SI, class SO, class C, int TH>
__global__ __launch_bounds__(256) void correlate_kernel(
    const SI* __restrict__ in, SO* __restrict__ out, const C* __restrict__ g,
    int k, int n1, int n2, int o1, int o2, int f) {
  extern __shared__ unsigned char smem_raw[];
  C* sg = reinterpret_cast<C*>(smem_raw);
  C* tile = sg + k * k;
  const int c = (k - 1) / 2;
  const int i0 = blockIdx.y * TH, j0 = blockIdx.x * kCorTW;
  const int th = f * (TH - 1) + k, tw = f * (kCorTW - 1) + k;
  const SI* src = in + static_cast<size_t>(blockIdx.z) * n1 * n2;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) sg[t] = g[t];
  const int r0 = f * i0 - c, q0 = f * j0 - c;
  for (int t = threadIdx.x; t < th * tw; t += blockDim.x) {
    int r = t / tw, q = t - r * tw;
    int gr = (r0 + r) % n1; if (gr < 0) gr += n1;
    int gq = (q0 + q) % n2; if (gq < 0) gq += n2;
    tile[t] = Io<SI>::ld(src, static_cast<size_t>(gr) * n2 + gq);
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  SO* dst = out + static_cast<size_t>(blockIdx.z) * o1 * o2;
  for (int rr = ty; rr < TH; rr += 4) {
    int oi = i0 + rr, oj = j0 + tx;
    if (oi >= o1 || oj >= o2) continue;
    C acc = 0;
    const C* base = tile + (f * rr) * tw + f * tx;
    for (int a = 0; a < k; ++a) {
      const C* row = base + a * tw;
      const C* grow = sg + a * k;
      for (int b = 0; b < k; ++b) acc += grow[b] * row[b];
    }
    Io<SO>::st(dst, static_cast<size_t>(oi) * o2 + oj, acc);
  }
}

// Adjoint of blur + decimation: out[p, q] = sum_{a,b} h[a, b] Z[p - c + a, q - c + b]
// with Z the zero-filled upsampling (by f) of the m1 x m2 input.
constexpr int kUpTW = 64;

__host__ __device__ inline int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// TH output rows per workgroup (32, or 8 when the grid would be small)
template <class SI, class SO, class C, int TH>
__global__ __launch_bounds__(256) void upcorrelate_kernel(
    const SI* __restrict__ in, SO* __restrict__ out, const C* __restrict__ h,
    int k, int m1, int m2, int f) {
  extern __shared__ unsigned char smem_raw[];
  C* sh = reinterpret_cast<C*>(smem_raw);
  C* tile = sh + k * k;
  const int n1 = m1 * f, n2 = m2 * f, c = (k - 1) / 2;
  const int p0 = blockIdx.y * TH, q0 = blockIdx.x * kUpTW;
  const int R0 = floor_div(p0 - c, f), R1 = floor_div(p0 + TH - 1 - c + k - 1, f);
  const int C0 = floor_div(q0 - c, f), C1 = floor_div(q0 + kUpTW - 1 - c + k - 1, f);
  const int th = R1 - R0 + 1, tw = C1 - C0 + 1;
  const SI* src = in + static_cast<size_t>(blockIdx.z) * m1 * m2;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) sh[t] = h[t];
  for (int t = threadIdx.x; t < th * tw; t += blockDim.x) {
    int r = t / tw, q = t - r * tw;
    int gr = (R0 + r) % m1; if (gr < 0) gr += m1;
    int gq = (C0 + q) % m2; if (gq < 0) gq += m2;
    tile[t] = Io<SI>::ld(src, static_cast<size_t>(gr) * m2 + gq);
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  SO* dst = out + static_cast<size_t>(blockIdx.z) * n1 * n2;
  const int q = q0 + tx;
  int bs = (c - q) % f; if (bs < 0) bs += f;
  for (int rr = ty; rr < TH; rr += 4) {
    int p = p0 + rr;
    if (p >= n1 || q >= n2) continue;
    int as = (c - p) % f; if (as < 0) as += f;
    C acc = 0;
    for (int a = as; a < k; a += f) {
      int lr = (p - c + a - f * R0) / f;
      const C* row = tile + lr * tw;
      for (int b = bs; b < k; b += f) {
        int lc = (q - c + b - f * C0) / f;
        acc += sh[a * k + b] * row[lc];
      }
    }
    Io<SO>::st(dst, static_cast<size_t>(p) * n2 + q, acc);
  }
}

// ================================================================ Haar
// In-place layout: the coefficients of each 2^L x 2^L block stay in the block.
// Analysis applies levels 0..L-1 (stride 1, 2, 4 inside the block), synthesis
// the reverse order; the 2 x 2 step is its own inverse.  B = 2^L consecutive
// lanes hold the B rows of a block (a wave covers 64 / B neighbouring blocks,
// so every row load is a contiguous run); at stride s the rows r and r + s of
// a 2 x 2 group (r a multiple of 2s) trade values through width-B shuffles.
template <int L, bool kAnalysis, class SI, class SO, class C>
__global__ __launch_bounds__(256) void haar_kernel(const SI* __restrict__ in,
                                                   SO* __restrict__ out, int n1, int n2) {
  constexpr int B = 1 << L;
  const int nb2 = n2 / B, nb1 = n1 / B;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = gt / B, r = gt % B;
  const bool live = blk < nb1 * nb2;
  const int bi = live ? blk / nb2 : 0, bj = live ? blk - bi * nb2 : 0;
  const size_t row = static_cast<size_t>(blockIdx.z) * n1 * n2 +
                     static_cast<size_t>(bi * B + r) * n2 + bj * B;
  C v[B];
#pragma unroll
  for (int q = 0; q < B; ++q) v[q] = live ? Io<SI>::ld(in, row + q) : C(0);
#pragma unroll
  for (int it = 0; it < L; ++it) {
    const int lev = kAnalysis ? it : (L - 1 - it);
    const int s = 1 << lev;
    const bool part = (r & (s - 1)) == 0;   // rows at this level's spacing
    const bool top = (r & s) == 0;
#pragma unroll
    for (int q = 0; q < B; q += 2 * s) {
      const C o0 = __shfl_xor(v[q], s, B), o1 = __shfl_xor(v[q + s], s, B);
      const C a = top ? v[q] : o0, b = top ? v[q + s] : o1;
      const C cc = top ? o0 : v[q], d = top ? o1 : v[q + s];
      if (part) {
        v[q] = top ? (a + b + cc + d) * C(0.5) : (a + b - cc - d) * C(0.5);
        v[q + s] = top ? (a - b + cc - d) * C(0.5) : (a - b - cc + d) * C(0.5);
      }
    }
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < B; ++q) Io<SO>::st(out, row + q, v[q]);
  }
}

// ================================================================ Joseph
// A view is stepped along image rows when |cos| >= |sin| (the "row branch")
// and along columns otherwise.  With (a, b) = (cos, sin) on the row branch
// and (sin, cos) on the column branch, the ray of detector coordinate s meets
// the stepped line at centred coordinate t at the interpolation coordinate
// f(t) = (s - t b) / a + c, c = (n - 1) / 2, and takes
// (1 - w) x[q] + w x[q + 1] with q = floor(f), w = f - q, weighted 1 / |a|.
// The forward evaluates f(t) = f0 + t g (f0 = s / a + c, g = -b / a) and
// reads a transposed copy of the image on column-branch views, so that every
// view walks rows and neighbouring rays read neighbouring pixels.
// Coordinates and interpolation weights are computed in FP64 (on MI355X the
// FP64 vector rate equals the unpacked FP32 rate); they reach a few hundred,
// where FP32 rounding would put ~1e-5 errors into every weight.  Samples are
// accumulated in the compute type C.
// One workgroup takes 256 consecutive bins of a view and stages the rows its
// rays cross in LDS.  Every ray of a view shares the slope g, so at step t
// the block's rays lie between those of its first and last bin: row t is
// needed only over [floor(min f), floor(max f) + 1], at most 255 / |a| + 3 <=
// 364 pixels (|a| >= 1/sqrt 2).  kJosRows rows at a time are copied into LDS
// (16-byte loads when the rows allow them, zeros outside the image), then
// every ray takes its kJosRows samples from LDS: out-of-image samples read
// zeros, so no per-sample bounds test is needed.  Staging replaces two
// gathered loads per sample (the texture-address rate bounded the gathering
// form) by two LDS reads.
constexpr int kJosRows = 16;
constexpr int kJosWin = 372;   // window: 364 pixels + alignment of its start to 4

template <class SI, class SO, class C, bool kVec>
__global__ __launch_bounds__(256) void joseph_fwd_lds_kernel(
    const SI* __restrict__ x, const SI* __restrict__ xT, SO* __restrict__ p, int n, int V, int B,
    const double* __restrict__ trig) {
  __shared__ __align__(16) C win[kJosRows][kJosWin];
  __shared__ int base[kJosRows];
  const int v = blockIdx.y;
  const int bfirst = blockIdx.x * 256, blast = min(B - 1, bfirst + 255);
  const int b = bfirst + threadIdx.x;
  const bool valid = b < B;
  const double ct = trig[2 * v], st = trig[2 * v + 1];
  const bool rows = fabs(ct) >= fabs(st);
  const double a = rows ? ct : st, bb = rows ? st : ct;
  const SI* img = (rows ? x : xT) + static_cast<size_t>(blockIdx.z) * n * n;
  const double c = 0.5 * (n - 1);
  const double ia = 1.0 / a;
  const double g = -bb * ia;
  const double f0 = (b - 0.5 * (B - 1)) * ia + c;
  const double fa0 = (bfirst - 0.5 * (B - 1)) * ia + c, fb0 = (blast - 0.5 * (B - 1)) * ia + c;
  // steps where any of the block's rays can meet the image: the interval
  // [lo + (t - c) g, hi + (t - c) g] of their coordinates meets [-1, n)
  // (widened by one step each way, bounds clamped before the conversion)
  const double lo0 = fmin(fa0, fb0), hi0 = fmax(fa0, fb0);
  int T0 = 0, T1 = n - 1;
  if (g != 0.0) {
    double ta = g > 0.0 ? (-1.0 - hi0) / g + c : (n - lo0) / g + c;
    double tb = g > 0.0 ? (n - lo0) / g + c : (-1.0 - hi0) / g + c;
    ta = fmin(fmax(ta, -2.0), n + 1.0);
    tb = fmin(fmax(tb, -2.0), n + 1.0);
    T0 = max(0, static_cast<int>(floor(ta)) - 1);
    T1 = min(n - 1, static_cast<int>(ceil(tb)) + 1);
  } else if (!(lo0 < n && hi0 >= -1.0)) {
    T1 = -1;
  }
  C acc = 0;
  for (int T = T0; T <= T1; T += kJosRows) {
    const int nr = min(kJosRows, T1 - T + 1);
    __syncthreads();   // the previous rows are no longer read
    if (threadIdx.x < nr) {
      const int t = T + threadIdx.x;
      const double fa = fa0 + (t - c) * g, fb = fb0 + (t - c) * g;
      const int lo = static_cast<int>(floor(fmin(fa, fb)));
      base[threadIdx.x] = lo - (((lo % 4) + 4) % 4);
    }
    __syncthreads();
    if constexpr (kVec) {
      static_assert(std::is_same<C, float>::value, "16-byte staging holds float rows");
      for (int e = threadIdx.x; e < nr * (kJosWin / 4); e += 256) {
        const int r = e / (kJosWin / 4), k = 4 * (e - r * (kJosWin / 4));
        const int col = base[r] + k;
        const SI* row = img + static_cast<size_t>(T + r) * n;
        float4 q4;
        if (col >= 0 && col + 3 < n) {
          q4 = *reinterpret_cast<const float4*>(row + col);
        } else {
          q4.x = (col >= 0 && col < n) ? static_cast<float>(row[col]) : 0.f;
          q4.y = (col + 1 >= 0 && col + 1 < n) ? static_cast<float>(row[col + 1]) : 0.f;
          q4.z = (col + 2 >= 0 && col + 2 < n) ? static_cast<float>(row[col + 2]) : 0.f;
          q4.w = (col + 3 >= 0 && col + 3 < n) ? static_cast<float>(row[col + 3]) : 0.f;
        }
        *reinterpret_cast<float4*>(&win[r][k]) = q4;
      }
    } else {
      for (int e = threadIdx.x; e < nr * kJosWin; e += 256) {
        const int r = e / kJosWin, k = e - r * kJosWin;
        const int col = base[r] + k;
        win[r][k] = (col >= 0 && col < n)
                        ? static_cast<C>(Io<SI>::ld(img + static_cast<size_t>(T + r) * n, col))
                        : C(0);
      }
    }
    __syncthreads();
    if (valid) {
      for (int r = 0; r < nr; ++r) {
        const double f = f0 + ((T + r) - c) * g;
        const double fl = floor(f);
        const int q = static_cast<int>(fl);
        const C w = static_cast<C>(f - fl);
        const int k = min(max(q - base[r], 0), kJosWin - 2);
        acc += (C(1) - w) * win[r][k] + w * win[r][k + 1];
      }
    }
  }
  if (valid)
    Io<SO>::st(p, (static_cast<size_t>(blockIdx.z) * V + v) * B + b,
               acc * static_cast<C>(1.0 / fabs(a)));
}

// out[k][j][i] = in[k][i][j] (n x n images), 32 x 32 tiles through LDS.
template <class T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                        int n) {
  __shared__ T tile[32][33];
  const size_t off = static_cast<size_t>(blockIdx.z) * n * n;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    if (i < n && j < n) tile[r][tx] = in[off + static_cast<size_t>(i) * n + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + tx;
    if (i < n && j < n) out[off + static_cast<size_t>(j) * n + i] = tile[tx][r];
  }
}

// Gather-form transpose: pixel (i, j) has stepped coordinate t and
// interpolated index q on each view; the rays that weight it are those with
// |f(t) - q| < 1, i.e. the bins within |a| of its exact bin coordinate
// bc = (q - c) a + t b + (B - 1) / 2 (at most two), with weight
// (1 - |bin - bc| / |a|) / |a| -- the forward's interpolation weight.
// A workgroup takes a 64 x 4 pixel tile; per view the tile reads at most
// 63 + 3 + 3 consecutive bins, so kJosViews sinogram rows at a time are
// staged in LDS over a window of kJosBins bins (16-byte loads when the rows
// allow them, zeros off the detector) and every sample is an LDS read.
constexpr int kJosViews = 16;
constexpr int kJosBins = 76;   // 69 bins + alignment of the window start to 4
template <class SI, class SO, class C, bool kVec>
__global__ __launch_bounds__(256) void joseph_adj_lds_kernel(
    const SI* __restrict__ p, SO* __restrict__ x, int n, int V, int B,
    const double* __restrict__ trig, const double* __restrict__ inv_abs_a) {
  __shared__ __align__(16) C win[kJosViews][kJosBins];
  __shared__ int base[kJosViews];
  const int i0 = blockIdx.y * 4, j0 = blockIdx.x * 64;
  const int j = j0 + (threadIdx.x & 63);
  const int i = i0 + (threadIdx.x >> 6);
  const bool valid = i < n && j < n;
  const SI* sino = p + static_cast<size_t>(blockIdx.z) * V * B;
  const double c = 0.5 * (n - 1);
  const double half = 0.5 * (B - 1);
  C acc = 0;
  for (int V0 = 0; V0 < V; V0 += kJosViews) {
    const int nv = min(kJosViews, V - V0);
    __syncthreads();   // the previous views are no longer read
    if (threadIdx.x < nv) {
      // lowest bin any pixel of the tile reads on this view (bc is affine in
      // (i, j): its minimum sits at a corner of the tile)
      const int v = V0 + threadIdx.x;
      const double ct = trig[2 * v], st = trig[2 * v + 1];
      const bool rows = fabs(ct) >= fabs(st);
      const double a = rows ? ct : st, bb = rows ? st : ct, aa = fabs(a);
      const double tl = (rows ? i0 : j0) - c, th = (rows ? i0 + 3 : j0 + 63) - c;
      const double ql = (rows ? j0 : i0) - c, qh = (rows ? j0 + 63 : i0 + 3) - c;
      const double bcmin = fmin(ql * a, qh * a) + fmin(tl * bb, th * bb) + half;
      const int lo = static_cast<int>(floor(bcmin - aa)) + 1;
      base[threadIdx.x] = lo - (((lo % 4) + 4) % 4);
    }
    __syncthreads();
    if constexpr (kVec) {
      static_assert(std::is_same<C, float>::value, "16-byte staging holds float rows");
      for (int e = threadIdx.x; e < nv * (kJosBins / 4); e += 256) {
        const int r = e / (kJosBins / 4), k = 4 * (e - r * (kJosBins / 4));
        const int col = base[r] + k;
        const SI* row = sino + static_cast<size_t>(V0 + r) * B;
        float4 q4;
        if (col >= 0 && col + 3 < B) {
          q4 = *reinterpret_cast<const float4*>(row + col);
        } else {
          q4.x = (col >= 0 && col < B) ? static_cast<float>(row[col]) : 0.f;
          q4.y = (col + 1 >= 0 && col + 1 < B) ? static_cast<float>(row[col + 1]) : 0.f;
          q4.z = (col + 2 >= 0 && col + 2 < B) ? static_cast<float>(row[col + 2]) : 0.f;
          q4.w = (col + 3 >= 0 && col + 3 < B) ? static_cast<float>(row[col + 3]) : 0.f;
        }
        *reinterpret_cast<float4*>(&win[r][k]) = q4;
      }
    } else {
      for (int e = threadIdx.x; e < nv * kJosBins; e += 256) {
        const int r = e / kJosBins, k = e - r * kJosBins;
        const int col = base[r] + k;
        win[r][k] = (col >= 0 && col < B)
                        ? static_cast<C>(Io<SI>::ld(sino + static_cast<size_t>(V0 + r) * B, col))
                        : C(0);
      }
    }
    __syncthreads();
    if (valid) {
      for (int r = 0; r < nv; ++r) {
        const int v = V0 + r;
        const double ct = trig[2 * v], st = trig[2 * v + 1];
        const bool rows = fabs(ct) >= fabs(st);
        const double a = rows ? ct : st, bb = rows ? st : ct;
        const double ia = inv_abs_a[v], aa = fabs(a);
        const double t = (rows ? i : j) - c;
        const double q = (rows ? j : i) - c;
        const double bc = q * a + t * bb + half;
        const int b0 = static_cast<int>(floor(bc - aa)) + 1;
        const int k = min(max(b0 - base[r], 0), kJosBins - 2);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double wgt = (1.0 - fabs(b0 + u - bc) * ia) * ia;
          acc += static_cast<C>(wgt > 0.0 ? wgt : 0.0) * win[r][k + u];
        }
      }
    }
  }
  if (valid)
    Io<SO>::st(x, static_cast<size_t>(blockIdx.z) * n * n + static_cast<size_t>(i) * n + j, acc);
}

// ---------------------------------------------------------------- FP32 pair
// Compute type FP32 with FP32 images.  Coordinates reach a few hundred, where
// an FP32 value carries absolute rounding errors near 1e-5; here every
// coordinate is instead split into an integer and a fraction.  The terms a
// coordinate is built from -- one per ray and one per step in the forward,
// one per view and pixel row in the adjoint -- are split in FP64, and only
// fractions (or exactly representable multiples of 2^-12) are added in FP32,
// so an interpolation weight is off by a few 1e-7 at any coordinate.
// Staging is double-buffered with one barrier per stage: the 16-byte loads of
// the next stage are issued before the current stage's samples are taken and
// are stored to the other LDS buffer after them.  The per-row (per-view)
// terms, window bases included, are built two stages ahead into a three-deep
// table, so that the loads of the next stage read their bases from LDS.  A
// 16-byte group of a row lies wholly inside or wholly outside the image
// (window starts aligned to 4, row lengths multiples of 4), so it is loaded
// or zero-filled whole.  The windows are sized so that every sample, its
// coordinate rounded either way across an integer, lies inside: no index is
// clamped.  The forward samples only the bins in the image's shadow, and on
// few columns halves its steps between two workgroups.
constexpr int kJfRows = 8;                                         // steps per stage
constexpr int kJfSlots = (kJfRows * (kJosWin / 4) + 255) / 256;    // loads per thread per stage
struct JosStep {
  float frac;   // fraction of (t - c) g - base, in [0, 1)
  int whole;    // its integer part plus the LDS offset of the step's window row
  int base;     // first pixel of the window (multiple of 4)
  int lbase;    // base for the loads: kJosNoRow past the image's last row
};
constexpr int kJosNoRow = -(1 << 29);   // makes every column of the row test as outside

// Leftmost pixel any ray of the block may read on step t, less one pixel of
// margin for a coordinate rounded down across an integer, aligned down to 4.
__device__ __forceinline__ int jos_fwd_base(double lo0, double g, double c, int t) {
  return (static_cast<int>(floor(lo0 + (t - c) * g)) - 1) & ~3;
}
__device__ __forceinline__ int jos_next3(int i) { return i == 2 ? 0 : i + 1; }
// the largest float below 1: fractions rounded to FP32 stay below 1, so that
// the sum of two stays below 2
constexpr float kJosBelowOne = 0x1.fffffep-1f;

template <class SO>
__global__ __launch_bounds__(256) void joseph_fwd_f32_kernel(
    const float* __restrict__ x, const float* __restrict__ xT, SO* __restrict__ p,
    float* __restrict__ part, int n, int V, int B, const double* __restrict__ trig) {
  __shared__ __align__(16) float win[2 * kJfRows * kJosWin];
  __shared__ JosStep tab[3][kJfRows];
  const int tid = threadIdx.x;
  const int v = blockIdx.y;
  const int bfirst = blockIdx.x * 256, blast = min(B - 1, bfirst + 255);
  const int b = bfirst + tid;
  const double ct = trig[2 * v], st = trig[2 * v + 1];
  const bool rows = fabs(ct) >= fabs(st);
  const double a = rows ? ct : st, bb = rows ? st : ct;
  // blockIdx.z: column, or column and half of the steps on a split forward
  const int split = part ? 2 : 1;
  const int col = blockIdx.z / split, h = blockIdx.z - col * split;
  const float* img = (rows ? x : xT) + static_cast<size_t>(col) * n * n;
  const size_t orow = (static_cast<size_t>(col) * V + v) * B;
  const double c = 0.5 * (n - 1), half = 0.5 * (B - 1);
  const double ia = 1.0 / a;
  const double g = -bb * ia;
  // the bins of the block in the image's shadow (one bin of margin): a
  // sample at centred position (f - c, t - c) with |f - c| < c + 1 and
  // |t - c| <= c lies on rays with |s| < (c + 1)(|cos| + |sin|), so every
  // other bin is exactly zero
  const double shadow = (c + 1.0) * (fabs(ct) + fabs(st)) + 1.0;
  const int bs0 = max(bfirst, static_cast<int>(floor(half - shadow)));
  const int bs1 = min(blast, static_cast<int>(ceil(half + shadow)));
  if (bs0 > bs1) {   // the block's bins all miss the image
    if (b < B) {
      if (part) part[static_cast<size_t>(h) * (gridDim.z / split) * V * B + orow + b] = 0.f;
      else Io<SO>::st(p, orow + b, 0.f);
    }
    return;
  }
  // a wave samples only if some of its bins are in the shadow
  const bool live = bfirst + (tid & ~63) <= bs1 && bfirst + (tid | 63) >= bs0;
  const double fa0 = (bs0 - half) * ia + c, fb0 = (bs1 - half) * ia + c;
  const double lo0 = fmin(fa0, fb0), hi0 = fmax(fa0, fb0);
  int T0 = 0, T1 = n - 1;
  if (g != 0.0) {
    double ta = g > 0.0 ? (-1.0 - hi0) / g + c : (n - lo0) / g + c;
    double tb = g > 0.0 ? (n - lo0) / g + c : (-1.0 - hi0) / g + c;
    ta = fmin(fmax(ta, -2.0), n + 1.0);
    tb = fmin(fmax(tb, -2.0), n + 1.0);
    T0 = max(0, static_cast<int>(floor(ta)) - 1);
    T1 = min(n - 1, static_cast<int>(ceil(tb)) + 1);
  } else if (!(lo0 < n && hi0 >= -1.0)) {
    T1 = -1;
  }
  if (part) {   // this block's half of the stages
    const int nst = T0 <= T1 ? (T1 - T0 + kJfRows) / kJfRows : 0;
    const int mid = T0 + (nst + 1) / 2 * kJfRows;
    if (h == 0) T1 = min(T1, mid - 1);
    else T0 = mid;
  }
  // window: pixels [floor(lo) - 1, floor(hi) + 2] of a step and up to 3 of
  // alignment, floor(hi0 - lo0) + 8 at most (<= kJosWin for |a| >= 1/sqrt 2)
  const int w4 = min(kJosWin / 4, (static_cast<int>(hi0 - lo0) + 11) / 4);
  // the slots: (row, column) of each 16-byte load; (e + 1/2) / w4 is at least
  // 1 / (2 w4) away from an integer, far beyond the FP32 product's error
  const float inv_w4 = 1.0f / static_cast<float>(w4);
  // per slot: its row (kJfRows: idle), its column in the window, its row's
  // offset in the image and its place in an LDS buffer
  int sr[kJfSlots], sk[kJfSlots], srn[kJfSlots], sld[kJfSlots];
#pragma unroll
  for (int m = 0; m < kJfSlots; ++m) {
    const int e = tid + 256 * m;
    const int r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv_w4);
    sr[m] = min(r, kJfRows);
    sk[m] = 4 * (e - r * w4);
    srn[m] = sr[m] * n;
    sld[m] = sr[m] * kJosWin + sk[m];
  }
  // steps T .. T + kJfRows - 1 into table tb, window buffer wb
  auto params = [&](int T, int tb, int wb) {
    if (tid < kJfRows) {
      const int t = T + tid;
      const int base = jos_fwd_base(lo0, g, c, t);
      const double d = (t - c) * g - base;
      const double dw = floor(d);
      tab[tb][tid] = JosStep{fminf(static_cast<float>(d - dw), kJosBelowOne),
                             static_cast<int>(dw) + (wb * kJfRows + tid) * kJosWin, base,
                             t < n ? base : kJosNoRow};
    }
  };
  float4 q[kJfSlots];
  // one unsigned test per 16-byte group: a column outside [0, n) or a row
  // past the image (its load base is kJosNoRow) reads zeros
  auto load = [&](int T, int tb) {
    const int Tn = T * n;
#pragma unroll
    for (int m = 0; m < kJfSlots; ++m) {
      const int col = tab[tb][min(sr[m], kJfRows - 1)].lbase + sk[m];
      q[m] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (sr[m] < kJfRows && static_cast<unsigned>(col) < static_cast<unsigned>(n))
        q[m] = *reinterpret_cast<const float4*>(img + static_cast<unsigned>(Tn + srn[m] + col));
    }
  };
  auto store = [&](int wb) {
    float* wbuf = win + wb * kJfRows * kJosWin;
#pragma unroll
    for (int m = 0; m < kJfSlots; ++m)
      if (sr[m] < kJfRows) *reinterpret_cast<float4*>(wbuf + sld[m]) = q[m];
  };
  // the ray's own offset f0 = (b - (B - 1) / 2) / a + c, split (lanes off
  // the shadow take its nearest ray, which stays inside the windows)
  const double f0 = (min(max(b, bs0), bs1) - half) * ia + c;
  const double f0w = floor(f0);
  const int F0 = static_cast<int>(f0w);
  const float phi0 = fminf(static_cast<float>(f0 - f0w), kJosBelowOne);
  float acc = 0.f;
  if (T0 <= T1) {
    params(T0, 0, 0);
    params(T0 + kJfRows, 1, 1);
    __syncthreads();
    load(T0, 0);
    store(0);
    __syncthreads();
    for (int T = T0, wb = 0, tb = 0;; T += kJfRows, wb ^= 1, tb = jos_next3(tb)) {
      const int tn = jos_next3(tb);
      const bool more = T + kJfRows <= T1;
      if (more) load(T + kJfRows, tn);
      if (live) {
#pragma unroll
      for (int r = 0; r < kJfRows; ++r) {
        const JosStep e = tab[tb][r];
        const float w = phi0 + e.frac;                     // in [0, 2)
        const int k = F0 + e.whole + (w >= 1.f ? 1 : 0);   // LDS index of the left pixel
        const float wf = __builtin_amdgcn_fractf(w);
        const float a0 = win[k], a1 = win[k + 1];
        acc += fmaf(wf, a1 - a0, a0);
      }
      }
      if (more) {
        store(wb ^ 1);
        params(T + 2 * kJfRows, jos_next3(tn), wb);
      }
      __syncthreads();
      if (!more) break;
    }
  }
  if (b < B) {
    const float val = b >= bs0 && b <= bs1 ? acc * static_cast<float>(1.0 / fabs(a)) : 0.f;
    if (part) part[static_cast<size_t>(h) * (gridDim.z / split) * V * B + orow + b] = val;
    else Io<SO>::st(p, orow + b, val);
  }
}

// p = part[0] + part[1], the two halves of a split forward.
template <class SO>
__global__ __launch_bounds__(256) void joseph_fwd_join_kernel(const float* __restrict__ part,
                                                              SO* __restrict__ p, size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < count) Io<SO>::st(p, i, part[i] + part[i + count]);
}

// A forward on few columns leaves the last round of workgroups mostly
// idle; below this many workgroups its steps are split in two halves that
// write FP32 partial sums, joined by a second pass.
constexpr int64_t kJfSplitBelow = 3072;
inline int64_t jos_fwd_blocks(int V, int B, int64_t ncols) {
  return static_cast<int64_t>((B + 255) / 256) * V * ncols;
}
inline bool jos_fwd_split(int V, int B, int64_t ncols) {
  return jos_fwd_blocks(V, B, ncols) < kJfSplitBelow;
}
// The most columns, up to ncols, of a split forward: a workspace sized for
// ncols columns serves every call on fewer.
inline int64_t jos_fwd_split_cols(int V, int B, int64_t ncols) {
  return std::min<int64_t>(ncols, (kJfSplitBelow - 1) / jos_fwd_blocks(V, B, 1));
}

// Adjoint: a workgroup takes a 64 x 4 pixel tile (one wave per pixel row),
// kJaViews views per stage.  Pixel (i, j) has bin coordinate
// bc = (j - c) cos + (i - c) sin + (B - 1) / 2 on every view (either branch),
// and with bc = K + phi (K integer, 0 <= phi < 1) only bins K and K + 1 lie
// within |a| <= 1 of it, weighted (1 - phi / |a|) / |a| and
// (1 - (1 - phi) / |a|) / |a| (clamped at 0).  Per view and pixel row the
// FP64 coordinate of the row's first pixel relative to the window, plus the
// LDS offset of the window row, is split as hi + lo with hi a multiple of
// 2^-12 below 2^12, and cos as hi' + lo' likewise; then hi + dj hi' is exact
// in FP32 (under 2^24 units of 2^-12), its integer part is the LDS index of
// bin K, and its fraction plus lo + dj lo' (below 2^-7) is phi to a few 1e-7.
constexpr int kJaViews = 24;                                        // views per stage
constexpr int kJaSlots = (kJaViews * (kJosBins / 4) + 255) / 256;   // loads per thread per stage
static_assert(2 * kJaViews * kJosBins + 128 < 4096, "LDS offsets must stay below 2^12");
struct JosView {
  float4 w;     // 1/|a|, 1/a^2, 1/|a| - 1/a^2, 0 (all zero on a padding view)
  int base;     // first bin of the window (multiple of 4)
};

template <class SO>
__global__ __launch_bounds__(256) void joseph_adj_f32_kernel(
    const float* __restrict__ p, SO* __restrict__ x, int n, int V, int B,
    const double* __restrict__ trig) {
  __shared__ __align__(16) float win[2 * kJaViews * kJosBins];
  __shared__ float4 tabs[3][kJaViews][4];   // per pixel row: hi, lo, cos hi', cos lo'
  __shared__ JosView tabv[3][kJaViews];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.y * 4, j0 = blockIdx.x * 64;
  const int dj = tid & 63, di = tid >> 6;
  const int j = j0 + dj, i = i0 + di;
  const float* sino = p + static_cast<size_t>(blockIdx.z) * V * B;
  const double c = 0.5 * (n - 1), half = 0.5 * (B - 1);
  const int nstage = (V + kJaViews - 1) / kJaViews;
  // per-view terms of stage s (window buffer s & 1), by threads tid < kJaViews
  auto params = [&](int s, int tb) {
    if (tid < kJaViews) {
      const int v = s * kJaViews + tid;
      const int off = ((s & 1) * kJaViews + tid) * kJosBins;
      if (v < V) {
        const double ct = trig[2 * v], st = trig[2 * v + 1];
        const double aa = fmax(fabs(ct), fabs(st)), ia = 1.0 / aa;
        // lowest bin coordinate of the tile: at a corner
        const double bcmin = fmin((j0 - c) * ct, (j0 + 63 - c) * ct) +
                             fmin((i0 - c) * st, (i0 + 3 - c) * st) + half;
        const int base = (static_cast<int>(floor(bcmin)) - 1) & ~3;
        const double chi = nearbyint(ct * 4096.0) / 4096.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double s0 = (j0 - c) * ct + (i0 + r - c) * st + half - base + off;
          const double shi = nearbyint(s0 * 4096.0) / 4096.0;
          tabs[tb][tid][r] = make_float4(static_cast<float>(shi), static_cast<float>(s0 - shi),
                                         static_cast<float>(chi), static_cast<float>(ct - chi));
        }
        tabv[tb][tid] = JosView{make_float4(static_cast<float>(ia), static_cast<float>(ia * ia),
                                            static_cast<float>(ia - ia * ia), 0.f),
                                base};
      } else {
        // a padding view reads the start of its own (zero) window row
#pragma unroll
        for (int r = 0; r < 4; ++r)
          tabs[tb][tid][r] = make_float4(static_cast<float>(off), 0.f, 0.f, 0.f);
        tabv[tb][tid] = JosView{make_float4(0.f, 0.f, 0.f, 0.f), 0};
      }
    }
  };
  int sr[kJaSlots], sk[kJaSlots];
#pragma unroll
  for (int m = 0; m < kJaSlots; ++m) {
    const int e = tid + 256 * m;
    sr[m] = e / (kJosBins / 4);
    sk[m] = 4 * (e - sr[m] * (kJosBins / 4));
  }
  float4 q[kJaSlots];
  auto load = [&](int s, int tb) {
#pragma unroll
    for (int m = 0; m < kJaSlots; ++m) {
      const int v = s * kJaViews + sr[m];
      q[m] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (sr[m] < kJaViews && v < V) {
        const int col = tabv[tb][sr[m]].base + sk[m];
        if (col >= 0 && col < B)
          q[m] = *reinterpret_cast<const float4*>(sino + static_cast<size_t>(v) * B + col);
      }
    }
  };
  auto store = [&](int wb) {
#pragma unroll
    for (int m = 0; m < kJaSlots; ++m)
      if (sr[m] < kJaViews)
        *reinterpret_cast<float4*>(&win[(wb * kJaViews + sr[m]) * kJosBins + sk[m]]) = q[m];
  };
  const float djf = static_cast<float>(dj);
  float acc = 0.f;
  params(0, 0);
  params(1, 1);
  __syncthreads();
  load(0, 0);
  store(0);
  __syncthreads();
  for (int s = 0, wb = 0, tb = 0;; ++s, wb ^= 1, tb = jos_next3(tb)) {
    const int tn = jos_next3(tb);
    const bool more = s + 1 < nstage;
    if (more) load(s + 1, tn);
#pragma unroll 8
    for (int r = 0; r < kJaViews; ++r) {
      const float4 sv = tabs[tb][r][di];
      const float4 w = tabv[tb][r].w;
      const float S = fmaf(djf, sv.z, sv.x);   // exact
      const float fl = floorf(S);
      float ph = (S - fl) + fmaf(djf, sv.w, sv.y);
      const float f2 = floorf(ph);
      ph -= f2;
      const int k = static_cast<int>(fl + f2);   // LDS index of bin K
      const float x0 = win[k], x1 = win[k + 1];
      acc = fmaf(fmaxf(fmaf(-ph, w.y, w.x), 0.f), x0, acc);
      acc = fmaf(fmaxf(fmaf(ph, w.y, w.z), 0.f), x1, acc);
    }
    if (more) {
      store(wb ^ 1);
      params(s + 2, jos_next3(tn));   // zeros past the last view
    }
    __syncthreads();
    if (!more) break;
  }
  if (i < n && j < n)
    Io<SO>::st(x, static_cast<size_t>(blockIdx.z) * n * n + static_cast<size_t>(i) * n + j, acc);
}

// ================================================================ launchers
template <class C> const C* psf_ptr(const nys_op_s* op, bool flipped);
template <> const double* psf_ptr<double>(const nys_op_s* op, bool flipped) {
  int kk = op->d.psf_size * op->d.psf_size;
  return op->psf_dev.as<double>() + (flipped ? 0 : kk);
}
template <> const float* psf_ptr<float>(const nys_op_s* op, bool flipped) {
  int kk = op->d.psf_size * op->d.psf_size;
  return reinterpret_cast<const float*>(op->psf_dev.as<double>() + 2 * kk) + (flipped ? 0 : kk);
}
// trig layout: cos, sin per view (FP64), then 1 / |a| per view (FP64), then
// the same two tables in FP32.
template <class C> const C* trig_ptr(const nys_op_s* op);
template <> const double* trig_ptr<double>(const nys_op_s* op) { return op->trig.as<double>(); }
template <> const float* trig_ptr<float>(const nys_op_s* op) {
  return reinterpret_cast<const float*>(op->trig.as<double>() + 3 * op->d.n_views);
}
template <class C> const C* inva_ptr(const nys_op_s* op) {
  return trig_ptr<C>(op) + 2 * op->d.n_views;
}

// ================================================================ fused forward
// psi(A W^T x - y) for the blur and blur-decimation operators, W^T the Haar
// synthesis of L levels (L = 0: x is the image), in one kernel.  A workgroup
// takes a kFwdTH x kFwdTW tile of the output grid: it synthesises the
// 2^L x 2^L coefficient blocks that cover the tile's input window (periodic,
// B = 2^L lanes a block as in haar_kernel) into LDS, correlates them with the
// flipped PSF at stride f (the same sums in the same order as
// correlate_kernel), and applies the loss derivative of residual_kernel
// (yobs null: the plain forward).
constexpr int kFwdTH = 8, kFwdTW = 32;

__host__ __device__ inline int fwd_win_blocks(int f, int T, int k, int B) {
  return (f * (T - 1) + k + B - 1) / B + 1;   // blocks covering any window of that length
}

template <int L, class T>
__global__ __launch_bounds__(256) void blur_fwd_fused_kernel(
    const T* __restrict__ x, T* __restrict__ out, const T* __restrict__ g, int k, int n1, int n2,
    int o1, int o2, int f, const T* __restrict__ yobs, int loss, T delta) {
  constexpr int B = 1 << L;
  extern __shared__ unsigned char smem_raw[];
  T* sg = reinterpret_cast<T*>(smem_raw);
  T* win = sg + k * k;
  const int c = (k - 1) / 2;
  const int i0 = blockIdx.y * kFwdTH, j0 = blockIdx.x * kFwdTW;
  const int nbr_max = fwd_win_blocks(f, kFwdTH, k, B), nbc_max = fwd_win_blocks(f, kFwdTW, k, B);
  const int LW = nbc_max * B;   // LDS row length
  // block range of the input window [f i0 - c, f (i0 + TH - 1) - c + k - 1]
  const int bR0 = floor_div(f * i0 - c, B), bC0 = floor_div(f * j0 - c, B);
  const int nbr = floor_div(f * (i0 + kFwdTH - 1) - c + k - 1, B) - bR0 + 1;
  const int nbc = floor_div(f * (j0 + kFwdTW - 1) - c + k - 1, B) - bC0 + 1;
  const size_t plane = static_cast<size_t>(n1) * n2;
  const T* src = x + static_cast<size_t>(blockIdx.z) * plane;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) sg[t] = g[t];
  const int nb1 = n1 / B, nb2 = n2 / B;
  const int ntask = nbr * nbc * B;
  for (int t0 = 0; t0 < ntask; t0 += blockDim.x) {
    const int task = t0 + threadIdx.x;
    const bool live = task < ntask;
    const int blk = live ? task / B : 0, r = task % B;
    const int lbr = blk / nbc, lbc = blk - lbr * nbc;
    int gbr = (bR0 + lbr) % nb1; if (gbr < 0) gbr += nb1;
    int gbc = (bC0 + lbc) % nb2; if (gbc < 0) gbc += nb2;
    const T* rowp = src + static_cast<size_t>(gbr * B + r) * n2 + gbc * B;
    T v[B];
#pragma unroll
    for (int q = 0; q < B; ++q) v[q] = live ? rowp[q] : T(0);
#pragma unroll
    for (int it = 0; it < L; ++it) {
      const int s = 1 << (L - 1 - it);   // synthesis: coarsest level first
      const bool part = (r & (s - 1)) == 0;
      const bool top = (r & s) == 0;
#pragma unroll
      for (int q = 0; q < B; q += 2 * s) {
        const T e0 = __shfl_xor(v[q], s, B), e1 = __shfl_xor(v[q + s], s, B);
        const T a = top ? v[q] : e0, b = top ? v[q + s] : e1;
        const T cc = top ? e0 : v[q], d = top ? e1 : v[q + s];
        if (part) {
          v[q] = top ? (a + b + cc + d) * T(0.5) : (a + b - cc - d) * T(0.5);
          v[q + s] = top ? (a - b + cc - d) * T(0.5) : (a - b - cc + d) * T(0.5);
        }
      }
    }
    if (live) {
      T* wrow = win + static_cast<size_t>(lbr * B + r) * LW + lbc * B;
#pragma unroll
      for (int q = 0; q < B; ++q) wrow[q] = v[q];
    }
  }
  __syncthreads();
  const int ty = threadIdx.x / kFwdTW, tx = threadIdx.x % kFwdTW;
  const int oi = i0 + ty, oj = j0 + tx;
  if (oi >= o1 || oj >= o2) return;
  // window coordinates of the output's first tap
  const int ly = f * oi - c - bR0 * B, lx = f * oj - c - bC0 * B;
  T acc = 0;
  for (int a = 0; a < k; ++a) {
    const T* row = win + static_cast<size_t>(ly + a) * LW + lx;
    const T* grow = sg + a * k;
    for (int b = 0; b < k; ++b) acc += grow[b] * row[b];
  }
  const size_t oidx = static_cast<size_t>(blockIdx.z) * o1 * o2 + static_cast<size_t>(oi) * o2 + oj;
  if (yobs != nullptr) {
    T v = acc - yobs[oidx];
    if (loss == NYS_LOSS_HUBER) v = fmin(T(1), fmax(T(-1), v / delta));
    acc = v;
  }
  out[oidx] = acc;
}

template <class T>
bool op_fwd_fused_ok(nys_op op) {
  const auto& d = op->d;
  if (d.kind != NYS_OP_BLUR && d.kind != NYS_OP_BLURDOWN) return false;
  if (d.wavelet_levels > 0 && d.wavelet != NYS_WAVELET_HAAR) return false;
  const int B = 1 << d.wavelet_levels;
  const int f = d.kind == NYS_OP_BLURDOWN ? d.factor : 1;
  return d.wavelet_levels >= 0 && d.wavelet_levels <= 3 && d.n1 % B == 0 && d.n2 % B == 0 &&
         d.n1 % f == 0 && d.n2 % f == 0;
}

template <class T>
nys_status op_fwd_psi(nys_op op, const T* x, const T* yobs, int loss, double delta, T* out,
                      int64_t ncols, hipStream_t st) {
  const auto& d = op->d;
  const int k = d.psf_size, L = d.wavelet_levels, B = 1 << L;
  const int f = d.kind == NYS_OP_BLURDOWN ? d.factor : 1;
  const int o1 = d.n1 / f, o2 = d.n2 / f;
  const size_t sm = sizeof(T) * (static_cast<size_t>(k) * k +
                                 static_cast<size_t>(fwd_win_blocks(f, kFwdTH, k, B) * B) *
                                     (fwd_win_blocks(f, kFwdTW, k, B) * B));
  dim3 grid(cdiv(o2, kFwdTW), cdiv(o1, kFwdTH), static_cast<unsigned>(ncols));
#define NYS_FWD_FUSED(LL)                                                                          \
  do {                                                                                             \
    if (sm > 64 * 1024)                                                                            \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&blur_fwd_fused_kernel<LL, T>),      \
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sm)); \
    hipLaunchKernelGGL((blur_fwd_fused_kernel<LL, T>), grid, dim3(256), sm, st, x, out,            \
                       psf_ptr<T>(op, true), k, d.n1, d.n2, o1, o2, f, yobs, loss,                 \
                       static_cast<T>(delta));                                                     \
  } while (0)
  switch (L) {
    case 0: NYS_FWD_FUSED(0); break;
    case 1: NYS_FWD_FUSED(1); break;
    case 2: NYS_FWD_FUSED(2); break;
    default: NYS_FWD_FUSED(3); break;
  }
#undef NYS_FWD_FUSED
  return launch_check("blur_fwd_fused_kernel");
}

template bool op_fwd_fused_ok<float>(nys_op);
template bool op_fwd_fused_ok<double>(nys_op);
template nys_status op_fwd_psi<float>(nys_op, const float*, const float*, int, double, float*,
                                      int64_t, hipStream_t);
template nys_status op_fwd_psi<double>(nys_op, const double*, const double*, int, double,
                                       double*, int64_t, hipStream_t);

template <class SI, class SO, class C>
static nys_status launch_correlate(const nys_op_s* op, const SI* in, SO* out, bool flipped,
                                   int n1, int n2, int f, int64_t ncols, hipStream_t st) {
  const int k = op->d.psf_size;
  const int o1 = n1 / f, o2 = n2 / f;
  // 16-row tiles when that still gives >= 512 workgroups, else 4-row tiles
  const bool tall = static_cast<int64_t>(cdiv(o2, kCorTW)) * cdiv(o1, 16) * ncols >= 512;
  const int TH = tall ? 16 : 4;
  dim3 grid(cdiv(o2, kCorTW), cdiv(o1, TH), static_cast<unsigned>(ncols));
  size_t sm = sizeof(C) * (k * k + (f * (TH - 1) + k) * (f * (kCorTW - 1) + k));
  if (tall)
    hipLaunchKernelGGL((correlate_kernel<SI, SO, C, 16>), grid, dim3(256), sm, st, in, out,
                       psf_ptr<C>(op, flipped), k, n1, n2, o1, o2, f);
  else
    hipLaunchKernelGGL((correlate_kernel<SI, SO, C, 4>), grid, dim3(256), sm, st, in, out,
                       psf_ptr<C>(op, flipped), k, n1, n2, o1, o2, f);
  return launch_check("correlate_kernel");
}

template <class SI, class SO, class C>
static nys_status launch_upcorrelate(const nys_op_s* op, const SI* in, SO* out, int m1,
                                     int m2, int f, int64_t ncols, hipStream_t st) {
  const int k = op->d.psf_size;
  const int n1 = m1 * f, n2 = m2 * f;
  // 32-row tiles when that still gives >= 512 workgroups, else 8-row tiles
  const bool tall = static_cast<int64_t>(cdiv(n2, kUpTW)) * cdiv(n1, 32) * ncols >= 512;
  const int TH = tall ? 32 : 8;
  dim3 grid(cdiv(n2, kUpTW), cdiv(n1, TH), static_cast<unsigned>(ncols));
  int th = (TH - 1 + k - 1) / f + 2, tw = (kUpTW - 1 + k - 1) / f + 2;
  size_t sm = sizeof(C) * (k * k + th * tw);
  if (tall)
    hipLaunchKernelGGL((upcorrelate_kernel<SI, SO, C, 32>), grid, dim3(256), sm, st, in, out,
                       psf_ptr<C>(op, false), k, m1, m2, f);
  else
    hipLaunchKernelGGL((upcorrelate_kernel<SI, SO, C, 8>), grid, dim3(256), sm, st, in, out,
                       psf_ptr<C>(op, false), k, m1, m2, f);
  return launch_check("upcorrelate_kernel");
}

template <bool kAnalysis, class SI, class SO, class C>
static nys_status launch_haar(int levels, const SI* in, SO* out, int n1, int n2, int64_t ncols,
                              hipStream_t st) {
  const int B = 1 << levels;
  const int64_t lanes = static_cast<int64_t>(n1 / B) * (n2 / B) * B;   // B lanes per block
  dim3 grid(cdiv(lanes, 256), 1, static_cast<unsigned>(ncols));
  switch (levels) {
    case 1: hipLaunchKernelGGL((haar_kernel<1, kAnalysis, SI, SO, C>), grid, dim3(256), 0, st, in, out, n1, n2); break;
    case 2: hipLaunchKernelGGL((haar_kernel<2, kAnalysis, SI, SO, C>), grid, dim3(256), 0, st, in, out, n1, n2); break;
    case 3: hipLaunchKernelGGL((haar_kernel<3, kAnalysis, SI, SO, C>), grid, dim3(256), 0, st, in, out, n1, n2); break;
    default: set_error("wavelet levels must be 1..3"); return NYS_EINVAL;
  }
  return launch_check("haar_kernel");
}

// ================================================================ Daubechies-4
// One pass of the periodised two-channel filter bank over the top-left
// m1 x m2 band (row pitch n2), along rows (kRows) or columns, one thread per
// output value.  Analysis: a_i = sum_k h_k x[(2i + k) mod m], d_i with g,
// a in the first half of the line and d in the second.  Synthesis (the
// transpose): x_j = sum over k with j - k even of h_k a_{((j - k) mod m) / 2}
// + g_k d_{((j - k) mod m) / 2}.
template <bool kAnalysis, bool kRows, class TI, class TO, class C>
__global__ __launch_bounds__(256) void db4_pass_kernel(const TI* __restrict__ in, TO* __restrict__ out,
                                                       int n1, int n2, int m1, int m2, Db4Coef f) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);   // column in the band
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);    // row in the band
  if (i >= m1 || j >= m2) return;
  const size_t plane = static_cast<size_t>(n1) * n2;
  const TI* src = in + blockIdx.z * plane;
  const int m = kRows ? m2 : m1, t = kRows ? j : i;     // length and position along the line
  auto at = [&](int q) -> C {                            // line element q
    return kRows ? static_cast<C>(Io<TI>::ld(src, static_cast<size_t>(i) * n2 + q))
                 : static_cast<C>(Io<TI>::ld(src, static_cast<size_t>(q) * n2 + j));
  };
  const C* h = std::is_same<C, double>::value ? reinterpret_cast<const C*>(f.hd) : reinterpret_cast<const C*>(f.hf);
  const C* g = std::is_same<C, double>::value ? reinterpret_cast<const C*>(f.gd) : reinterpret_cast<const C*>(f.gf);
  C acc = 0;
  const int half = m / 2;
  if (kAnalysis) {
    const bool detail = t >= half;
    const int b = 2 * (detail ? t - half : t);
    const C* w = detail ? g : h;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += w[k] * at((b + k) % m);
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (((t - k) & 1) != 0) continue;
      int q = (t - k) % m;
      if (q < 0) q += m;
      const int idx = q / 2;
      acc += h[k] * at(idx) + g[k] * at(half + idx);
    }
  }
  Io<TO>::st(out + blockIdx.z * plane, static_cast<size_t>(i) * n2 + j, acc);
}

template <class TI, class TO>
__global__ void convert_kernel(const TI* __restrict__ in, TO* __restrict__ out, size_t n) {
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<size_t>(gridDim.x) * blockDim.x)
    Io<TO>::st(out, e, static_cast<typename Io<TO>::C>(Io<TI>::ld(in, e)));
}

// W x (analysis) or W^T x (synthesis) with `levels` Daubechies-4 levels.  The
// passes go through scratch; every level works on `work` (C values: out
// itself when SO is C, else a second buffer converted into out once at the
// end, so a narrow output is rounded only once).  scratch and work each hold
// n1 n2 ncols values.
template <bool kAnalysis, class SI, class SO, class C>
static nys_status launch_db4(const nys_op_s* op, int levels, const SI* in, SO* out, C* scratch,
                             C* work_buf, int n1, int n2, int64_t ncols, hipStream_t st) {
  const Db4Coef& f = op->db4;
  const size_t n = static_cast<size_t>(n1) * n2 * ncols;
  const dim3 cgrid(std::min<size_t>(cdiv(n, 256), 4096));
  constexpr bool kSame = std::is_same<SO, C>::value;
  C* work = kSame ? reinterpret_cast<C*>(out) : work_buf;
  auto grid = [&](int m1, int m2) { return dim3(cdiv(m2, 64), cdiv(m1, 4), static_cast<unsigned>(ncols)); };
  if (kAnalysis) {
    // level 0 reads the input; later levels read work's LL band
    hipLaunchKernelGGL((db4_pass_kernel<true, true, SI, C, C>), grid(n1, n2), dim3(256), 0, st, in,
                       scratch, n1, n2, n1, n2, f);
    hipLaunchKernelGGL((db4_pass_kernel<true, false, C, C, C>), grid(n1, n2), dim3(256), 0, st,
                       scratch, work, n1, n2, n1, n2, f);
    for (int lev = 1; lev < levels; ++lev) {
      const int m1 = n1 >> lev, m2 = n2 >> lev;
      hipLaunchKernelGGL((db4_pass_kernel<true, true, C, C, C>), grid(m1, m2), dim3(256), 0, st,
                         work, scratch, n1, n2, m1, m2, f);
      hipLaunchKernelGGL((db4_pass_kernel<true, false, C, C, C>), grid(m1, m2), dim3(256), 0, st,
                         scratch, work, n1, n2, m1, m2, f);
    }
  } else {
    // work = in, then the levels coarsest first, columns then rows
    hipLaunchKernelGGL((convert_kernel<SI, C>), cgrid, dim3(256), 0, st, in, work, n);
    for (int lev = levels - 1; lev >= 0; --lev) {
      const int m1 = n1 >> lev, m2 = n2 >> lev;
      hipLaunchKernelGGL((db4_pass_kernel<false, false, C, C, C>), grid(m1, m2), dim3(256), 0, st,
                         work, scratch, n1, n2, m1, m2, f);
      hipLaunchKernelGGL((db4_pass_kernel<false, true, C, C, C>), grid(m1, m2), dim3(256), 0, st,
                         scratch, work, n1, n2, m1, m2, f);
    }
  }
  if (!kSame) hipLaunchKernelGGL((convert_kernel<C, SO>), cgrid, dim3(256), 0, st, work, out, n);
  return launch_check("db4_pass_kernel");
}

// The wavelet of the operator: Haar (haar_kernel) or Daubechies-4.
template <bool kAnalysis, class SI, class SO, class C>
static nys_status launch_wavelet(nys_op_s* op, const SI* in, SO* out, int64_t ncols,
                                 hipStream_t st) {
  const auto& d = op->d;
  if (d.wavelet != NYS_WAVELET_DB4)
    return launch_haar<kAnalysis, SI, SO, C>(d.wavelet_levels, in, out, d.n1, d.n2, ncols, st);
  const size_t n = static_cast<size_t>(d.n1) * d.n2 * ncols;
  Scratch::Mark mark(op->scr);
  C* scratch = nullptr;
  C* work = nullptr;
  NYS_TAKE(op->scr, C, scratch, n);
  if (!std::is_same<SO, C>::value) NYS_TAKE(op->scr, C, work, n);
  return launch_db4<kAnalysis, SI, SO, C>(op, d.wavelet_levels, in, out, scratch, work, d.n1,
                                          d.n2, ncols, st);
}

// Filters of the Daubechies-4 wavelet by spectral factorisation (host, FP64):
// |H|^2 = 2 cos^8(w/2) Q(sin^2(w/2)), Q(y) = 1 + 4y + 10y^2 + 20y^3; the
// roots of Q (Durand-Kerner iteration) give z from z^2 - (2 - 4y) z + 1 = 0,
// the root inside the unit circle is kept, h(z) is proportional to
// (z + 1)^4 prod (z - z_j) (coefficients from the highest power down),
// normalised to a sum of sqrt(2).
static Db4Coef db4_filters() {
  using cd = std::complex<double>;
  const double q[4] = {1.0 / 20.0, 4.0 / 20.0, 10.0 / 20.0, 1.0};   // monic, y^0 .. y^3
  cd r[3] = {cd(0.4, 0.9), cd(0.4, 0.9) * cd(0.4, 0.9), cd(0.4, 0.9) * cd(0.4, 0.9) * cd(0.4, 0.9)};
  for (int it = 0; it < 500; ++it) {
    for (int a = 0; a < 3; ++a) {
      cd num = q[3];
      for (int c = 2; c >= 0; --c) num = num * r[a] + q[c];
      cd den = 1.0;
      for (int b = 0; b < 3; ++b)
        if (b != a) den *= (r[a] - r[b]);
      r[a] -= num / den;
    }
  }
  std::vector<cd> poly{cd(1.0)};
  auto mul = [&](cd c0, cd c1) {   // poly *= (c0 z + c1), highest power first
    std::vector<cd> out(poly.size() + 1, cd(0.0));
    for (size_t t = 0; t < poly.size(); ++t) {
      out[t] += poly[t] * c0;
      out[t + 1] += poly[t] * c1;
    }
    poly.swap(out);
  };
  for (int t = 0; t < 4; ++t) mul(cd(1.0), cd(1.0));
  for (int a = 0; a < 3; ++a) {
    const cd b = 1.0 - 2.0 * r[a];
    const cd disc = std::sqrt(b * b - 1.0);
    const cd z1 = b + disc, z2 = b - disc;
    mul(cd(1.0), -(std::abs(z1) < 1.0 ? z1 : z2));
  }
  Db4Coef f{};
  double sum = 0;
  for (int k = 0; k < 8; ++k) sum += poly[k].real();
  for (int k = 0; k < 8; ++k) f.hd[k] = poly[k].real() * (std::sqrt(2.0) / sum);
  for (int k = 0; k < 8; ++k) f.gd[k] = ((k & 1) ? -1.0 : 1.0) * f.hd[7 - k];
  for (int k = 0; k < 8; ++k) {
    f.hf[k] = static_cast<float>(f.hd[k]);
    f.gf[k] = static_cast<float>(f.gd[k]);
  }
  return f;
}

template <class SI, class SO, class C>
static nys_status launch_joseph_fwd(const nys_op_s* op, const SI* x, SO* p, int64_t ncols,
                                    hipStream_t st) {
  const int n = op->d.n1, V = op->d.n_views, B = op->d.n_bins;
  Scratch::Mark mark(op->scr);
  SI* xT = nullptr;
  NYS_TAKE(op->scr, SI, xT, static_cast<size_t>(n) * n * ncols);
  hipLaunchKernelGGL((transpose_kernel<SI>), dim3(cdiv(n, 32), cdiv(n, 32), static_cast<unsigned>(ncols)),
                     dim3(256), 0, st, x, xT, n);
  NYS_TRY(launch_check("transpose_kernel"));
  dim3 grid(cdiv(B, 256), V, static_cast<unsigned>(ncols));
  if constexpr (std::is_same<SI, float>::value) {
    // 16-byte row loads need 16-byte aligned rows of both images
    if (n % 4 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(xT) % 16 == 0) {
      if constexpr (std::is_same<C, float>::value) {
        float* part = nullptr;
        if (jos_fwd_split(V, B, ncols)) {
          NYS_TAKE(op->scr, float, part, 2 * ncols * V * B);
          grid.z *= 2;
        }
        hipLaunchKernelGGL((joseph_fwd_f32_kernel<SO>), grid, dim3(256), 0, st, x, xT, p, part, n,
                           V, B, trig_ptr<double>(op));
        NYS_TRY(launch_check("joseph_fwd_f32_kernel"));
        if (part) {
          const size_t count = static_cast<size_t>(ncols) * V * B;
          hipLaunchKernelGGL((joseph_fwd_join_kernel<SO>),
                             dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, st,
                             part, p, count);
          NYS_TRY(launch_check("joseph_fwd_join_kernel"));
        }
        return NYS_OK;
      } else {
        hipLaunchKernelGGL((joseph_fwd_lds_kernel<SI, SO, C, true>), grid, dim3(256), 0, st, x, xT,
                           p, n, V, B, trig_ptr<double>(op));
        return launch_check("joseph_fwd_lds_kernel");
      }
    }
  }
  hipLaunchKernelGGL((joseph_fwd_lds_kernel<SI, SO, C, false>), grid, dim3(256), 0, st, x, xT, p,
                     n, V, B, trig_ptr<double>(op));
  return launch_check("joseph_fwd_lds_kernel");
}

template <class SI, class SO, class C>
static nys_status launch_joseph_adj(const nys_op_s* op, const SI* p, SO* x, int64_t ncols,
                                    hipStream_t st) {
  const int n = op->d.n1, V = op->d.n_views, B = op->d.n_bins;
  dim3 grid(cdiv(n, 64), cdiv(n, 4), static_cast<unsigned>(ncols));
  if constexpr (std::is_same<SI, float>::value) {
    if (B % 4 == 0 && reinterpret_cast<uintptr_t>(p) % 16 == 0) {
      if constexpr (std::is_same<C, float>::value) {
        hipLaunchKernelGGL((joseph_adj_f32_kernel<SO>), grid, dim3(256), 0, st, p, x, n, V, B,
                           trig_ptr<double>(op));
        return launch_check("joseph_adj_f32_kernel");
      } else {
        hipLaunchKernelGGL((joseph_adj_lds_kernel<SI, SO, C, true>), grid, dim3(256), 0, st, p, x, n,
                           V, B, trig_ptr<double>(op), inva_ptr<double>(op));
        return launch_check("joseph_adj_lds_kernel");
      }
    }
  }
  hipLaunchKernelGGL((joseph_adj_lds_kernel<SI, SO, C, false>), grid, dim3(256), 0, st, p, x, n, V,
                     B, trig_ptr<double>(op), inva_ptr<double>(op));
  return launch_check("joseph_adj_lds_kernel");
}

// ================================================================ fan beam
template <class T> nys_status fill_zero(T* p, size_t n, hipStream_t st);   // prox.hip

// The ray (view v, bin b) as the line cs x + sn y = s (FP64): normal
// proportional to (R_s + R_d) e - u d0 with e = (cos, sin), d0 = (-sin, cos)
// of theta = 2 pi v / V, s = u R_s / |.|.
__device__ __forceinline__ void fan_ray(int v, int b, int V, int B, double src, double det,
                                        double du, double& cs, double& sn, double& s) {
  const double th = 2.0 * M_PI * v / V;
  const double ce = cos(th), se = sin(th);
  const double u = (b - 0.5 * (B - 1)) * du;
  const double Rt = src + det;
  const double nrm = sqrt(Rt * Rt + u * u);
  cs = (Rt * ce + u * se) / nrm;
  sn = (Rt * se - u * ce) / nrm;
  s = u * src / nrm;
}

// Joseph sampling of one line: the stepped index range and, per step t, the
// interpolation coordinate f0 + (t - c) g along the other axis.
__device__ __forceinline__ void fan_steps(double cs, double sn, double s, int n, bool& rows,
                                          double& f0, double& g, double& scale, int& t0, int& t1) {
  rows = fabs(cs) >= fabs(sn);
  const double a = rows ? cs : sn, bb = rows ? sn : cs;
  const double c = 0.5 * (n - 1);
  f0 = s / a + c;
  g = -bb / a;
  scale = 1.0 / fabs(a);
  t0 = 0;
  t1 = n - 1;
  if (g != 0.0) {
    double ta = (-1.0 - f0) / g + c, tb = (n - f0) / g + c;
    if (ta > tb) { const double tt = ta; ta = tb; tb = tt; }
    ta = fmin(fmax(ta, -2.0), n + 1.0);
    tb = fmin(fmax(tb, -2.0), n + 1.0);
    t0 = max(0, static_cast<int>(floor(ta)) - 1);
    t1 = min(n - 1, static_cast<int>(ceil(tb)) + 1);
  } else if (!(f0 >= -1.0 && f0 < n)) {
    t1 = -1;
  }
}

// Lanes per ray (forward) and per pixel (gathered transpose): each takes a
// contiguous share of the ray's steps (every kFanAdjSeg-th view), summed by
// shuffles.
constexpr int kFanSeg = 32;
constexpr int kFanAdjSeg = 2;

template <class SI, class SO, class C>
__global__ __launch_bounds__(256) void fan_fwd_kernel(const SI* __restrict__ x, SO* __restrict__ p,
                                                      int n, int V, int B, double src, double det,
                                                      double du) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = gid / kFanSeg, seg = gid % kFanSeg;   // a ray's lanes share a wave
  const int v = blockIdx.y;
  const bool valid = b < B;
  double cs = 1.0, sn = 0.0, s = 0.0, f0 = 0.0, g = 0.0, scale = 0.0;
  bool rows = true;
  int t0 = 0, t1 = -1;
  if (valid) {
    fan_ray(v, b, V, B, src, det, du, cs, sn, s);
    fan_steps(cs, sn, s, n, rows, f0, g, scale, t0, t1);
  }
  const int chunk = (t1 - t0 + kFanSeg) / kFanSeg;   // ceil(len / kFanSeg), len >= 0
  const int ta = t0 + seg * chunk, tb = min(t1, ta + chunk - 1);
  const SI* img = x + static_cast<size_t>(blockIdx.z) * n * n;
  const double c = 0.5 * (n - 1);
  C acc = 0;
  for (int t = ta; t <= tb; ++t) {
    const double f = f0 + (t - c) * g;
    const double fl = floor(f);
    const int q = static_cast<int>(fl);
    const C w = static_cast<C>(f - fl);
    const int qa = min(max(q, 0), n - 1), qb = min(max(q + 1, 0), n - 1);
    const C lo = Io<SI>::ld(img, rows ? static_cast<size_t>(t) * n + qa : static_cast<size_t>(qa) * n + t);
    const C hi = Io<SI>::ld(img, rows ? static_cast<size_t>(t) * n + qb : static_cast<size_t>(qb) * n + t);
    if (q >= 0 && q < n) acc += (C(1) - w) * lo;
    if (q + 1 >= 0 && q + 1 < n) acc += w * hi;
  }
  for (int o = kFanSeg / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kFanSeg);
  if (valid && seg == 0)
    Io<SO>::st(p, (static_cast<size_t>(blockIdx.z) * V + v) * B + b, static_cast<C>(scale) * acc);
}

// x += A^T p ray by ray (x zeroed by the caller): the forward's samples,
// scattered with atomic additions.
template <class SI, class C>
__global__ __launch_bounds__(256) void fan_adj_kernel(const SI* __restrict__ p, C* __restrict__ x,
                                                      int n, int V, int B, double src, double det,
                                                      double du) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (b >= B) return;
  double cs, sn, s, f0, g, scale;
  fan_ray(v, b, V, B, src, det, du, cs, sn, s);
  bool rows;
  int t0, t1;
  fan_steps(cs, sn, s, n, rows, f0, g, scale, t0, t1);
  const C val = static_cast<C>(scale) *
                static_cast<C>(Io<SI>::ld(p, (static_cast<size_t>(blockIdx.z) * V + v) * B + b));
  if (val == C(0)) return;
  C* img = x + static_cast<size_t>(blockIdx.z) * n * n;
  const double c = 0.5 * (n - 1);
  for (int t = t0; t <= t1; ++t) {
    const double f = f0 + (t - c) * g;
    const double fl = floor(f);
    const int q = static_cast<int>(fl);
    const C w = static_cast<C>(f - fl);
    if (q >= 0 && q < n)
      atomicAdd(img + (rows ? static_cast<size_t>(t) * n + q : static_cast<size_t>(q) * n + t),
                (C(1) - w) * val);
    if (q + 1 >= 0 && q + 1 < n)
      atomicAdd(img + (rows ? static_cast<size_t>(t) * n + q + 1 : static_cast<size_t>(q + 1) * n + t),
                w * val);
  }
}

// Ray table for the gathered adjoint (one thread per ray, plus the per-view
// trigonometry from the rays of bin 0).
__global__ __launch_bounds__(256) void fan_table_kernel(double* __restrict__ tab, int n, int V,
                                                        int B, double src, double det, double du) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V * B) return;
  const int v = r / B, b = r - v * B;
  double cs, sn, s, f0, g, scale;
  fan_ray(v, b, V, B, src, det, du, cs, sn, s);
  bool rows;
  int t0, t1;
  fan_steps(cs, sn, s, n, rows, f0, g, scale, t0, t1);
  double* e = tab + 2 * static_cast<size_t>(V) + 3 * static_cast<size_t>(r);
  e[0] = f0;
  e[1] = g;
  e[2] = rows ? scale : -scale;
  if (b == 0) {
    const double th = 2.0 * M_PI * v / V;
    tab[2 * v] = cos(th);
    tab[2 * v + 1] = sin(th);
  }
}

// Fractional bin of the ray from the source through the point (X, Y) (offsets
// from the image centre, X along columns): the source is at -src d0 and the
// detector at det d0, d0 = (-sin, cos), bins along e = (cos, sin).
__device__ __forceinline__ double fan_bin(double X, double Y, double ce, double se, double Rt,
                                          double src, double inv_du, double half) {
  return Rt * (X * ce + Y * se) / (src + (Y * ce - X * se)) * inv_du + half;
}

// x = A^T p gathered pixel by pixel (source outside the image's circumscribed
// circle).  A ray stepping along rows samples pixel (i, j) at its step t = i
// iff it crosses row i within one pixel of column j; the rays from the source
// through that two-pixel segment are a bin interval (the bin of a point is
// monotone along any segment that misses the source).  Likewise for rays
// stepping along columns and the column segment.  Every candidate repeats the
// forward's own sample, so the weights are the transpose's.
template <class SI, class SO, class C>
__global__ __launch_bounds__(256) void fan_adj_gather_kernel(
    const SI* __restrict__ p, SO* __restrict__ x, const double* __restrict__ tab, int n, int V,
    int B, double src, double det, double du) {
  const int64_t gid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t pix = gid / kFanAdjSeg;   // a pixel's lanes share a wave
  const int vs = static_cast<int>(gid % kFanAdjSeg);
  const bool valid = pix < static_cast<int64_t>(n) * n;
  const int i = valid ? static_cast<int>(pix / n) : 0, j = valid ? static_cast<int>(pix % n) : 0;
  const double c = 0.5 * (n - 1), half = 0.5 * (B - 1), inv_du = 1.0 / du, Rt = src + det;
  const double X = j - c, Y = i - c;
  const SI* pz = p + static_cast<size_t>(blockIdx.y) * V * B;
  const double* rays = tab + 2 * static_cast<size_t>(V);
  C acc = 0;
  for (int v = valid ? vs : V; v < V; v += kFanAdjSeg) {
    const double ce = tab[2 * v], se = tab[2 * v + 1];
    const SI* pv = pz + static_cast<size_t>(v) * B;
    const double* rv = rays + 3 * static_cast<size_t>(v) * B;
    // rays stepping along rows, through the segment of row i
    {
      const double b1 = fan_bin(X - 1.0, Y, ce, se, Rt, src, inv_du, half);
      const double b2 = fan_bin(X + 1.0, Y, ce, se, Rt, src, inv_du, half);
      const int lo = max(0, static_cast<int>(ceil(fmax(fmin(b1, b2), -1.0))));
      const int hi = min(B - 1, static_cast<int>(floor(fmin(fmax(b1, b2), static_cast<double>(B)))));
      for (int b = lo; b <= hi; ++b) {
        const double* e = rv + 3 * b;
        const double sc = e[2];
        if (sc <= 0.0) continue;
        const double f = e[0] + (i - c) * e[1];
        const double fl = floor(f);
        const int q = static_cast<int>(fl);
        const C w = static_cast<C>(f - fl);
        const C val = static_cast<C>(sc) * static_cast<C>(Io<SI>::ld(pv, b));
        if (q == j) acc += (C(1) - w) * val;
        else if (q == j - 1) acc += w * val;
      }
    }
    // rays stepping along columns, through the segment of column j
    {
      const double b1 = fan_bin(X, Y - 1.0, ce, se, Rt, src, inv_du, half);
      const double b2 = fan_bin(X, Y + 1.0, ce, se, Rt, src, inv_du, half);
      const int lo = max(0, static_cast<int>(ceil(fmax(fmin(b1, b2), -1.0))));
      const int hi = min(B - 1, static_cast<int>(floor(fmin(fmax(b1, b2), static_cast<double>(B)))));
      for (int b = lo; b <= hi; ++b) {
        const double* e = rv + 3 * b;
        const double sc = e[2];
        if (sc >= 0.0) continue;
        const double f = e[0] + (j - c) * e[1];
        const double fl = floor(f);
        const int q = static_cast<int>(fl);
        const C w = static_cast<C>(f - fl);
        const C val = static_cast<C>(-sc) * static_cast<C>(Io<SI>::ld(pv, b));
        if (q == i) acc += (C(1) - w) * val;
        else if (q == i - 1) acc += w * val;
      }
    }
  }
  for (int o = kFanAdjSeg / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kFanAdjSeg);
  if (valid && vs == 0)
    Io<SO>::st(x + static_cast<size_t>(blockIdx.y) * n * n, static_cast<size_t>(i) * n + j, acc);
}

template <class SI, class SO, class C>
static nys_status launch_fan_fwd(const nys_op_s* op, const SI* x, SO* p, int64_t ncols,
                                 hipStream_t st) {
  const auto& d = op->d;
  dim3 grid(cdiv(static_cast<int64_t>(d.n_bins) * kFanSeg, 256), d.n_views,
            static_cast<unsigned>(ncols));
  hipLaunchKernelGGL((fan_fwd_kernel<SI, SO, C>), grid, dim3(256), 0, st, x, p, d.n1, d.n_views,
                     d.n_bins, d.fan_src, d.fan_det, d.fan_du);
  return launch_check("fan_fwd_kernel");
}

template <class SI, class SO, class C>
static nys_status launch_fan_adj(nys_op_s* op, const SI* p, SO* x, int64_t ncols, hipStream_t st) {
  const auto& d = op->d;
  if (op->fan_gather) {
    dim3 grid(cdiv(static_cast<int64_t>(d.n1) * d.n1 * kFanAdjSeg, 256), static_cast<unsigned>(ncols));
    hipLaunchKernelGGL((fan_adj_gather_kernel<SI, SO, C>), grid, dim3(256), 0, st, p, x,
                       op->rays.as<double>(), d.n1, d.n_views, d.n_bins, d.fan_src, d.fan_det,
                       d.fan_du);
    return launch_check("fan_adj_gather_kernel");
  }
  const size_t n = static_cast<size_t>(d.n1) * d.n2 * ncols;
  C* acc;
  if constexpr (std::is_same<SO, C>::value) {
    acc = x;
  } else {
    NYS_TAKE(op->scr, C, acc, n);
  }
  NYS_TRY(fill_zero<C>(acc, n, st));
  dim3 grid(cdiv(d.n_bins, 256), d.n_views, static_cast<unsigned>(ncols));
  hipLaunchKernelGGL((fan_adj_kernel<SI, C>), grid, dim3(256), 0, st, p, acc, d.n1, d.n_views,
                     d.n_bins, d.fan_src, d.fan_det, d.fan_du);
  NYS_TRY(launch_check("fan_adj_kernel"));
  if constexpr (!std::is_same<SO, C>::value) {
    hipLaunchKernelGGL((convert_kernel<C, SO>), dim3(std::min<size_t>(cdiv(n, 256), 4096)),
                       dim3(256), 0, st, acc, x, n);
    return launch_check("convert_kernel");
  }
  return NYS_OK;
}

// A applied to an image (no wavelet composition): SI -> SO.
template <class SI, class SO, class C>
static nys_status apply_A_plain(nys_op_s* op, const SI* x, SO* y, int64_t ncols, hipStream_t st) {
  const auto& d = op->d;
  switch (d.kind) {
    case NYS_OP_BLUR:
      return launch_correlate<SI, SO, C>(op, x, y, true, d.n1, d.n2, 1, ncols, st);
    case NYS_OP_BLURDOWN:
      return launch_correlate<SI, SO, C>(op, x, y, true, d.n1, d.n2, d.factor, ncols, st);
    case NYS_OP_PARALLEL_BEAM:
      return launch_joseph_fwd<SI, SO, C>(op, x, y, ncols, st);
    case NYS_OP_FAN_BEAM:
      return launch_fan_fwd<SI, SO, C>(op, x, y, ncols, st);
    default: break;
  }
  set_error("apply_A_plain: bad operator kind");
  return NYS_EINVAL;
}

template <class SI, class SO, class C>
static nys_status apply_At_plain(nys_op_s* op, const SI* y, SO* x, int64_t ncols, hipStream_t st) {
  const auto& d = op->d;
  switch (d.kind) {
    case NYS_OP_BLUR:
      return launch_correlate<SI, SO, C>(op, y, x, false, d.n1, d.n2, 1, ncols, st);
    case NYS_OP_BLURDOWN:
      return launch_upcorrelate<SI, SO, C>(op, y, x, d.n1 / d.factor, d.n2 / d.factor,
                                           d.factor, ncols, st);
    case NYS_OP_PARALLEL_BEAM:
      return launch_joseph_adj<SI, SO, C>(op, y, x, ncols, st);
    case NYS_OP_FAN_BEAM:
      return launch_fan_adj<SI, SO, C>(op, y, x, ncols, st);
    default: break;
  }
  set_error("apply_At_plain: bad operator kind");
  return NYS_EINVAL;
}

template <class T>
static nys_status copy_cols(const T* src, T* dst, size_t count, hipStream_t st) {
  if (src == dst) return NYS_OK;
  NYS_CHECK_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToDevice, st));
  return NYS_OK;
}

// y = A x with the optional wavelet synthesis in front (x holds coefficients).
template <class T>
nys_status op_fwd(nys_op op, const T* x, T* y, int64_t ncols, hipStream_t st) {
  const auto& d = op->d;
  const T* src = x;
  Scratch::Mark mark(op->scr);
  if (d.wavelet_levels > 0) {
    T* t = nullptr;
    if (d.kind != NYS_OP_IDENTITY) NYS_TAKE(op->scr, T, t, static_cast<size_t>(op->N) * ncols);
    NYS_TRY((launch_wavelet<false, T, T, T>(op, x, d.kind == NYS_OP_IDENTITY ? y : t, ncols, st)));
    if (d.kind == NYS_OP_IDENTITY) return NYS_OK;
    src = t;
  } else if (d.kind == NYS_OP_IDENTITY) {
    return copy_cols(x, y, static_cast<size_t>(op->N) * ncols, st);
  }
  return apply_A_plain<T, T, T>(op, src, y, ncols, st);
}

template <class T>
nys_status op_adj(nys_op op, const T* y, T* x, int64_t ncols, hipStream_t st) {
  const auto& d = op->d;
  if (d.kind == NYS_OP_IDENTITY) {
    if (d.wavelet_levels > 0)
      return launch_wavelet<true, T, T, T>(op, y, x, ncols, st);
    return copy_cols(y, x, static_cast<size_t>(op->N) * ncols, st);
  }
  if (d.wavelet_levels > 0) {
    Scratch::Mark mark(op->scr);
    T* t = nullptr;
    NYS_TAKE(op->scr, T, t, static_cast<size_t>(op->N) * ncols);
    NYS_TRY((apply_At_plain<T, T, T>(op, y, t, ncols, st)));
    return launch_wavelet<true, T, T, T>(op, t, x, ncols, st);
  }
  return apply_At_plain<T, T, T>(op, y, x, ncols, st);
}

template nys_status op_fwd<double>(nys_op, const double*, double*, int64_t, hipStream_t);
template nys_status op_fwd<float>(nys_op, const float*, float*, int64_t, hipStream_t);
template nys_status op_adj<double>(nys_op, const double*, double*, int64_t, hipStream_t);
template nys_status op_adj<float>(nys_op, const float*, float*, int64_t, hipStream_t);

// ---------------------------------------------------------------- sketch
// Y = Phi Omega.  S is the storage type of Omega and Y; C the compute type.
// Intermediates are kept in C.  Each stage processes all columns at once.
template <class S, class C>
static nys_status sketch_chain(nys_op op, const S* omega, S* Y, int64_t ell, hipStream_t st) {
  const auto& d = op->d;
  const int64_t N = op->N, M = op->M;
  const bool wav = d.wavelet_levels > 0;
  Scratch::Mark mark(op->scr);
  if (d.kind == NYS_OP_IDENTITY) {
    // Phi = W W^T = I
    if (wav) {
      C* t = nullptr;
      NYS_TAKE(op->scr, C, t, static_cast<size_t>(N) * ell);
      NYS_TRY((launch_wavelet<false, S, C, C>(op, omega, t, ell, st)));
      return launch_wavelet<true, C, S, C>(op, t, Y, ell, st);
    }
    NYS_CHECK_HIP(hipMemcpyAsync(Y, omega, sizeof(S) * N * ell, hipMemcpyDeviceToDevice, st));
    return NYS_OK;
  }
  C* img = nullptr;
  C* meas = nullptr;
  if (wav) NYS_TAKE(op->scr, C, img, static_cast<size_t>(N) * ell);
  NYS_TAKE(op->scr, C, meas, static_cast<size_t>(std::max(M, wav ? N : 0)) * ell);
  if (wav) {
    NYS_TRY((launch_wavelet<false, S, C, C>(op, omega, img, ell, st)));
    NYS_TRY((apply_A_plain<C, C, C>(op, img, meas, ell, st)));
    NYS_TRY((apply_At_plain<C, C, C>(op, meas, img, ell, st)));
    return launch_wavelet<true, C, S, C>(op, img, Y, ell, st);
  }
  NYS_TRY((apply_A_plain<S, C, C>(op, omega, meas, ell, st)));
  return apply_At_plain<C, S, C>(op, meas, Y, ell, st);
}

nys_status sketch_dispatch(nys_op op, nys_dtype dt, const void* omega, void* Y, int64_t ell,
                           hipStream_t st) {
  switch (dt) {
    case NYS_F64:
      return sketch_chain<double, double>(op, static_cast<const double*>(omega),
                                          static_cast<double*>(Y), ell, st);
    case NYS_F32:
      if (op->d.kind == NYS_OP_BLURDOWN && op->d.wavelet_levels == 3 && op->d.factor == 2 &&
          op->d.wavelet == NYS_WAVELET_HAAR)
        return sketch_sr_fused<float>(op, static_cast<const float*>(omega),
                                      static_cast<float*>(Y), ell, st);
      return sketch_chain<float, float>(op, static_cast<const float*>(omega),
                                        static_cast<float*>(Y), ell, st);
    case NYS_BF16:
      if (op->d.kind == NYS_OP_BLURDOWN && op->d.wavelet_levels == 3 && op->d.factor == 2 &&
          op->d.wavelet == NYS_WAVELET_HAAR)
        return sketch_sr_fused<uint16_t>(op, static_cast<const uint16_t*>(omega),
                                         static_cast<uint16_t*>(Y), ell, st);
      return sketch_chain<uint16_t, float>(op, static_cast<const uint16_t*>(omega),
                                           static_cast<uint16_t*>(Y), ell, st);
  }
  set_error("nys_sketch: bad dtype");
  return NYS_EINVAL;
}

// Reference (unfused) chain for the fused super-resolution sketch; exposed to
// the fused path's own fallback and to tests through an environment switch.
nys_status sketch_sr_chain_bf16(nys_op op, const uint16_t* omega, uint16_t* Y, int64_t ell,
                                hipStream_t st) {
  return sketch_chain<uint16_t, float>(op, omega, Y, ell, st);
}
nys_status sketch_sr_chain_f32(nys_op op, const float* omega, float* Y, int64_t ell,
                               hipStream_t st) {
  return sketch_chain<float, float>(op, omega, Y, ell, st);
}

}  // namespace nys

// ================================================================ C ABI
using namespace nys;

extern "C" const char* nys_last_error(void) { return nys::g_err; }
extern "C" const char* nys_version(void) { return "nys-mi355x 0.1 (gfx950)"; }

extern "C" nys_status nys_op_create(const nys_op_desc* desc, nys_op* out) {
  NYS_REQUIRE(desc && out, "nys_op_create: null argument");
  const nys_op_desc& d = *desc;
  NYS_REQUIRE(d.n1 > 0 && d.n2 > 0, "nys_op_create: bad image size %d x %d", d.n1, d.n2);
  NYS_REQUIRE(d.wavelet == NYS_WAVELET_HAAR || d.wavelet == NYS_WAVELET_DB4, "unknown wavelet");
  NYS_REQUIRE(d.wavelet_levels >= 0 && d.wavelet_levels <= (d.wavelet == NYS_WAVELET_DB4 ? 6 : 3),
              "wavelet_levels must be 0..3 (Haar) or 0..6 (Daubechies-4)");
  if (d.wavelet_levels > 0) {
    int B = 1 << d.wavelet_levels;
    NYS_REQUIRE(d.n1 % B == 0 && d.n2 % B == 0, "image size not divisible by 2^levels");
  }
  auto* op = new nys_op_s();
  op->d = d;
  op->d.psf = nullptr;
  if (d.wavelet == NYS_WAVELET_DB4) op->db4 = db4_filters();
  op->N = static_cast<int64_t>(d.n1) * d.n2;
  nys_status st = NYS_OK;
  switch (d.kind) {
    case NYS_OP_BLUR:
    case NYS_OP_BLURDOWN: {
      int k = d.psf_size;
      int f = d.kind == NYS_OP_BLUR ? 1 : d.factor;
      if (!(k >= 1 && k % 2 == 1 && k <= 31 && d.psf && f >= 1 && d.n1 % f == 0 &&
            d.n2 % f == 0 && k <= d.n1 && k <= d.n2)) {
        delete op;
        set_error("nys_op_create: bad PSF size %d / factor %d for %d x %d", k, d.factor, d.n1, d.n2);
        return NYS_EINVAL;
      }
      op->d.factor = f;
      op->M = static_cast<int64_t>(d.n1 / f) * (d.n2 / f);
      op->psf.assign(d.psf, d.psf + k * k);
      {
        // rank-1 test, pivoting on the largest entry: psf = u v^T exactly up
        // to rounding enables the separable kernels
        int ap = 0, bp = 0;
        double mx = 0;
        for (int a = 0; a < k; ++a)
          for (int b = 0; b < k; ++b)
            if (std::fabs(op->psf[a * k + b]) > mx) { mx = std::fabs(op->psf[a * k + b]); ap = a; bp = b; }
        double err = 0;
        if (mx > 0) {
          for (int a = 0; a < k; ++a) op->sep_u[a] = op->psf[a * k + bp];
          for (int b = 0; b < k; ++b) op->sep_v[b] = op->psf[ap * k + b] / op->psf[ap * k + bp];
          for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
              err = std::fmax(err, std::fabs(op->psf[a * k + b] - op->sep_u[a] * op->sep_v[b]));
        }
        op->sep = (mx > 0 && err <= 1e-14 * mx) ? 1 : 0;
      }
      std::vector<double> h64(2 * k * k);
      std::vector<float> h32(2 * k * k);
      for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
          h64[a * k + b] = op->psf[(k - 1 - a) * k + (k - 1 - b)];
          h64[k * k + a * k + b] = op->psf[a * k + b];
        }
      for (int t = 0; t < 2 * k * k; ++t) h32[t] = static_cast<float>(h64[t]);
      st = op->psf_dev.ensure(2 * k * k * (8 + 4));
      if (st == NYS_OK) {
        hipMemcpy(op->psf_dev.p, h64.data(), 8 * 2 * k * k, hipMemcpyHostToDevice);
        hipMemcpy(op->psf_dev.as<double>() + 2 * k * k, h32.data(), 4 * 2 * k * k,
                  hipMemcpyHostToDevice);
      }
      break;
    }
    case NYS_OP_FAN_BEAM: {
      if (!(d.n1 == d.n2 && d.n_views > 0 && d.n_bins > 0 && d.fan_src > 0 && d.fan_det >= 0 &&
            d.fan_du > 0 && std::isfinite(d.fan_src) && std::isfinite(d.fan_det) &&
            std::isfinite(d.fan_du))) {
        delete op;
        set_error("nys_op_create: fan beam needs a square image, views, bins > 0, "
                  "fan_src > 0, fan_det >= 0, fan_du > 0");
        return NYS_EINVAL;
      }
      op->M = static_cast<int64_t>(d.n_views) * d.n_bins;
      // the gathered adjoint needs the source outside the circle through the
      // corners of the image grown by one pixel (n > that radius for n >= 4)
      op->fan_gather = d.fan_src > d.n1 && d.n1 >= 4;
      if (op->fan_gather) {
        const size_t nt = 2 * static_cast<size_t>(d.n_views) + 3 * static_cast<size_t>(op->M);
        nys_status s = op->rays.ensure(nt * sizeof(double));
        if (s == NYS_OK) {
          hipLaunchKernelGGL(fan_table_kernel, dim3(cdiv(op->M, 256)), dim3(256), 0, nullptr,
                             op->rays.as<double>(), d.n1, d.n_views, d.n_bins, d.fan_src,
                             d.fan_det, d.fan_du);
          s = launch_check("fan_table_kernel");
        }
        if (s == NYS_OK && hipStreamSynchronize(nullptr) != hipSuccess) {
          set_error("nys_op_create: fan-beam ray table failed");
          s = NYS_EHIP;
        }
        if (s != NYS_OK) {
          op->rays.release();
          delete op;
          return s;
        }
      }
      break;
    }
    case NYS_OP_PARALLEL_BEAM: {
      if (!(d.n1 == d.n2 && d.n_views > 0 && d.n_bins > 0)) {
        delete op;
        set_error("nys_op_create: parallel beam needs a square image and views, bins > 0");
        return NYS_EINVAL;
      }
      op->M = static_cast<int64_t>(d.n_views) * d.n_bins;
      // per view: cos, sin, then 1 / |a| with a the cosine on row-branch
      // views (|cos| >= |sin|) and the sine otherwise
      const int V = d.n_views;
      std::vector<double> t64(3 * V);
      std::vector<float> t32(3 * V);
      for (int v = 0; v < V; ++v) {
        double th = M_PI * v / V;
        const double cv = std::cos(th), sv = std::sin(th);
        t64[2 * v] = cv;
        t64[2 * v + 1] = sv;
        t32[2 * v] = static_cast<float>(cv);
        t32[2 * v + 1] = static_cast<float>(sv);
      }
      for (int v = 0; v < V; ++v) {
        // the kernels pick the branch from the rounded values of each precision
        const double c64 = t64[2 * v], s64 = t64[2 * v + 1];
        t64[2 * V + v] = 1.0 / std::fabs(std::fabs(c64) >= std::fabs(s64) ? c64 : s64);
        const float c32 = t32[2 * v], s32 = t32[2 * v + 1];
        t32[2 * V + v] = 1.0f / std::fabs(std::fabs(c32) >= std::fabs(s32) ? c32 : s32);
      }
      st = op->trig.ensure(V * 3 * (8 + 4));
      if (st == NYS_OK) {
        hipMemcpy(op->trig.p, t64.data(), 8 * 3 * V, hipMemcpyHostToDevice);
        hipMemcpy(op->trig.as<double>() + 3 * V, t32.data(), 4 * 3 * V, hipMemcpyHostToDevice);
      }
      break;
    }
    case NYS_OP_IDENTITY:
      op->M = op->N;
      break;
    default:
      delete op;
      set_error("nys_op_create: unknown kind %d", d.kind);
      return NYS_EINVAL;
  }
  if (st != NYS_OK) {
    delete op;
    return st;
  }
  *out = op;
  return NYS_OK;
}

extern "C" void nys_op_destroy(nys_op op) {
  if (!op) return;
  op->psf_dev.release();
  op->trig.release();
  op->rays.release();
  delete op;
}

extern "C" nys_status nys_op_shape(nys_op op, int64_t* n_unknowns, int64_t* n_meas) {
  NYS_REQUIRE(op, "nys_op_shape: null op");
  if (n_unknowns) *n_unknowns = op->N;
  if (n_meas) *n_meas = op->M;
  return NYS_OK;
}

namespace nys {
// Workspace of op_fwd / op_adj on ncols columns of es-byte values: the
// larger of the two directions (the synthesis / analysis intermediate of a
// wavelet composition, then the Daubechies-4 pass scratch or the transposed
// images of the parallel-beam forward).
size_t op_ws_bytes(nys_op op, size_t es, int64_t ncols) {
  const auto& d = op->d;
  const size_t img = ws_round(es * static_cast<size_t>(op->N) * ncols);
  const bool wav = d.wavelet_levels > 0;
  size_t inner = 0;
  if (wav && d.wavelet == NYS_WAVELET_DB4) inner = img;
  if (d.kind == NYS_OP_PARALLEL_BEAM) {
    inner = img;
    // FP32 partial sums of a split whole-view forward
    if (es == 4)
      inner += ws_round(2 * sizeof(float) * static_cast<size_t>(op->M) *
                        jos_fwd_split_cols(d.n_views, d.n_bins, ncols));
  }
  return (wav && d.kind != NYS_OP_IDENTITY ? img : 0) + inner;
}

// Workspace of the sketch on ell columns stored in dt: the image and
// measurement stacks of the chain (compute type), then the pass scratch.
size_t sketch_ws_bytes(nys_op op, nys_dtype dt, int64_t ell) {
  const auto& d = op->d;
  const size_t cs = dt == NYS_F64 ? 8 : 4, ss = dtype_size(dt);
  const size_t nimg = static_cast<size_t>(op->N) * ell;
  const bool wav = d.wavelet_levels > 0;
  const bool db4 = wav && d.wavelet == NYS_WAVELET_DB4;
  const size_t db4_b = db4 ? ws_round(cs * nimg) * (ss == cs ? 1 : 2) : 0;
  if (d.kind == NYS_OP_IDENTITY) return wav ? ws_round(cs * nimg) + db4_b : 0;
  size_t inner = db4_b;
  if (d.kind == NYS_OP_PARALLEL_BEAM) {
    inner = std::max(inner, ws_round(std::max(ss, cs) * nimg));
    // FP32 partial sums of a split whole-view forward
    if (cs == 4)
      inner += ws_round(2 * sizeof(float) * static_cast<size_t>(op->M) *
                        jos_fwd_split_cols(d.n_views, d.n_bins, ell));
  }
  if (d.kind == NYS_OP_FAN_BEAM && ss != cs) inner = std::max(inner, ws_round(cs * nimg));
  return (wav ? ws_round(cs * nimg) : 0) +
         ws_round(cs * static_cast<size_t>(std::max(op->M, wav ? op->N : 0)) * ell) + inner;
}
}  // namespace nys

extern "C" nys_status nys_op_workspace_size(nys_op op, nys_dtype dt, int64_t ncols,
                                            size_t* bytes) {
  NYS_REQUIRE(op && bytes && ncols > 0, "nys_op_workspace_size: bad argument");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "nys_op_workspace_size: dtype must be F64 or F32");
  *bytes = op_ws_bytes(op, dtype_size(dt), ncols);
  return NYS_OK;
}

extern "C" nys_status nys_sketch_workspace_size(nys_op op, nys_dtype dt, int64_t ell,
                                                size_t* bytes) {
  NYS_REQUIRE(op && bytes && ell > 0, "nys_sketch_workspace_size: bad argument");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32 || dt == NYS_BF16, "nys_sketch_workspace_size: bad dtype");
  *bytes = sketch_ws_bytes(op, dt, ell);
  return NYS_OK;
}

extern "C" nys_status op_forward(nys_op op, nys_dtype dt, const void* x, void* y, int64_t ncols,
                                 void* ws, size_t ws_bytes, void* stream) {
  NYS_REQUIRE(op && x && y && ncols > 0, "op_forward: bad argument");
  NYS_REQUIRE(ncols <= 65535, "op_forward: ncols > 65535");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "op_forward: dtype must be F64 or F32");
  NYS_TRY(check_workspace(ws, ws_bytes, op_ws_bytes(op, dtype_size(dt), ncols), "op_forward"));
  WsBind bind(ws, ws_bytes, op, nullptr);
  if (dt == NYS_F64)
    return op_fwd<double>(op, static_cast<const double*>(x), static_cast<double*>(y), ncols,
                          as_stream(stream));
  return op_fwd<float>(op, static_cast<const float*>(x), static_cast<float*>(y), ncols,
                       as_stream(stream));
}

extern "C" nys_status op_adjoint(nys_op op, nys_dtype dt, const void* y, void* x, int64_t ncols,
                                 void* ws, size_t ws_bytes, void* stream) {
  NYS_REQUIRE(op && x && y && ncols > 0, "op_adjoint: bad argument");
  NYS_REQUIRE(ncols <= 65535, "op_adjoint: ncols > 65535");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32, "op_adjoint: dtype must be F64 or F32");
  NYS_TRY(check_workspace(ws, ws_bytes, op_ws_bytes(op, dtype_size(dt), ncols), "op_adjoint"));
  WsBind bind(ws, ws_bytes, op, nullptr);
  if (dt == NYS_F64)
    return op_adj<double>(op, static_cast<const double*>(y), static_cast<double*>(x), ncols,
                          as_stream(stream));
  return op_adj<float>(op, static_cast<const float*>(y), static_cast<float*>(x), ncols,
                       as_stream(stream));
}

extern "C" nys_status nys_sketch(nys_op op, nys_dtype dt, const void* omega, void* Y, int64_t ell,
                                 void* ws, size_t ws_bytes, void* stream) {
  NYS_REQUIRE(op && omega && Y && ell > 0, "nys_sketch: bad argument");
  NYS_REQUIRE(ell <= 65535, "nys_sketch: ell > 65535");
  NYS_REQUIRE(omega != Y, "nys_sketch: omega and Y must not alias");
  NYS_REQUIRE(dt == NYS_F64 || dt == NYS_F32 || dt == NYS_BF16, "nys_sketch: bad dtype");
  NYS_TRY(check_workspace(ws, ws_bytes, sketch_ws_bytes(op, dt, ell), "nys_sketch"));
  WsBind bind(ws, ws_bytes, op, nullptr);
  return sketch_dispatch(op, dt, omega, Y, ell, as_stream(stream));
}
