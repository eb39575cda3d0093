// Many periodic-blur reconstructions of different sizes solved together.
//
// Each instance solves eq. (4) with f = 1/2 ||h * x - y||^2 and a TV / HS1
// prior by WAPG (Alg. 3) preconditioned with P of eq. (11), which is built
// from the sketch Y = A^T A Omega (Alg. 1, step 2) and the shifted Nystrom
// factorisation (Alg. 1, steps 3-7); the step follows the power-method bound
// of L_f^P (the constant of eq. (20)).  Every launch covers all instances:
//   * A^T A of a periodic blur is the periodic correlation with the
//     autocorrelation of the PSF, separable for a separable PSF.  One
//     persistent kernel applies it (and H, H^T) to every (instance, column,
//     tile) item, pulling items from eight work queues, one per XCD, each
//     holding a contiguous run of tiles so that neighbouring tiles share that
//     XCD's L2;
//   * the Gram, the FP64 factorisation (one workgroup per instance) and U
//     are batched over segment tables;
//   * the WAPG loop, its P^{-1} applications and the inner dual iterations
//     of the P-weighted prox run as batched launches.
// The whole pipeline is captured once into a HIP graph; a run is one graph
// launch.  Tile heights of the stencil kernel come from a timing autotuner
// run when the plan is created.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "fused.hpp"
#include "internal.hpp"
#include "stencil.hpp"

namespace nys {

template <class T> nys_status fill_zero(T* p, size_t n, hipStream_t st);

// ================================================================ stencil
constexpr int kStW = 64;          // tile columns: one wave64 row
constexpr int kStMaxTaps = 61;    // autocorrelation of a 31-tap PSF factor
constexpr int kQueues = 8;        // one work queue per XCD

// out[c][i][j] = sum_{a,b} tr[a] tc[b] in[c][(i + lo_r + a) mod n1][(j + lo_c + b) mod n2]
//                (- sub[i][j] when sub != null); columns cstride elements apart.
struct StTask {
  const float* in;
  float* out;
  const float* sub;
  int64_t cstride;
  int32_t n1, n2;
  int32_t lo_r, nt_r, lo_c, nt_c;
  int32_t taps;     // offset of nt_r row taps, then nt_c column taps
  int32_t ty;       // tile rows (tile kernel) or run length (streaming kernel)
  int32_t ss;       // 1: streaming kernel (see ss_eligible)
};

struct StItem {
  int32_t task, col, y0, x0;
};

// Row pitch (floats) of the register-blocked path for NT taps: the tile's
// 64 + NT - 1 input columns plus at least 4 floats of slack for the float4
// window reads of the horizontal pass.
__host__ __device__ constexpr int st_pitch(int nt) { return (kStW + nt - 1 + 7) & ~3; }

__host__ __device__ inline bool st_fast(int ty, int nt_r, int nt_c) {
  return nt_r == nt_c && nt_r <= 29 && (nt_r & 1) && (ty & 7) == 0;
}

__host__ __device__ inline int st_lds_floats(int ty, int nt_r, int nt_c) {
  const int hr = ty + nt_r - 1;
  if (st_fast(ty, nt_r, nt_c)) return (hr + ty) * st_pitch(nt_r);
  return hr * (kStW + nt_c - 1) + hr * kStW;
}

__device__ __forceinline__ int wrap_idx(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Loads rows [0, hr) x columns [0, wc) (wc <= 128) of the periodic input
// window starting at (y0 + lo_r, x0 + lo_c) into tin (row pitch `pitch`).
// Eight rows per batch are loaded into registers before any is stored, so a
// thread keeps up to 16 global loads in flight.
__device__ __forceinline__ void st_load_window(const StTask& T, const StItem& I, int hr, int wc,
                                               int pitch, float* tin) {
  constexpr int kLB = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* src = T.in + static_cast<int64_t>(I.col) * T.cstride;
  const int gj0 = wrap_idx(I.x0 + T.lo_c + lane, T.n2);
  const bool two = lane + kStW < wc;
  const int gj1 = two ? wrap_idx(I.x0 + T.lo_c + lane + kStW, T.n2) : gj0;
  for (int r0 = wave; r0 < hr; r0 += 4 * kLB) {
    float va[kLB], vb[kLB];
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int r = r0 + 4 * t;
      const int gr = wrap_idx(I.y0 + T.lo_r + (r < hr ? r : 0), T.n1);
      const float* row = src + static_cast<int64_t>(gr) * T.n2;
      va[t] = row[gj0];
      vb[t] = row[gj1];
    }
#pragma unroll
    for (int t = 0; t < kLB; ++t) {
      const int r = r0 + 4 * t;
      if (r < hr) {
        tin[r * pitch + lane] = va[t];
        if (two) tin[r * pitch + lane + kStW] = vb[t];
      }
    }
  }
}

// One tile with NT taps per axis (odd, <= 29) and a tile height that is a
// multiple of 8: the vertical pass first, over the 64 + NT - 1 input columns,
// then the horizontal pass.  Vertical: a thread owns one column and 8
// consecutive output rows and slides the NT taps (registers) down the
// column, so each LDS value it reads feeds up to NT accumulators.
// Horizontal: a thread owns 4 consecutive outputs of a row and reads its
// NT + 3 inputs as float4 runs.  The periodic halo is loaded whole even for
// a ragged last tile; only rows and columns inside the image are stored.
template <int NT>
__device__ __forceinline__ void st_tile_fast(const StTask& T, const StItem& I, float* sm,
                                             const float* s_tr, const float* s_tc) {
  constexpr int WC = kStW + NT - 1;
  constexpr int WP = st_pitch(NT);
  const int tid = threadIdx.x;
  const int ty = T.ty;
  const int HR = ty + NT - 1;
  float* tin = sm;
  float* mid = sm + HR * WP;
  st_load_window(T, I, HR, WC, WP, tin);
  __syncthreads();
  // row taps live only through the vertical pass, column taps only through
  // the horizontal one (fewer registers, more resident workgroups)
  float tr[NT];
#pragma unroll
  for (int a = 0; a < NT; ++a) tr[a] = s_tr[a];
  const int nrb = ty >> 3;
  for (int u = tid; u < nrb * WC; u += 256) {
    const int rb = u / WC, q = u - rb * WC;
    float acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = 0.f;
    const float* p = tin + (rb * 8) * WP + q;
#pragma unroll
    for (int m = 0; m < 8 + NT - 1; ++m) {
      const float v = p[m * WP];
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        const int o = m - a;
        if (o >= 0 && o < 8) acc[o] = fmaf(tr[a], v, acc[o]);
      }
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) mid[(rb * 8 + o) * WP + q] = acc[o];
  }
  __syncthreads();
  const int rows = min(ty, T.n1 - I.y0);
  float* dst = T.out + static_cast<int64_t>(I.col) * T.cstride;
  const bool vec = (T.n2 & 3) == 0;
  float tc[NT];
#pragma unroll
  for (int a = 0; a < NT; ++a) tc[a] = s_tc[a];
  for (int u = tid; u < rows * 16; u += 256) {
    const int r = u >> 4, g = u & 15;
    const float* p = mid + r * WP + 4 * g;
    constexpr int NW = (NT + 3 + 3) / 4;
    float w[4 * NW];
#pragma unroll
    for (int e = 0; e < NW; ++e) {
      const float4 x = *reinterpret_cast<const float4*>(p + 4 * e);
      w[4 * e] = x.x; w[4 * e + 1] = x.y; w[4 * e + 2] = x.z; w[4 * e + 3] = x.w;
    }
    float o4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < NT; ++b) acc = fmaf(tc[b], w[k + b], acc);
      o4[k] = acc;
    }
    const int j = I.x0 + 4 * g;
    const int64_t o = static_cast<int64_t>(I.y0 + r) * T.n2 + j;
    if (vec && j + 3 < T.n2) {
      float4 v = make_float4(o4[0], o4[1], o4[2], o4[3]);
      if (T.sub) {
        const float4 sb = *reinterpret_cast<const float4*>(T.sub + o);
        v.x -= sb.x; v.y -= sb.y; v.z -= sb.z; v.w -= sb.w;
      }
      *reinterpret_cast<float4*>(dst + o) = v;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (j + k < T.n2) dst[o + k] = T.sub ? o4[k] - T.sub[o + k] : o4[k];
    }
  }
}

// Generic tile: any tap counts and tile height, runtime loops.
__device__ __forceinline__ void st_tile_generic(const StTask& T, const StItem& I, float* sm,
                                                const float* s_tr, const float* s_tc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = min(T.ty, T.n1 - I.y0);
  const int hr = rows + T.nt_r - 1, wc = kStW + T.nt_c - 1;
  float* tin = sm;
  float* mid = sm + hr * wc;
  st_load_window(T, I, hr, wc, wc, tin);
  __syncthreads();
  for (int r = wave; r < hr; r += 4) {
    const float* p = tin + r * wc + lane;
    float acc = 0.f;
    for (int b = 0; b < T.nt_c; ++b) acc = fmaf(s_tc[b], p[b], acc);
    mid[r * kStW + lane] = acc;
  }
  __syncthreads();
  const int j = I.x0 + lane;
  float* dst = T.out + static_cast<int64_t>(I.col) * T.cstride;
  for (int r = wave; r < rows; r += 4) {
    const float* p = mid + r * kStW + lane;
    float acc = 0.f;
    for (int a = 0; a < T.nt_r; ++a) acc = fmaf(s_tr[a], p[a * kStW], acc);
    if (j < T.n2) {
      const int64_t o = static_cast<int64_t>(I.y0 + r) * T.n2 + j;
      if (T.sub) acc -= T.sub[o];
      dst[o] = acc;
    }
  }
}

// Persistent: block b serves queue b % 8 first (its XCD), then the others.
// Each queue is a contiguous range of items; ctr[q] counts tickets of queue
// q, ctr[8] counts blocks that finished, and the last block to finish resets
// all counters, so consecutive launches on one stream reuse them.
__global__ __launch_bounds__(256) void bstencil_kernel(const StTask* __restrict__ tasks,
                                                       const StItem* __restrict__ items,
                                                       const int* __restrict__ qbase,
                                                       const float* __restrict__ taps,
                                                       int* __restrict__ ctr) {
  extern __shared__ float sm[];
  __shared__ float s_tr[kStMaxTaps], s_tc[kStMaxTaps];
  __shared__ int s_ticket;
  const int tid = threadIdx.x;
  const int home = blockIdx.x % kQueues;
  for (int qi = 0; qi < kQueues; ++qi) {
    const int q = (home + qi) % kQueues;
    const int q0 = qbase[q], qn = qbase[q + 1] - q0;
    if (tid == 0) s_ticket = atomicAdd(&ctr[q], 1);
    __syncthreads();
    int t = __builtin_amdgcn_readfirstlane(s_ticket);
    __syncthreads();
    while (t < qn) {
      // the next ticket is requested now; its latency overlaps this tile
      int nxt = 0;
      if (tid == 0) nxt = atomicAdd(&ctr[q], 1);
      const StItem I = items[q0 + t];
      const StTask T = tasks[I.task];
      if (tid < T.nt_r) s_tr[tid] = taps[T.taps + tid];
      else if (tid < T.nt_r + T.nt_c) s_tc[tid - T.nt_r] = taps[T.taps + tid];
      __syncthreads();
      if (st_fast(T.ty, T.nt_r, T.nt_c)) {
        switch (T.nt_r) {
          case 1: st_tile_fast<1>(T, I, sm, s_tr, s_tc); break;
          case 3: st_tile_fast<3>(T, I, sm, s_tr, s_tc); break;
          case 5: st_tile_fast<5>(T, I, sm, s_tr, s_tc); break;
          case 7: st_tile_fast<7>(T, I, sm, s_tr, s_tc); break;
          case 9: st_tile_fast<9>(T, I, sm, s_tr, s_tc); break;
          case 11: st_tile_fast<11>(T, I, sm, s_tr, s_tc); break;
          case 13: st_tile_fast<13>(T, I, sm, s_tr, s_tc); break;
          case 15: st_tile_fast<15>(T, I, sm, s_tr, s_tc); break;
          case 17: st_tile_fast<17>(T, I, sm, s_tr, s_tc); break;
          case 19: st_tile_fast<19>(T, I, sm, s_tr, s_tc); break;
          case 21: st_tile_fast<21>(T, I, sm, s_tr, s_tc); break;
          case 23: st_tile_fast<23>(T, I, sm, s_tr, s_tc); break;
          case 25: st_tile_fast<25>(T, I, sm, s_tr, s_tc); break;
          case 27: st_tile_fast<27>(T, I, sm, s_tr, s_tc); break;
          default: st_tile_fast<29>(T, I, sm, s_tr, s_tc); break;
        }
      } else {
        st_tile_generic(T, I, sm, s_tr, s_tc);
      }
      if (tid == 0) s_ticket = nxt;
      __syncthreads();
      t = __builtin_amdgcn_readfirstlane(s_ticket);
      __syncthreads();
    }
  }
  if (tid == 0 && atomicAdd(&ctr[kQueues], 1) == static_cast<int>(gridDim.x) - 1) {
    for (int q = 0; q < kQueues; ++q) atomicExch(&ctr[q], 0);
    atomicExch(&ctr[kQueues], 0);
  }
}

// ---------------------------------------------------------------- streaming
// One wave per item: a strip of 128 output columns (two per lane) and a run
// of up to T.ty output rows, for NT row taps = NT column taps (odd, <= 29,
// palindromic: the autocorrelation of a PSF always is).  The wave walks down
// the periodic input window one row at a time:
//   * row m is staged in LDS (128 + NT - 1 values: a float2 per lane plus one
//     halo value on NT - 1 lanes), from registers that were loaded NT rows
//     earlier, so NT rows of global loads stay in flight;
//   * horizontal pass: each lane reads its NT + 1 window values as float2
//     runs and forms its two columns' sums;
//   * vertical pass: the row's two results are added, with each row tap, to
//     a ring of NT partial outputs per column held in registers; after row m
//     the ring slot of output row m - NT + 1 is complete, stored and cleared.
// Per output pixel that is 2 NT (1 + (NT - 1) / rows) FMAs and 8 bytes of
// HBM traffic (plus the halo re-reads of neighbouring strips and runs).
// Only this wave touches its LDS row, and LDS operations of a wave complete
// in order, so a compiler-only memory barrier (no instruction) is the only
// synchronisation.  Global pointers are cast to the global address space so
// that loads are global (not flat) loads, which leave the LDS counter alone.
constexpr int kSsW = 128;
constexpr int kSsMaxNT = 29;
constexpr int kSsBuf = kSsW + 64;           // a float2 per lane, then one value per lane

typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const float gcf32;
typedef __attribute__((address_space(1))) const v2f32 gcf32x2;
typedef __attribute__((address_space(1))) float gf32;
typedef __attribute__((address_space(1))) v2f32 gf32x2;

// taps of a task palindromic (t[a] == t[nt - 1 - a] on both axes)
inline bool taps_palindromic(const std::vector<double>& t, int off, int nr, int nc) {
  for (int a = 0; a < nr; ++a)
    if (t[off + a] != t[off + nr - 1 - a]) return false;
  for (int a = 0; a < nc; ++a)
    if (t[off + nr + a] != t[off + nr + nc - 1 - a]) return false;
  return true;
}

// The streaming kernel takes equal odd row and column tap counts up to 29,
// palindromic taps, an even row length and an even first column offset (so
// that every lane's column pair is one aligned float2 that never straddles
// the periodic wrap).
inline bool ss_eligible(int nt_r, int nt_c, int lo_c, int n2, bool palindromic) {
  return nt_r == nt_c && (nt_r & 1) && nt_r <= kSsMaxNT && n2 % 2 == 0 && lo_c % 2 == 0 &&
         palindromic;
}

__device__ __forceinline__ void wave_fence() { asm volatile("" ::: "memory"); }

template <int NT, bool SUB>
__device__ __forceinline__ void ss_item(const StTask& T, const StItem& I,
                                        const float* __restrict__ taps, float* buf) {
  constexpr int NH = (NT + 1) / 2;        // distinct taps per axis (palindromic)
  constexpr int RG = (NT + 7) / 8 * 8;    // ring slots: >= NT, a multiple of the prefetch depth
  constexpr int PD = 8;                   // rows of global loads in flight
  const int lane = threadIdx.x;
  const int n1 = T.n1, n2 = T.n2;
  const int rows = min(T.ty, n1 - I.y0);
  const int M = rows + NT - 1;                       // input rows of the run
  gcf32* src = (gcf32*)(T.in + static_cast<int64_t>(I.col) * T.cstride);
  gf32* dst = (gf32*)(T.out + static_cast<int64_t>(I.col) * T.cstride);
  const int cb = I.x0 + T.lo_c;                     // even (see ss_eligible)
  const int c0 = wrap_idx(cb + 2 * lane, n2);
  const bool hal = lane < NT - 1;
  const int chl = wrap_idx(cb + kSsW + (hal ? lane : 0), n2);
  const int j = I.x0 + 2 * lane;
  const bool inb = j < n2;                           // n2 even: j + 1 < n2 as well
  const int jc = inb ? j : 0;
  float tr[NH], tc[NH];
#pragma unroll
  for (int a = 0; a < NH; ++a) {
    tr[a] = taps[T.taps + a];
    tc[a] = taps[T.taps + NT + a];
  }
  float px[PD], py[PD], ph[PD];
  float a0[RG], a1[RG];
#pragma unroll
  for (int s = 0; s < RG; ++s) {
    a0[s] = 0.f;
    a1[s] = 0.f;
  }
  // Loads and stores are issued on every step without uniform branches (the
  // loads past the run wrap to valid rows and go unused; a step before the
  // first complete output row stores into row y0, which the first complete
  // row overwrites later), so the compiler's wait counts keep PD rows of
  // loads in flight.
  int rl = wrap_idx(I.y0 + T.lo_r, n1);              // next input row to load
  auto load_row = [&](const int q) __attribute__((always_inline)) {
    gcf32* row = src + static_cast<int64_t>(rl) * n2;
    const v2f32 v = *(gcf32x2*)(row + c0);
    px[q] = v.x;
    py[q] = v.y;
    ph[q] = row[chl];
    rl = rl + 1 == n1 ? 0 : rl + 1;
  };
#pragma unroll
  for (int q = 0; q < PD; ++q) load_row(q);
  // one input row: s is the (compile-time) step within a block of RG rows
  auto step = [&](const int s, const int m) __attribute__((always_inline)) {
    const int q = s % PD;
    wave_fence();
    *reinterpret_cast<float2*>(buf + 2 * lane) = make_float2(px[q], py[q]);
    buf[kSsW + lane] = ph[q];                        // lanes >= NT - 1 write unread slots
    load_row(q);
    const int o = m - (NT - 1);
    const int orow = I.y0 + (o > 0 ? o : 0);
    v2f32 sb = {0.f, 0.f};
    if (SUB) sb = *(gcf32x2*)((gcf32*)T.sub + static_cast<int64_t>(orow) * n2 + jc);
    wave_fence();
    float h0 = 0.f, h1 = 0.f;
#pragma unroll
    for (int e = 0; e < NH; ++e) {
      const float2 w = *reinterpret_cast<const float2*>(buf + 2 * lane + 2 * e);
      // window value b feeds column 0 with tap b and column 1 with tap b - 1
      const int b0 = 2 * e, b1 = 2 * e + 1;
      h0 = fmaf(tc[b0 < NH ? b0 : NT - 1 - b0], w.x, h0);
      if (b1 < NT) h0 = fmaf(tc[b1 < NH ? b1 : NT - 1 - b1], w.y, h0);
      if (b0 >= 1) h1 = fmaf(tc[b0 - 1 < NH ? b0 - 1 : NT - b0], w.x, h1);
      h1 = fmaf(tc[b0 < NH ? b0 : NT - 1 - b0], w.y, h1);
    }
    // input row m feeds output row m - a with row tap a
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int sl = (s - a + RG) % RG;
      const float t = tr[a < NH ? a : NT - 1 - a];
      a0[sl] = fmaf(t, h0, a0[sl]);
      a1[sl] = fmaf(t, h1, a1[sl]);
    }
    // output row o = m - NT + 1 is complete (o < 0: a placeholder store)
    const int so = (s - (NT - 1) + RG) % RG;
    if (inb)
      *(gf32x2*)(dst + static_cast<int64_t>(orow) * n2 + j) = v2f32{a0[so] - sb.x, a1[so] - sb.y};
    a0[so] = 0.f;
    a1[so] = 0.f;
  };
  int m0 = 0;
  for (; m0 + RG <= M; m0 += RG) {
#pragma unroll
    for (int s = 0; s < RG; ++s) step(s, m0 + s);
  }
#pragma unroll
  for (int s = 0; s < RG; ++s)
    if (m0 + s < M) step(s, m0 + s);
}

// Workgroups go to the eight XCDs in turn (block b to XCD b mod 8); chunks
// of kSsChunk consecutive items are dealt to the XCDs in turn, so that each
// XCD runs whole chunks -- neighbouring runs of a strip, whose windows
// overlap -- back to back and serves the overlap from its own L2.
constexpr int kSsChunk = 16;

__device__ __forceinline__ int ss_item_of(int b) {
  const int x = b & 7, j = b >> 3;
  return ((j / kSsChunk) * 8 + x) * kSsChunk + j % kSsChunk;
}

inline int64_t ss_grid(int64_t nitems) {
  const int64_t per = 8 * kSsChunk;
  return (nitems + per - 1) / per * per;
}

// One workgroup (one wave) per item; items are sorted by tap count, largest
// first, so the longest items start first.
template <bool SUB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
void bstream_kernel(const StTask* __restrict__ tasks, const StItem* __restrict__ items,
                    const float* __restrict__ taps, int nitems) {
  __shared__ float buf[kSsBuf];
  const int it = ss_item_of(blockIdx.x);
  if (it >= nitems) return;
  const StItem I = items[it];
  const StTask T = tasks[I.task];
  switch (T.nt_r) {
    case 1: ss_item<1, SUB>(T, I, taps, buf); break;
    case 3: ss_item<3, SUB>(T, I, taps, buf); break;
    case 5: ss_item<5, SUB>(T, I, taps, buf); break;
    case 7: ss_item<7, SUB>(T, I, taps, buf); break;
    case 9: ss_item<9, SUB>(T, I, taps, buf); break;
    case 11: ss_item<11, SUB>(T, I, taps, buf); break;
    case 13: ss_item<13, SUB>(T, I, taps, buf); break;
    case 15: ss_item<15, SUB>(T, I, taps, buf); break;
    case 17: ss_item<17, SUB>(T, I, taps, buf); break;
    case 19: ss_item<19, SUB>(T, I, taps, buf); break;
    case 21: ss_item<21, SUB>(T, I, taps, buf); break;
    case 23: ss_item<23, SUB>(T, I, taps, buf); break;
    case 25: ss_item<25, SUB>(T, I, taps, buf); break;
    case 27: ss_item<27, SUB>(T, I, taps, buf); break;
    default: ss_item<29, SUB>(T, I, taps, buf); break;
  }
}

// ================================================================ pixel kernels
// All over 1024-pixel blocks (256 threads x 4) of a segment table.
#define BSEG_PROLOGUE                                              \
  const BSeg& sg = seg[seg_find(seg, nseg, blockIdx.x)];          \
  const BDesc& D = d[sg.inst];                                    \
  const int64_t lb = blockIdx.x - sg.first;                       \
  const int64_t base = lb * 1024;

__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  return red[0];
}

// D.part[lb] = sum of squares of the block (source f[fsrc], or v0 if fsrc < 0)
__global__ __launch_bounds__(256) void bsumsq_kernel(const BDesc* __restrict__ d,
                                                     const BSeg* __restrict__ seg, int nseg,
                                                     int fsrc) {
  __shared__ double red[256];
  BSEG_PROLOGUE
  const float* src = fsrc >= 0 ? D.f[fsrc] : D.v0;
  double s = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t n = base + q * 256 + threadIdx.x;
    if (n < D.N) {
      const double v = src[n];
      s += v * v;
    }
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) D.part[lb] = s;
}

// The warm start's coefficients c = d . U^T L^T Q of every instance
// (block = instance).  The last fused dual iteration of a prox forms them for
// its final Q (the partials of L^T Q+), and the next prox starts from that
// same Q, so they are kept instead of formed again with a pass over U:
// mode 0 clears the kept ones (Q = 0 at the start of a solve), 1 restores
// them into cd, 2 keeps cd, 3 clears cd (a cold start, Q = 0).
__global__ __launch_bounds__(64) void bcq_kernel(const BDesc* __restrict__ d, int mode) {
  const BDesc& D = d[blockIdx.x];
  for (int k = threadIdx.x; k < D.ell; k += blockDim.x) {
    switch (mode) {
      case 0: D.cq[k] = 0.0; break;
      case 1: D.cd[k] = D.cq[k]; break;
      case 2: D.cq[k] = D.cd[k]; break;
      default: D.cd[k] = 0.0; break;
    }
  }
}

// Sum of an instance's block partials, fixed order (blockIdx.x = segment):
// which = 0: scal[kNorm] = sqrt(sum); which = 1: costs[k] = sum.
__global__ __launch_bounds__(256) void bpart_tail_kernel(const BDesc* __restrict__ d,
                                                         const BSeg* __restrict__ seg, int which,
                                                         int k) {
  __shared__ double red[256];
  const BSeg& sg = seg[blockIdx.x];
  const BDesc& D = d[sg.inst];
  double s = 0;
  for (int64_t b = threadIdx.x; b < sg.nblk; b += blockDim.x) s += D.part[b];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) {
    if (which == 0) D.scal[BScal::kNorm] = sqrt(s);
    else if (D.costs) D.costs[k] = s;
  }
}

// f[fdst] = src / scal[kNorm]
__global__ __launch_bounds__(256) void bnormalize_kernel(const BDesc* __restrict__ d,
                                                         const BSeg* __restrict__ seg, int nseg,
                                                         int fsrc, int fdst) {
  BSEG_PROLOGUE
  const double nrm = D.scal[BScal::kNorm];
  const float inv = static_cast<float>(nrm > 0 ? 1.0 / nrm : 0.0);
  const float* src = fsrc >= 0 ? D.f[fsrc] : D.v0;
  float* dst = D.f[fdst];
  for (int q = 0; q < 4; ++q) {
    const int64_t n = base + q * 256 + threadIdx.x;
    if (n < D.N) dst[n] = src[n] * inv;
  }
}

// Step sizes from the power-method estimate (curvature 1 for the LS loss):
// alpha = 1 / (safety L), lam_bar = alpha lambda, dual step
// 1 / (lam_bar ||L||^2 ||P^{-1}||).
__global__ void bscalars_kernel(const BDesc* __restrict__ d, int n, double safety,
                                double lnorm2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BDesc& D = d[i];
  const double L = D.scal[BScal::kNorm];
  const double alpha = (L > 0 && isfinite(L)) ? 1.0 / (safety * L) : 0.0;
  double pn = D.ell > 0 ? D.meta[PcMeta::kPinvNorm] : 1.0;
  if (!(pn >= 1.0) || !isfinite(pn)) pn = 1.0;
  const double lam_bar = alpha * D.lambda;
  D.scal[BScal::kL] = L;
  D.scal[BScal::kAlpha] = alpha;
  D.scal[BScal::kLamBar] = lam_bar;
  D.scal[BScal::kPinvNorm] = pn;
  D.scal[BScal::kDualStep] = lam_bar > 0 ? 1.0 / (lam_bar * lnorm2 * pn) : 0.0;
}

// f[fout] = L^T f[fq]  (adjoint of the regulariser's map)
__global__ __launch_bounds__(256) void blt_kernel(const BDesc* __restrict__ d,
                                                  const BSeg* __restrict__ seg, int nseg, int reg,
                                                  int fq, int fout) {
  BSEG_PROLOGUE
  const float* q = D.f[fq];
  float* out = D.f[fout];
  for (int k = 0; k < 4; ++k) {
    const int64_t n = base + k * 256 + threadIdx.x;
    if (n >= D.N) break;
    const int i = static_cast<int>(n / D.n2), j = static_cast<int>(n - static_cast<int64_t>(i) * D.n2);
    out[n] = lt_at(q, reg, i, j, D.n1, D.n2);
  }
}

// accelerated projected dual step on every pixel, step = scal[kDualStep]
__global__ __launch_bounds__(256) void bdual_update_kernel(const BDesc* __restrict__ d,
                                                           const BSeg* __restrict__ seg, int nseg,
                                                           int reg, float beta) {
  BSEG_PROLOGUE
  const float step = static_cast<float>(D.scal[BScal::kDualStep]);
  for (int k = 0; k < 4; ++k) {
    const int64_t n = base + k * 256 + threadIdx.x;
    if (n >= D.N) break;
    const int i = static_cast<int>(n / D.n2), j = static_cast<int>(n - static_cast<int64_t>(i) * D.n2);
    dual_update_at<float>(D.f[kFldXN], D.f[kFldQ], D.f[kFldR], reg, i, j, D.n1, D.n2, step, beta);
  }
}

// u = x+ + beta (x+ - x); x = x+  (flat over the packed images)
__global__ __launch_bounds__(256) void bmomentum_kernel(const float* __restrict__ xn,
                                                        float* __restrict__ x,
                                                        float* __restrict__ u, float beta,
                                                        int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float a = xn[e];
    u[e] = a + beta * (a - x[e]);
    x[e] = a;
  }
}

// D.part[lb] = sum over the block of 1/2 (Hx - y)^2 + lambda g(x)  (Hx in f[kFldW])
__global__ __launch_bounds__(256) void bcost_partial_kernel(const BDesc* __restrict__ d,
                                                            const BSeg* __restrict__ seg, int nseg,
                                                            int term) {
  __shared__ double red[256];
  BSEG_PROLOGUE
  double s = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t n = base + k * 256 + threadIdx.x;
    if (n < D.N)
      s += term_at<float>(D.f[kFldW], D.y, n, kSq, 0.f, D.n1, D.n2) +
           D.lambda * term_at<float>(D.f[kFldX], nullptr, n, term, 0.f, D.n1, D.n2);
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) D.part[lb] = s;
}

__global__ __launch_bounds__(256) void bcopy_out_kernel(const BDesc* __restrict__ d,
                                                        const BSeg* __restrict__ seg, int nseg) {
  BSEG_PROLOGUE
  for (int k = 0; k < 4; ++k) {
    const int64_t n = base + k * 256 + threadIdx.x;
    if (n < D.N) D.x_out[n] = D.f[kFldX][n];
  }
}

// One fused inner iteration of the P-weighted prox (fused.hpp) of the
// instances whose U has KR rows: block b -> tile g of the launch
// (XCD-contiguous runs) -> instance and tile.  One launch per row count, so
// that the register budget (and with it the workgroups resident per CU:
// four at 16 rows, three at 32, two at 64) follows the rows each launch
// keeps; the tiles' phases are latency-bound, so residency is what hides
// them.
template <int KR> constexpr int bfused_waves() { return KR <= 16 ? 8 : KR <= 32 ? 6 : 4; }
template <int TW, int KR>
__global__ __launch_bounds__(kFThreads) __attribute__((amdgpu_waves_per_eu(bfused_waves<KR>())))
void bfused_kernel(const BDesc* __restrict__ d, const BSeg* __restrict__ seg, int nseg,
                   int ntiles, int reg, int fqi, int fri, int fqo, int fro, float beta, int last) {
  __shared__ FusedLds<TW> L;
  const int g = fused_tile_of(blockIdx.x, ntiles);
  if (g >= ntiles) return;
  const BSeg& sg = seg[seg_find(seg, nseg, g)];
  const BDesc& D = d[sg.inst];
  FusedArgs A;
  A.n1 = D.n1;
  A.n2 = D.n2;
  A.reg = reg;
  A.ell = D.ell;
  A.ell_pad = D.ell_pad;
  A.ldu = D.ldu;
  A.U = D.U;
  A.cd = D.cd;
  A.s = D.f[kFldS];
  A.Qi = D.f[fqi];
  A.Ri = D.f[fri];
  A.Qo = D.f[fqo];
  A.Ro = D.f[fro];
  A.lam_bar = static_cast<float>(D.scal[BScal::kLamBar]);
  A.step = static_cast<float>(D.scal[BScal::kDualStep]);
  A.beta = beta;
  A.last = last;
  A.part = D.fpart;
  const int tile = static_cast<int>(g - sg.first);
  const int ntx = (D.n2 + TW - 1) / TW;
  fused_tile<KR, TW>(A, tile, ntx, L);
}

// D.cd[k] = d_k sum_b D.fpart[b][k] for 16 coefficients a block: block
// (segment, group of 16); 64 groups of 16 lanes read 128-byte runs of the
// tile partials, then an LDS tree sums the groups (fixed order).
__global__ __launch_bounds__(1024) void bftail_kernel(const BDesc* __restrict__ d,
                                                      const BSeg* __restrict__ seg) {
  __shared__ double red[64][17];
  const BSeg& sg = seg[blockIdx.x];
  const BDesc& D = d[sg.inst];
  const int kk = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int k = blockIdx.y * 16 + kk;
  if (blockIdx.y * 16 >= D.ell) return;
  double s = 0.0;
  if (k < D.ell) {
    // eight loads in flight, added in tile order
    int64_t b = grp;
    for (; b + 7 * 64 < sg.nblk; b += 8 * 64) {
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = D.fpart[(b + 64 * i) * D.ell_pad + k];
#pragma unroll
      for (int i = 0; i < 8; ++i) s += v[i];
    }
    for (; b < sg.nblk; b += 64) s += D.fpart[b * D.ell_pad + k];
  }
  // the four groups of a wave by lane exchange, then the 16 waves in order
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) < 16) red[wave][kk] = s;
  __syncthreads();
  if (threadIdx.x < 16 && k < D.ell) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w][kk];
    D.cd[k] = D.meta[PcMeta::kD + k] * t;
  }
}

#undef BSEG_PROLOGUE

// ================================================================ autotuner
// Tile height per (row taps, column taps), chosen by timing the sketch items
// of that class at every candidate height; shared by the plans of a process.
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, int> g_tile_table;
constexpr int kTyCandidates[] = {8, 16, 32, 64};
constexpr int kTyDefault = 32;
// run lengths (output rows per item) of the streaming kernel
constexpr int kRunCandidates[] = {32, 64, 128, 256};
constexpr int kRunDefault = 64;

}  // namespace nys

using namespace nys;

// ================================================================ plan
struct nys_batch_s {
  nys_batch_opts o{};
  int count = 0;
  int nch = 2;
  DevBuf arena;
  DevBuf tables;
  int* ctr = nullptr;                        // stencil counters (in tables)
  std::vector<BDesc> hd;                     // host copy of the descriptors
  std::vector<int64_t> pix_off;              // packed offsets of the images
  int64_t P = 0;                             // packed image length
  BDesc* dd = nullptr;                       // device descriptors
  BLaunch pix, cmb, red, upix, fac, gram, ftl;
  BLaunch ftlk[3];                           // the tiles of the instances with 16, 32, 64 rows of U
  int kgroups = 0;
  int max_ell = 0;
  int64_t lds_doubles = 0;
  int64_t stencil_lds_max = 0;
  // stencil launches: tasks, items, queue bases, LDS bytes
  struct St {
    const StTask* tasks = nullptr;
    const StItem* items = nullptr;       // tile kernel items (queued)
    const int* qbase = nullptr;
    int64_t nitems = 0;
    size_t lds = 0;
    const StItem* sitems = nullptr;      // streaming kernel items
    int64_t nsitems = 0;
    bool sub = false;                    // tasks subtract an image
  } st_sketch, st_phi_v, st_grad, st_aty, st_hx;
  const float* taps = nullptr;
  std::vector<std::pair<int, int>> tiles;    // (taps class packed, ty) used
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool have_costs = false;
};

namespace nys {
namespace {

// Host builder of one device table region: appends POD arrays, 256-byte aligned.
// One fused dual iteration of every instance: a launch per row count of U
// (instances without tiles of that count are skipped).
template <int TW>
static nys_status bfused_launch_tw(const nys_batch_s* b, int reg, int qi, int ri, int qo, int ro,
                                   float beta, int last, hipStream_t st) {
  for (int c = 0; c < 3; ++c) {
    const BLaunch& l = b->ftlk[c];
    if (l.nblk == 0) continue;
    const int ntiles = static_cast<int>(l.nblk);
    const dim3 fg(static_cast<unsigned>((ntiles + 7) / 8 * 8));
    switch (c) {
      case 0: hipLaunchKernelGGL((bfused_kernel<TW, 16>), fg, dim3(kFThreads), 0, st, b->dd, l.seg, l.nseg, ntiles, reg, qi, ri, qo, ro, beta, last); break;
      case 1: hipLaunchKernelGGL((bfused_kernel<TW, 32>), fg, dim3(kFThreads), 0, st, b->dd, l.seg, l.nseg, ntiles, reg, qi, ri, qo, ro, beta, last); break;
      default: hipLaunchKernelGGL((bfused_kernel<TW, 64>), fg, dim3(kFThreads), 0, st, b->dd, l.seg, l.nseg, ntiles, reg, qi, ri, qo, ro, beta, last); break;
    }
    NYS_TRY(launch_check("bfused_kernel"));
  }
  return NYS_OK;
}

static nys_status bfused_launch(const nys_batch_s* b, int reg, int qi, int ri, int qo, int ro,
                                float beta, int last, hipStream_t st) {
  return reg_hessian(reg) ? bfused_launch_tw<fused_tw(true)>(b, reg, qi, ri, qo, ro, beta, last, st)
                          : bfused_launch_tw<fused_tw(false)>(b, reg, qi, ri, qo, ro, beta, last, st);
}

struct TableBuilder {
  std::vector<unsigned char> bytes;
  template <class T>
  size_t add(const std::vector<T>& v) {
    const size_t off = (bytes.size() + 255) / 256 * 256;
    bytes.resize(off + sizeof(T) * v.size());
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), sizeof(T) * v.size());
    return off;
  }
};

nys_status rank1_psf(const double* psf, int k, std::vector<double>& u, std::vector<double>& v) {
  int ap = 0, bp = 0;
  double mx = 0;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b)
      if (std::fabs(psf[a * k + b]) > mx) { mx = std::fabs(psf[a * k + b]); ap = a; bp = b; }
  NYS_REQUIRE(mx > 0, "batch_solve_create: zero PSF");
  u.assign(k, 0.0);
  v.assign(k, 0.0);
  for (int a = 0; a < k; ++a) u[a] = psf[a * k + bp];
  for (int b = 0; b < k; ++b) v[b] = psf[ap * k + b] / psf[ap * k + bp];
  double err = 0;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) err = std::fmax(err, std::fabs(psf[a * k + b] - u[a] * v[b]));
  NYS_REQUIRE(err <= 1e-12 * mx, "batch_solve_create: PSF is not separable (rank-1 residual %g)", err);
  return NYS_OK;
}

// r[d + k - 1] = sum_a w[a] w[a + d], d = -(k-1) .. k-1; r[-d] = r[d] is
// stored bit for bit (the sum is formed once per |d|)
std::vector<double> autocorr(const std::vector<double>& w) {
  const int k = static_cast<int>(w.size());
  std::vector<double> r(2 * k - 1, 0.0);
  for (int dd = 0; dd <= k - 1; ++dd) {
    double s = 0;
    for (int a = 0; a + dd < k; ++a) s += w[a] * w[a + dd];
    r[k - 1 + dd] = s;
    r[k - 1 - dd] = s;
  }
  return r;
}

// tiles of the fused inner iteration in an n1 x n2 image
int64_t batch_tiles(int n1, int n2, int reg) {
  const int tw = fused_tw(reg_hessian(reg));
  return static_cast<int64_t>(cdiv(n1, kFThreads / tw)) * static_cast<int64_t>(cdiv(n2, tw));
}

struct TaskSpec {
  StTask t;
  int ncols;
};

// Items of a list of tasks.  Tasks with equal odd row and column tap counts
// up to 29 go to the streaming kernel (strips of 128 columns, runs of ty
// rows), sorted by tap count, largest first (stable: neighbouring runs of a
// strip stay adjacent); the others to the tile kernel, split into kQueues
// contiguous queues.
void build_items(const std::vector<TaskSpec>& ts, std::vector<StItem>& items,
                 std::vector<int>& qbase, std::vector<StItem>& sitems) {
  items.clear();
  sitems.clear();
  for (size_t i = 0; i < ts.size(); ++i) {
    const StTask& t = ts[i].t;
    if (t.ss) {
      // runs of a strip consecutive: a run's window overlaps the previous
      // run's by NT - 1 rows
      for (int c = 0; c < ts[i].ncols; ++c)
        for (int x0 = 0; x0 < t.n2; x0 += kSsW)
          for (int y0 = 0; y0 < t.n1; y0 += t.ty) sitems.push_back({static_cast<int32_t>(i), c, y0, x0});
    } else {
      for (int c = 0; c < ts[i].ncols; ++c)
        for (int y0 = 0; y0 < t.n1; y0 += t.ty)
          for (int x0 = 0; x0 < t.n2; x0 += kStW) items.push_back({static_cast<int32_t>(i), c, y0, x0});
    }
  }
  std::stable_sort(sitems.begin(), sitems.end(), [&](const StItem& a, const StItem& b) {
    return ts[a.task].t.nt_r > ts[b.task].t.nt_r;
  });
  qbase.assign(kQueues + 1, 0);
  const int64_t n = static_cast<int64_t>(items.size());
  for (int q = 0; q <= kQueues; ++q) qbase[q] = static_cast<int>(n * q / kQueues);
}

size_t tasks_lds(const std::vector<TaskSpec>& ts) {
  size_t m = 0;
  for (const auto& s : ts)
    if (!s.t.ss)
      m = std::max<size_t>(m, sizeof(float) * st_lds_floats(s.t.ty, s.t.nt_r, s.t.nt_c));
  return m;
}

int stencil_grid(size_t lds) {
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t per_cu = 160 * 1024;
  int bpc = lds > 0 ? static_cast<int>(per_cu / (lds + 1024)) : 8;
  bpc = std::max(1, std::min(8, bpc));
  return ncu * bpc;
}

nys_status stencil_launch(const nys_batch_s::St& s, const float* taps, int* ctr, hipStream_t st) {
  if (s.nsitems > 0) {
    const dim3 grid(static_cast<unsigned>(ss_grid(s.nsitems)));
    if (s.sub)
      hipLaunchKernelGGL(bstream_kernel<true>, grid, dim3(64), 0, st, s.tasks, s.sitems, taps,
                         static_cast<int>(s.nsitems));
    else
      hipLaunchKernelGGL(bstream_kernel<false>, grid, dim3(64), 0, st, s.tasks, s.sitems, taps,
                         static_cast<int>(s.nsitems));
    NYS_TRY(launch_check("bstream_kernel"));
  }
  if (s.nitems == 0) return NYS_OK;
  hipLaunchKernelGGL(bstencil_kernel, dim3(stencil_grid(s.lds)), dim3(256), s.lds, st, s.tasks,
                     s.items, s.qbase, taps, ctr);
  return launch_check("bstencil_kernel");
}

}  // namespace
}  // namespace nys

namespace {

using namespace nys;

nys_status plan_destroy(nys_batch_s* b) {
  if (!b) return NYS_OK;
  if (b->cs) (void)hipStreamSynchronize(b->cs);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  b->arena.release();
  b->tables.release();
  delete b;
  return NYS_OK;
}

// Capture the whole pipeline on b->cs.
nys_status enqueue_all(nys_batch_s* b) {
  hipStream_t st = b->cs;
  const nys_batch_opts& o = b->o;
  const bool pc = o.precondition != 0;
  const BDesc* d = b->dd;
  const int nseg = b->pix.nseg;
  const int reg = o.reg;
  // ---- sketch and factorisation (Alg. 1)
  if (pc) {
    NYS_TRY(stencil_launch(b->st_sketch, b->taps, b->ctr, st));
    NYS_TRY(batch_factor_enqueue(d, b->gram, b->fac, b->upix, b->kgroups, b->max_ell,
                                 b->lds_doubles, o.nu_mode, o.tail, o.mu, 6, st));
  }
  // ---- power method on P^{-1} A^T A
  const dim3 pg(static_cast<unsigned>(b->pix.nblk));
  hipLaunchKernelGGL(bsumsq_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, -1);
  NYS_TRY(launch_check("bsumsq_kernel"));
  hipLaunchKernelGGL(bpart_tail_kernel, dim3(nseg), dim3(256), 0, st, d, b->pix.seg, 0, 0);
  NYS_TRY(launch_check("bpart_tail_kernel"));
  hipLaunchKernelGGL(bnormalize_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, -1, int(kFldV));
  NYS_TRY(launch_check("bnormalize_kernel"));
  for (int it = 0; it < o.power_iters; ++it) {
    NYS_TRY(stencil_launch(b->st_phi_v, b->taps, b->ctr, st));
    if (pc) {
      NYS_TRY(batch_pinv_coeffs(d, b->red.seg, b->red.nseg, b->red.nblk, kFldW, st));
      NYS_TRY(batch_combine(d, b->cmb.seg, b->cmb.nseg, b->cmb.nblk, -1, kFldW, kFldW, -1, st));
    }
    hipLaunchKernelGGL(bsumsq_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, int(kFldW));
    NYS_TRY(launch_check("bsumsq_kernel"));
    hipLaunchKernelGGL(bpart_tail_kernel, dim3(nseg), dim3(256), 0, st, d, b->pix.seg, 0, 0);
    NYS_TRY(launch_check("bpart_tail_kernel"));
    hipLaunchKernelGGL(bnormalize_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, int(kFldW),
                       int(kFldV));
    NYS_TRY(launch_check("bnormalize_kernel"));
  }
  const double safety = o.safety > 0 ? o.safety : 1.01;
  const double lnorm2 = reg_hessian(reg) ? 34.0 : 8.0;
  hipLaunchKernelGGL(bscalars_kernel, dim3(cdiv(b->count, 64)), dim3(64), 0, st, d, b->count,
                     safety, lnorm2);
  NYS_TRY(launch_check("bscalars_kernel"));
  // ---- WAPG (Alg. 3) from x = u = 0, dual variable 0
  NYS_TRY(stencil_launch(b->st_aty, b->taps, b->ctr, st));
  const BDesc& d0 = b->hd[0];
  NYS_TRY(fill_zero<float>(d0.f[kFldX], b->P, st));
  NYS_TRY(fill_zero<float>(d0.f[kFldU], b->P, st));
  NYS_TRY(fill_zero<float>(d0.f[kFldQ], static_cast<size_t>(b->nch) * b->P, st));
  const dim3 ig(static_cast<unsigned>(b->hd.size()));
  if (pc) {
    hipLaunchKernelGGL(bcq_kernel, ig, dim3(64), 0, st, d, 0);
    NYS_TRY(launch_check("bcq_kernel"));
  }
  const int term = reg_term_of(reg);
  double t_prev = 1.0;
  for (int k = 0; k < o.max_iter; ++k) {
    // s = u - alpha P^{-1} A^T (A u - y), with A^T A u - A^T y from one stencil pass
    NYS_TRY(stencil_launch(b->st_grad, b->taps, b->ctr, st));
    if (pc) NYS_TRY(batch_pinv_coeffs(d, b->red.seg, b->red.nseg, b->red.nblk, kFldG, st));
    NYS_TRY(batch_combine(d, b->cmb.seg, b->cmb.nseg, b->cmb.nblk, kFldU, kFldG, kFldS, BScal::kAlpha, st));
    // x+ = prox^P_{lam_bar g}(s): accelerated projected gradient on the dual
    if (!o.warm_start) NYS_TRY(fill_zero<float>(d0.f[kFldQ], static_cast<size_t>(b->nch) * b->P, st));
    if (pc) {
      // with P^{-1} inside: the warm start's coefficients (kept from the
      // last prox, whose final Q this one starts from), then one fused
      // launch per row count and the coefficient tail per dual iteration
      // (R = Q at the start; the duals alternate between Q, R and Q2, R2)
      hipLaunchKernelGGL(bcq_kernel, ig, dim3(64), 0, st, d, o.warm_start ? 1 : 3);
      NYS_TRY(launch_check("bcq_kernel"));
      int qi = kFldQ, ri = kFldQ;
      double tau = 1.0;
      const dim3 tg(static_cast<unsigned>(b->ftl.nseg), static_cast<unsigned>(cdiv(b->max_ell, 16)));
      for (int it = 0; it < o.n_inner; ++it) {
        const double tau_n = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
        const double beta = (tau - 1.0) / tau_n;
        const int qo = (it & 1) ? kFldQ : kFldQ2;
        const int ro = (it & 1) ? kFldR2 : kFldR;
        NYS_TRY(bfused_launch(b, reg, qi, ri, qo, ro, static_cast<float>(beta),
                              int(it == o.n_inner - 1), st));
        hipLaunchKernelGGL(bftail_kernel, tg, dim3(1024), 0, st, d, b->ftl.seg);
        NYS_TRY(launch_check("bftail_kernel"));
        qi = qo;
        ri = ro;
        tau = tau_n;
      }
      hipLaunchKernelGGL(bcq_kernel, ig, dim3(64), 0, st, d, 2);
      NYS_TRY(launch_check("bcq_kernel"));
      if (qi != kFldQ)
        NYS_CHECK_HIP(hipMemcpyAsync(d0.f[kFldQ], d0.f[qi], sizeof(float) * b->nch * b->P,
                                     hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(blt_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, reg, int(kFldQ),
                         int(kFldT));
      NYS_TRY(launch_check("blt_kernel"));
      NYS_TRY(batch_combine(d, b->cmb.seg, b->cmb.nseg, b->cmb.nblk, kFldS, kFldT, kFldXN, BScal::kLamBar, st));
    } else {
      NYS_CHECK_HIP(hipMemcpyAsync(d0.f[kFldR], d0.f[kFldQ], sizeof(float) * b->nch * b->P,
                                   hipMemcpyDeviceToDevice, st));
      double tau = 1.0;
      for (int it = 0; it <= o.n_inner; ++it) {
        const bool last = it == o.n_inner;
        hipLaunchKernelGGL(blt_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, reg,
                           int(last ? kFldQ : kFldR), int(kFldT));
        NYS_TRY(launch_check("blt_kernel"));
        NYS_TRY(batch_combine(d, b->cmb.seg, b->cmb.nseg, b->cmb.nblk, kFldS, kFldT, kFldXN, BScal::kLamBar, st));
        if (last) break;
        const double tau_n = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
        const double beta = (tau - 1.0) / tau_n;
        hipLaunchKernelGGL(bdual_update_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, reg,
                           static_cast<float>(beta));
        NYS_TRY(launch_check("bdual_update_kernel"));
        tau = tau_n;
      }
    }
    const double t = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t_prev * t_prev));
    const double beta = (t_prev - 1.0) / t;
    hipLaunchKernelGGL(bmomentum_kernel, dim3(std::min<int64_t>(cdiv(b->P, 256), 4096)), dim3(256),
                       0, st, d0.f[kFldXN], d0.f[kFldX], d0.f[kFldU], static_cast<float>(beta), b->P);
    NYS_TRY(launch_check("bmomentum_kernel"));
    t_prev = t;
    if (b->have_costs) {
      NYS_TRY(stencil_launch(b->st_hx, b->taps, b->ctr, st));
      hipLaunchKernelGGL(bcost_partial_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg, term);
      NYS_TRY(launch_check("bcost_partial_kernel"));
      hipLaunchKernelGGL(bpart_tail_kernel, dim3(nseg), dim3(256), 0, st, d, b->pix.seg, 1, k);
      NYS_TRY(launch_check("bpart_tail_kernel"));
    }
  }
  hipLaunchKernelGGL(bcopy_out_kernel, pg, dim3(256), 0, st, d, b->pix.seg, nseg);
  return launch_check("bcopy_out_kernel");
}

}  // namespace

extern "C" nys_status batch_solve_create(const nys_batch_item* items, int32_t count,
                                         const nys_batch_opts* opts, nys_batch* out,
                                         void* stream) {
  NYS_REQUIRE(items && opts && out && count >= 1, "batch_solve_create: bad argument");
  const nys_batch_opts o = *opts;
  NYS_REQUIRE(o.reg == NYS_REG_TV || o.reg == NYS_REG_TV_ANISO || reg_hessian(o.reg),
              "batch_solve_create: reg must be TV, TV_ANISO, HS1, HS2 or HSINF");
  NYS_REQUIRE(o.max_iter >= 0 && o.n_inner >= 0 && o.power_iters >= 1,
              "batch_solve_create: bad iteration counts");
  NYS_REQUIRE(o.nu_mode == 0 || o.nu_mode == 1, "batch_solve_create: nu_mode must be 0 or 1");
  NYS_REQUIRE(o.tail == 0 || o.tail == 1, "batch_solve_create: tail must be 0 or 1");
  const bool pc = o.precondition != 0;
  hipStream_t ust = as_stream(stream);
  auto* b = new nys_batch_s();
  b->o = o;
  b->count = count;
  b->nch = reg_hessian(o.reg) ? 3 : 2;
  auto fail = [&](nys_status s) { plan_destroy(b); return s; };

  // ---- per-instance sizes, taps
  std::vector<double> tap_host;
  std::vector<int> taps_aa(count), taps_h(count), taps_hf(count), kk(count);
  b->pix_off.resize(count);
  int64_t P = 0;
  int max_ell = 0;
  for (int i = 0; i < count; ++i) {
    const nys_batch_item& it = items[i];
    if (!(it.n1 >= 1 && it.n2 >= 1 && (static_cast<int64_t>(it.n1) * it.n2) % 4 == 0)) {
      set_error("batch_solve_create: item %d: n1 * n2 must be a positive multiple of 4", i);
      return fail(NYS_EINVAL);
    }
    if (!(it.psf_k >= 1 && it.psf_k <= 31 && it.psf_k % 2 == 1 && it.psf)) {
      set_error("batch_solve_create: item %d: psf_k must be odd in [1, 31]", i);
      return fail(NYS_EINVAL);
    }
    if (!it.y || !it.v0 || !it.x || !(it.lambda >= 0)) {
      set_error("batch_solve_create: item %d: y, v0, x and lambda >= 0 are required", i);
      return fail(NYS_EINVAL);
    }
    if (pc && !(it.ell >= 1 && it.ell <= 64 && it.omega &&
                (reinterpret_cast<uintptr_t>(it.omega) & 15) == 0 &&
                it.ell <= static_cast<int64_t>(it.n1) * it.n2)) {
      set_error("batch_solve_create: item %d: ell in [1, 64] and a 16-byte aligned omega are required", i);
      return fail(NYS_EINVAL);
    }
    std::vector<double> u, v;
    nys_status s = rank1_psf(it.psf, it.psf_k, u, v);
    if (s != NYS_OK) return fail(s);
    const int k = it.psf_k;
    kk[i] = k;
    // A^T A: correlation with (u * u)(v * v)^T over offsets -(k-1)..(k-1)
    const std::vector<double> ru = autocorr(u), rv = autocorr(v);
    taps_aa[i] = static_cast<int>(tap_host.size());
    tap_host.insert(tap_host.end(), ru.begin(), ru.end());
    tap_host.insert(tap_host.end(), rv.begin(), rv.end());
    // H^T: correlation with the PSF (u, v), offsets -c..k-1-c
    taps_h[i] = static_cast<int>(tap_host.size());
    tap_host.insert(tap_host.end(), u.begin(), u.end());
    tap_host.insert(tap_host.end(), v.begin(), v.end());
    // H: correlation with the flipped PSF
    taps_hf[i] = static_cast<int>(tap_host.size());
    tap_host.insert(tap_host.end(), u.rbegin(), u.rend());
    tap_host.insert(tap_host.end(), v.rbegin(), v.rend());
    b->pix_off[i] = P;
    P += (static_cast<int64_t>(it.n1) * it.n2 + 63) / 64 * 64;
    if (pc) max_ell = std::max(max_ell, it.ell);
    if (it.costs) b->have_costs = true;
  }
  b->P = P;

  // ---- arena layout
  struct Off { size_t Y, U, meta, G, gpart, fwork, part, fpart, cd, cq, scal; };
  std::vector<Off> off(count);
  size_t cur = 0;
  auto take = [&](size_t bytes) { size_t o0 = cur; cur += (bytes + 255) / 256 * 256; return o0; };
  const size_t fields_off = take(0);
  cur += 0;
  size_t field_off[kNumFields];
  for (int f = 0; f < kNumFields; ++f) {
    const int ch = field_is_dual(f) ? b->nch : 1;
    field_off[f] = take(sizeof(float) * ch * P);
  }
  (void)fields_off;
  std::vector<int64_t> red_nblk(count), red_chunk(count), gram_nblk(count), gram_chunk(count);
  for (int i = 0; i < count; ++i) {
    const nys_batch_item& it = items[i];
    const int64_t N = static_cast<int64_t>(it.n1) * it.n2;
    const int ell = pc ? it.ell : 0;
    // rows of U rounded to 16, 32 or 64 (zero padding) for the U^T v kernel
    const int ell_pad = ell == 0 ? 0 : ell <= 16 ? 16 : ell <= 32 ? 32 : 64;
    const int64_t ldu = (N + 63) / 64 * 64 + (N >= 16384 ? 96 : 0);
    // U^T v reduction: chunks of 8192 pixels
    int64_t ch = 8192;
    red_nblk[i] = (N + ch - 1) / ch;
    red_chunk[i] = ch;
    int64_t nb;
    // Gram: <= 256 chunks of >= 4096 pixels, chunk a multiple of 32;
    // 64 x 64 tile pairs of the 2 ell x 2 ell result
    nb = std::min<int64_t>(256, std::max<int64_t>(1, N / 4096));
    ch = ((N + nb - 1) / nb + 31) / 32 * 32;
    gram_nblk[i] = (N + ch - 1) / ch;
    gram_chunk[i] = ch;
    const int ntl = (2 * ell + 63) / 64;
    const int ntri = ntl * (ntl + 1) / 2;
    const int64_t pblk = (N + 1023) / 1024;
    Off& q = off[i];
    q.Y = take(sizeof(float) * ell * N);
    q.U = take(sizeof(float) * ldu * std::max(ell_pad, 1));
    q.meta = take(sizeof(double) * PcMeta::kTotal);
    q.G = take(sizeof(double) * 4 * ell * ell);
    q.gpart = take(sizeof(double) * gram_nblk[i] * ntri * 4096);
    q.fwork = take(sizeof(double) * (5 * ell * ell + ell + 1));
    q.part = take(sizeof(double) * std::max<int64_t>(red_nblk[i] * std::max(ell_pad, 16), pblk));
    q.fpart = take(ell > 0 ? sizeof(double) * batch_tiles(it.n1, it.n2, o.reg) * ell_pad : 0);
    q.cd = take(sizeof(double) * std::max(ell_pad, 16));
    q.cq = take(sizeof(double) * std::max(ell_pad, 16));
    q.scal = take(sizeof(double) * BScal::kTotal);
    BDesc D{};
    D.n1 = it.n1;
    D.n2 = it.n2;
    D.N = N;
    D.ell = ell;
    D.ell_pad = ell_pad;
    D.ldu = ldu;
    D.lambda = it.lambda;
    b->hd.push_back(D);
  }
  {
    nys_status s = b->arena.ensure(cur + 256);
    if (s != NYS_OK) return fail(s);
    if (hipMemsetAsync(b->arena.p, 0, cur, ust) != hipSuccess) {
      set_error("batch_solve_create: clearing the arena failed");
      return fail(NYS_EHIP);
    }
  }
  char* A = b->arena.as<char>();
  for (int i = 0; i < count; ++i) {
    BDesc& D = b->hd[i];
    const nys_batch_item& it = items[i];
    const Off& q = off[i];
    D.omega = pc ? it.omega : nullptr;
    D.y = it.y;
    D.v0 = it.v0;
    D.Y = reinterpret_cast<float*>(A + q.Y);
    D.U = reinterpret_cast<float*>(A + q.U);
    D.meta = reinterpret_cast<double*>(A + q.meta);
    D.G = reinterpret_cast<double*>(A + q.G);
    D.gpart = reinterpret_cast<double*>(A + q.gpart);
    D.fwork = reinterpret_cast<double*>(A + q.fwork);
    D.part = reinterpret_cast<double*>(A + q.part);
    D.fpart = reinterpret_cast<double*>(A + q.fpart);
    D.cd = reinterpret_cast<double*>(A + q.cd);
    D.cq = reinterpret_cast<double*>(A + q.cq);
    D.scal = reinterpret_cast<double*>(A + q.scal);
    D.costs = it.costs;
    D.x_out = it.x;
    for (int f = 0; f < kNumFields; ++f) {
      const int ch = field_is_dual(f) ? b->nch : 1;
      D.f[f] = reinterpret_cast<float*>(A + field_off[f]) + ch * b->pix_off[i];
    }
  }

  // ---- segment tables
  auto segs = [&](const std::vector<int>& inst, auto nblk_of, auto chunk_of) {
    std::vector<BSeg> v;
    int64_t first = 0;
    for (int i : inst) {
      BSeg s{};
      s.first = first;
      s.nblk = nblk_of(i);
      s.chunk = chunk_of(i);
      s.inst = i;
      v.push_back(s);
      first += s.nblk;
    }
    return std::make_pair(v, first);
  };
  std::vector<int> all(count);
  for (int i = 0; i < count; ++i) all[i] = i;
  auto pixs = segs(all, [&](int i) { return (b->hd[i].N + 1023) / 1024; }, [](int) { return int64_t(1024); });
  auto cmbs = segs(all, [&](int i) { return (b->hd[i].N + 4095) / 4096; }, [](int) { return int64_t(4096); });
  auto reds = segs(all, [&](int i) { return red_nblk[i]; }, [&](int i) { return red_chunk[i]; });
  auto upxs = segs(all, [&](int i) { return (b->hd[i].N + 255) / 256; }, [](int) { return int64_t(256); });
  auto facs = segs(all, [](int) { return int64_t(1); }, [](int) { return int64_t(0); });
  auto grms = segs(all, [&](int i) { return gram_nblk[i]; }, [&](int i) { return gram_chunk[i]; });
  auto ftls = segs(all, [&](int i) { return batch_tiles(b->hd[i].n1, b->hd[i].n2, o.reg); },
                   [](int) { return int64_t(kFThreads); });
  std::pair<std::vector<BSeg>, int64_t> ftlks[3];
  for (int c = 0; c < 3; ++c) {
    std::vector<int> inst;
    for (int i = 0; i < count; ++i)
      if (b->hd[i].ell_pad == (16 << c)) inst.push_back(i);
    ftlks[c] = segs(inst, [&](int i) { return batch_tiles(b->hd[i].n1, b->hd[i].n2, o.reg); },
                    [](int) { return int64_t(kFThreads); });
  }

  // ---- stencil tasks (tile heights from the autotuner table)
  // tuner classes: (row taps, column taps + 65536 for the streaming kernel)
  auto tkey = [](const StTask& t) { return std::make_pair(t.nt_r, t.nt_c + (t.ss ? 65536 : 0)); };
  auto ty_for = [&](const StTask& t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto itr = g_tile_table.find(tkey(t));
    if (itr != g_tile_table.end()) return itr->second;
    return t.ss ? kRunDefault : kTyDefault;
  };
  auto mk = [&](int i, const float* in, float* outp, const float* sub, int64_t cstride, int ncols,
                int which) {
    const BDesc& D = b->hd[i];
    const int k = kk[i], c = (k - 1) / 2;
    TaskSpec s{};
    s.t.in = in;
    s.t.out = outp;
    s.t.sub = sub;
    s.t.cstride = cstride;
    s.t.n1 = D.n1;
    s.t.n2 = D.n2;
    if (which == 0) {           // A^T A
      s.t.lo_r = -(k - 1); s.t.nt_r = 2 * k - 1; s.t.lo_c = -(k - 1); s.t.nt_c = 2 * k - 1;
      s.t.taps = taps_aa[i];
    } else {                    // H^T (which 1) or H (which 2)
      s.t.lo_r = -c; s.t.nt_r = k; s.t.lo_c = -c; s.t.nt_c = k;
      s.t.taps = which == 1 ? taps_h[i] : taps_hf[i];
    }
    s.t.ss = ss_eligible(s.t.nt_r, s.t.nt_c, s.t.lo_c, s.t.n2,
                         taps_palindromic(tap_host, s.t.taps, s.t.nt_r, s.t.nt_c));
    s.t.ty = ty_for(s.t);
    s.ncols = ncols;
    return s;
  };
  std::vector<TaskSpec> t_sketch, t_phi, t_grad, t_aty, t_hx;
  for (int i = 0; i < count; ++i) {
    BDesc& D = b->hd[i];
    if (pc) t_sketch.push_back(mk(i, D.omega, D.Y, nullptr, D.N, D.ell, 0));
    t_phi.push_back(mk(i, D.f[kFldV], D.f[kFldW], nullptr, D.N, 1, 0));
    t_grad.push_back(mk(i, D.f[kFldU], D.f[kFldG], D.f[kFldB], D.N, 1, 0));
    t_aty.push_back(mk(i, D.y, D.f[kFldB], nullptr, D.N, 1, 1));
    t_hx.push_back(mk(i, D.f[kFldX], D.f[kFldW], nullptr, D.N, 1, 2));
  }
  std::vector<float> tapf(tap_host.begin(), tap_host.end());

  // device tables: taps, descriptors, segments, counters, then the stencil
  // tables (rebuilt after tuning)
  auto upload_tables = [&](bool with_stencils) -> nys_status {
    TableBuilder tb;
    const size_t o_taps = tb.add(tapf);
    const size_t o_desc = tb.add(b->hd);
    const size_t o_pix = tb.add(pixs.first);
    const size_t o_cmb = tb.add(cmbs.first);
    const size_t o_red = tb.add(reds.first);
    const size_t o_upx = tb.add(upxs.first);
    const size_t o_fac = tb.add(facs.first);
    const size_t o_gram = tb.add(grms.first);
    const size_t o_ftl = tb.add(ftls.first);
    size_t o_ftlk[3];
    for (int c = 0; c < 3; ++c) o_ftlk[c] = tb.add(ftlks[c].first);
    const size_t o_ctr = tb.add(std::vector<int>(kQueues + 1 + 63, 0));
    struct StOff { size_t tasks, items, qbase, sitems; int64_t n, ns; size_t lds; bool sub; };
    std::vector<TaskSpec>* lists[5] = {&t_sketch, &t_phi, &t_grad, &t_aty, &t_hx};
    StOff so[5] = {};
    if (with_stencils) {
      for (int l = 0; l < 5; ++l) {
        std::vector<StTask> tv;
        for (auto& s : *lists[l]) tv.push_back(s.t);
        std::vector<StItem> iv, sv;
        std::vector<int> qb;
        build_items(*lists[l], iv, qb, sv);
        so[l].tasks = tb.add(tv);
        so[l].items = tb.add(iv);
        so[l].qbase = tb.add(qb);
        so[l].sitems = tb.add(sv);
        so[l].n = static_cast<int64_t>(iv.size());
        so[l].ns = static_cast<int64_t>(sv.size());
        so[l].lds = tasks_lds(*lists[l]);
        so[l].sub = !tv.empty() && tv[0].sub != nullptr;
      }
    }
    NYS_TRY(b->tables.ensure(tb.bytes.size() + 256));
    NYS_CHECK_HIP(hipMemcpyAsync(b->tables.p, tb.bytes.data(), tb.bytes.size(),
                                 hipMemcpyHostToDevice, ust));
    NYS_CHECK_HIP(hipStreamSynchronize(ust));
    char* T = b->tables.as<char>();
    b->taps = reinterpret_cast<const float*>(T + o_taps);
    b->dd = reinterpret_cast<BDesc*>(T + o_desc);
    b->pix = {reinterpret_cast<const BSeg*>(T + o_pix), static_cast<int>(pixs.first.size()), pixs.second};
    b->cmb = {reinterpret_cast<const BSeg*>(T + o_cmb), static_cast<int>(cmbs.first.size()), cmbs.second};
    b->red = {reinterpret_cast<const BSeg*>(T + o_red), static_cast<int>(reds.first.size()), reds.second};
    b->upix = {reinterpret_cast<const BSeg*>(T + o_upx), static_cast<int>(upxs.first.size()), upxs.second};
    b->fac = {reinterpret_cast<const BSeg*>(T + o_fac), pc ? static_cast<int>(facs.first.size()) : 0, facs.second};
    b->gram = {reinterpret_cast<const BSeg*>(T + o_gram), static_cast<int>(grms.first.size()),
               grms.second};
    b->ftl = {reinterpret_cast<const BSeg*>(T + o_ftl), static_cast<int>(ftls.first.size()), ftls.second};
    for (int c = 0; c < 3; ++c)
      b->ftlk[c] = {reinterpret_cast<const BSeg*>(T + o_ftlk[c]), static_cast<int>(ftlks[c].first.size()),
                    ftlks[c].second};
    b->ctr = reinterpret_cast<int*>(T + o_ctr);
    nys_batch_s::St* sts[5] = {&b->st_sketch, &b->st_phi_v, &b->st_grad, &b->st_aty, &b->st_hx};
    for (int l = 0; l < 5; ++l) {
      sts[l]->tasks = reinterpret_cast<const StTask*>(T + so[l].tasks);
      sts[l]->items = reinterpret_cast<const StItem*>(T + so[l].items);
      sts[l]->qbase = reinterpret_cast<const int*>(T + so[l].qbase);
      sts[l]->nitems = with_stencils ? so[l].n : 0;
      sts[l]->lds = so[l].lds;
      sts[l]->sitems = reinterpret_cast<const StItem*>(T + so[l].sitems);
      sts[l]->nsitems = with_stencils ? so[l].ns : 0;
      sts[l]->sub = so[l].sub;
    }
    return NYS_OK;
  };
  {
    nys_status s = upload_tables(false);
    if (s != NYS_OK) return fail(s);
  }
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(bstencil_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(sizeof(float) * st_lds_floats(64, kStMaxTaps, kStMaxTaps))) !=
      hipSuccess) {
    set_error("batch_solve_create: hipFuncSetAttribute failed");
    return fail(NYS_EHIP);
  }

  // ---- autotuner: time every candidate tile height on the sketch items of
  // each tap class not yet in the table (A^T A columns of the real inputs)
  if (o.tune && pc) {
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (size_t i = 0; i < t_sketch.size(); ++i)
      classes[tkey(t_sketch[i].t)].push_back(static_cast<int>(i));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      set_error("batch_solve_create: hipEventCreate failed");
      return fail(NYS_EHIP);
    }
    DevBuf tb;
    for (auto& cl : classes) {
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tile_table.count(cl.first)) continue;
      }
      const bool ss = cl.first.second >= 65536;
      double best_t = 1e300;
      int best_ty = ss ? kRunDefault : kTyDefault;
      std::vector<int> cands;
      if (ss) cands.assign(std::begin(kRunCandidates), std::end(kRunCandidates));
      else cands.assign(std::begin(kTyCandidates), std::end(kTyCandidates));
      for (int ty : cands) {
        std::vector<TaskSpec> ts;
        for (int i : cl.second) {
          TaskSpec s = t_sketch[i];
          s.t.ty = ty;
          ts.push_back(s);
        }
        std::vector<StTask> tv;
        for (auto& s : ts) tv.push_back(s.t);
        std::vector<StItem> iv, sv;
        std::vector<int> qb;
        build_items(ts, iv, qb, sv);
        TableBuilder tbb;
        const size_t ot = tbb.add(tv), oi = tbb.add(iv), oq = tbb.add(qb), os = tbb.add(sv);
        if (tb.ensure(tbb.bytes.size() + 256) != NYS_OK ||
            hipMemcpyAsync(tb.p, tbb.bytes.data(), tbb.bytes.size(), hipMemcpyHostToDevice, ust) != hipSuccess) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          tb.release();
          set_error("batch_solve_create: autotuner upload failed");
          return fail(NYS_EHIP);
        }
        nys_batch_s::St s;
        s.tasks = reinterpret_cast<const StTask*>(tb.as<char>() + ot);
        s.items = reinterpret_cast<const StItem*>(tb.as<char>() + oi);
        s.qbase = reinterpret_cast<const int*>(tb.as<char>() + oq);
        s.nitems = static_cast<int64_t>(iv.size());
        s.lds = tasks_lds(ts);
        s.sitems = reinterpret_cast<const StItem*>(tb.as<char>() + os);
        s.nsitems = static_cast<int64_t>(sv.size());
        float ms = 0;
        nys_status st2 = stencil_launch(s, b->taps, b->ctr, ust);        // warm-up
        if (st2 == NYS_OK && hipEventRecord(e0, ust) == hipSuccess) {
          for (int rep = 0; rep < 3 && st2 == NYS_OK; ++rep) st2 = stencil_launch(s, b->taps, b->ctr, ust);
          if (st2 == NYS_OK && (hipEventRecord(e1, ust) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st2 = NYS_EHIP;
        }
        if (st2 != NYS_OK) {
          (void)hipStreamSynchronize(ust);
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          tb.release();
          return fail(st2 == NYS_EHIP ? NYS_EHIP : st2);
        }
        if (ms < best_t) { best_t = ms; best_ty = ty; }
      }
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tile_table[cl.first] = best_ty;
    }
    (void)hipStreamSynchronize(ust);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tb.release();
    // re-derive tile heights from the table
    for (auto* l : {&t_sketch, &t_phi, &t_grad, &t_aty, &t_hx})
      for (auto& s : *l) s.t.ty = ty_for(s.t);
  }
  for (auto* l : {&t_sketch, &t_phi, &t_grad, &t_aty, &t_hx})
    for (auto& s : *l) {
      const int key = s.t.nt_r * 256 + s.t.nt_c;
      bool seen = false;
      for (auto& pr : b->tiles) seen |= pr.first == key;
      if (!seen) b->tiles.push_back({key, s.t.ty});
    }
  {
    nys_status s = upload_tables(true);
    if (s != NYS_OK) return fail(s);
  }

  // ---- batched factor: LDS for up to four ell x ell FP64 matrices
  if (pc) {
    int dev = 0, maxsh = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const int64_t avail = maxsh > 8192 ? (maxsh - 8192) / 8 : 0;
    const int64_t want = 4 * static_cast<int64_t>(max_ell) * max_ell;
    b->lds_doubles = std::min(avail, want);
    b->kgroups = (max_ell + 31) / 32;
    b->max_ell = max_ell;
    nys_status s = batch_factor_prepare(b->lds_doubles * 8);
    if (s != NYS_OK) return fail(s);
  }

  // ---- capture the pipeline
  if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess) {
    set_error("batch_solve_create: hipStreamCreate failed");
    return fail(NYS_EHIP);
  }
  if (hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("batch_solve_create: hipStreamBeginCapture failed");
    return fail(NYS_EHIP);
  }
  nys_status es = enqueue_all(b);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->cs, &g);
  if (es != NYS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return fail(es);
  }
  if (ee != hipSuccess || !g) {
    set_error("batch_solve_create: hipStreamEndCapture failed: %s", hipGetErrorString(ee));
    return fail(NYS_EHIP);
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    set_error("batch_solve_create: hipGraphInstantiate failed");
    return fail(NYS_EHIP);
  }
  *out = b;
  return NYS_OK;
}

extern "C" nys_status batch_solve_run(nys_batch b, void* stream) {
  NYS_REQUIRE(b && b->exec, "batch_solve_run: bad plan");
  NYS_CHECK_HIP(hipGraphLaunch(b->exec, as_stream(stream)));
  return NYS_OK;
}

extern "C" nys_status batch_solve_sketch(nys_batch b, void* stream) {
  NYS_REQUIRE(b && b->o.precondition, "batch_solve_sketch: plan without a preconditioner");
  return stencil_launch(b->st_sketch, b->taps, b->ctr, as_stream(stream));
}

extern "C" nys_status batch_solve_info(nys_batch b, int32_t i, double* out, void* stream) {
  NYS_REQUIRE(b && out && i >= 0 && i < b->count, "batch_solve_info: bad argument");
  NYS_CHECK_HIP(hipStreamSynchronize(as_stream(stream)));
  double sc[BScal::kTotal];
  NYS_CHECK_HIP(hipMemcpy(sc, b->hd[i].scal, sizeof sc, hipMemcpyDeviceToHost));
  double meta[PcMeta::kTotal] = {};
  if (b->hd[i].ell > 0)
    NYS_CHECK_HIP(hipMemcpy(meta, b->hd[i].meta, sizeof meta, hipMemcpyDeviceToHost));
  out[0] = sc[BScal::kAlpha];
  out[1] = sc[BScal::kL];
  out[2] = sc[BScal::kPinvNorm];
  out[3] = b->hd[i].ell > 0 ? meta[PcMeta::kNu] : 0.0;
  out[4] = b->hd[i].ell > 0 ? meta[PcMeta::kStatus] : static_cast<double>(NYS_OK);
  out[5] = b->hd[i].ell > 0 ? meta[PcMeta::kKeff] : 0.0;
  return NYS_OK;
}

extern "C" nys_status batch_solve_shat(nys_batch b, int32_t i, double* shat, void* stream) {
  NYS_REQUIRE(b && shat && i >= 0 && i < b->count && b->hd[i].ell > 0,
              "batch_solve_shat: bad argument");
  NYS_CHECK_HIP(hipStreamSynchronize(as_stream(stream)));
  NYS_CHECK_HIP(hipMemcpy(shat, b->hd[i].meta + PcMeta::kShat, sizeof(double) * b->hd[i].ell,
                          hipMemcpyDeviceToHost));
  return NYS_OK;
}

extern "C" nys_status batch_solve_buffers(nys_batch b, int32_t i, const float** Y, const float** U,
                                          int64_t* ldu) {
  NYS_REQUIRE(b && i >= 0 && i < b->count, "batch_solve_buffers: bad argument");
  if (Y) *Y = b->hd[i].ell > 0 ? b->hd[i].Y : nullptr;
  if (U) *U = b->hd[i].ell > 0 ? b->hd[i].U : nullptr;
  if (ldu) *ldu = b->hd[i].ldu;
  return NYS_OK;
}

extern "C" nys_status batch_solve_copy(nys_batch b, int32_t i, int32_t what, float* dst,
                                       void* stream) {
  NYS_REQUIRE(b && dst && i >= 0 && i < b->count && (what == 0 || what == 1) && b->hd[i].ell > 0,
              "batch_solve_copy: bad argument");
  const BDesc& D = b->hd[i];
  const size_t es = sizeof(float);
  if (what == 0)
    NYS_CHECK_HIP(hipMemcpyAsync(dst, D.Y, es * D.N * D.ell, hipMemcpyDeviceToDevice,
                                 as_stream(stream)));
  else
    NYS_CHECK_HIP(hipMemcpy2DAsync(dst, es * D.N, D.U, es * D.ldu, es * D.N, D.ell,
                                   hipMemcpyDeviceToDevice, as_stream(stream)));
  return NYS_OK;
}

extern "C" nys_status batch_solve_tiles(nys_batch b, int32_t* nt_r, int32_t* nt_c, int32_t* ty,
                                        int32_t cap, int32_t* count) {
  NYS_REQUIRE(b && count, "batch_solve_tiles: bad argument");
  const int n = static_cast<int>(b->tiles.size());
  for (int i = 0; i < n && i < cap; ++i) {
    if (nt_r) nt_r[i] = b->tiles[i].first / 256;
    if (nt_c) nt_c[i] = b->tiles[i].first % 256;
    if (ty) ty[i] = b->tiles[i].second;
  }
  *count = n;
  return NYS_OK;
}

extern "C" void batch_solve_destroy(nys_batch b) { plan_destroy(b); }
