// Device tables of the batched solver: one descriptor per reconstruction and
// segment tables that map the blocks of a batched launch to instances.
//
// A batched launch covers many instances of different sizes with one grid.
// Its segment table lists, per instance, the first block and the number of
// blocks (and the pixel chunk each block owns); a block finds its instance by
// a binary search over the first-block column.  Every per-instance buffer
// sits in one arena, and the images of all instances are packed one after
// another so that purely elementwise steps run as one flat launch.
#pragma once

#include "common.hpp"

namespace nys {

// Image fields of a batched instance (all N floats, Q and R nch * N).
// Q2 / R2: the second dual buffers of the fused inner iteration.
enum BField {
  kFldX = 0, kFldU, kFldG, kFldS, kFldXN, kFldT, kFldB, kFldV, kFldW, kFldQ, kFldR, kFldQ2, kFldR2,
  kNumFields
};
__host__ __device__ inline bool field_is_dual(int f) {
  return f == kFldQ || f == kFldR || f == kFldQ2 || f == kFldR2;
}

// Per-instance FP64 scalars produced on the device.
struct BScal {
  static constexpr int kL = 0;         // power-method estimate of L_f^P
  static constexpr int kAlpha = 1;     // WAPG step 1 / (safety L)
  static constexpr int kLamBar = 2;    // alpha * lambda
  static constexpr int kDualStep = 3;  // dual step of the P-weighted prox
  static constexpr int kPinvNorm = 4;  // ||P^{-1}||_2 (1 without a preconditioner)
  static constexpr int kNorm = 5;      // last power-method norm
  static constexpr int kTotal = 8;
};

struct BDesc {
  int32_t n1, n2;
  int64_t N;
  int32_t ell, ell_pad;      // ell = 0: no preconditioner
  int64_t ldu;               // column pitch of U (elements)
  const float* omega;        // ell x N test images
  const float* v0;           // N power-method start
  const float* y;            // N measurements
  float* Y;                  // ell x N sketch
  float* U;                  // ldu x ell_pad, padding columns zero
  double* meta;              // factorisation metadata (PcMeta layout)
  double* G;                 // (2 ell)^2 Gram
  double* gpart;             // Gram partials (FP64)
  double* fwork;             // factor scratch (5 ell^2 + ell)
  float* f[kNumFields];      // image fields
  double* part;              // per-block reduction partials
  double* fpart;             // per-tile partials of the fused inner iteration
  double* cd;                // ell coefficients d . U^T v
  double* cq;                // d . U^T L^T Q of the last prox's final dual (the next prox's warm start)
  double* scal;              // BScal::kTotal scalars
  double* costs;             // optional cost per outer iteration
  float* x_out;              // caller's output image
  double lambda;
};

struct BSeg {
  int64_t first;    // first block of this segment in the launch
  int64_t nblk;     // blocks of the segment
  int64_t chunk;    // pixels per block
  int32_t inst;     // instance index into the descriptor table
  int32_t pad;
};

__device__ __forceinline__ int seg_find(const BSeg* __restrict__ seg, int nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace nys

namespace nys {

// One batched launch: its segment table (device), segments and total blocks.
struct BLaunch {
  const BSeg* seg = nullptr;
  int nseg = 0;
  int64_t nblk = 0;
};

// Batched Alg. 1 after the sketch: Gram Z^T Z (FP32 columns, FP64
// accumulation; gram: blocks of pixel chunks), one FP64 factor workgroup per
// instance, then U.
nys_status batch_factor_prepare(int64_t lds_bytes);
nys_status batch_factor_enqueue(const BDesc* d, const BLaunch& gram, const BLaunch& fac,
                                const BLaunch& upix, int kgroups, int max_ell, int64_t lds_doubles,
                                int nu_mode, int tail, double mu, int max_esc, hipStream_t st);
// D.cd = d . U^T f[fsrc] per instance (rseg: blocks of 1024 threads).
nys_status batch_pinv_coeffs(const BDesc* d, const BSeg* rseg, int nrseg, int64_t rblk, int fsrc,
                             hipStream_t st);
// f[fout] = f[fs] + c (f[ft] + U cd) per instance (pseg: 1024-pixel blocks).
nys_status batch_combine(const BDesc* d, const BSeg* pseg, int npseg, int64_t pblk, int fs,
                         int ft, int fout, int sidx, hipStream_t st);

}  // namespace nys
