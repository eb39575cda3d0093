// Cross-file internal entry points of libnys (not part of the public ABI).
#pragma once

#include "common.hpp"

namespace nys {

// Workspace bytes of op_fwd / op_adj on ncols columns of es-byte values, and
// of the sketch on ell columns stored in dt (ops.hip).
size_t op_ws_bytes(nys_op op, size_t es, int64_t ncols);
size_t sketch_ws_bytes(nys_op op, nys_dtype dt, int64_t ell);

// y = A x / x = A^T y with the optional wavelet composition (ops.hip).  The
// scratch comes from the workspace bound to op (op->scr).
template <class T> nys_status op_fwd(nys_op op, const T* x, T* y, int64_t ncols, hipStream_t st);
template <class T> nys_status op_adj(nys_op op, const T* y, T* x, int64_t ncols, hipStream_t st);
// out = psi(A x - yobs) in one kernel (psi of the loss: identity for least
// squares, clip((.) / delta, -1, 1) for Huber; yobs null: out = A x), for the
// operators where op_fwd_fused_ok holds: blur and blur-decimation with the Haar
// synthesis of 0..3 levels.
template <class T> bool op_fwd_fused_ok(nys_op op);
template <class T>
nys_status op_fwd_psi(nys_op op, const T* x, const T* yobs, int loss, double delta, T* out,
                      int64_t ncols, hipStream_t st);

// Fused W H^T S^T S H W^T sketch for factor-2 decimation with 3 Haar levels
// (sketch_sr.hip).  S is float or uint16_t (bfloat16).
template <class S>
nys_status sketch_sr_fused(nys_op op, const S* omega, S* Y, int64_t ell, hipStream_t st);
nys_status sketch_sr_chain_bf16(nys_op op, const uint16_t* omega, uint16_t* Y, int64_t ell,
                                hipStream_t st);
nys_status sketch_sr_chain_f32(nys_op op, const float* omega, float* Y, int64_t ell,
                               hipStream_t st);

// Preconditioner application on T-typed vectors (pinv.hip); the scratch
// comes from the workspace bound to pc (pc->scr), pc_ws_bytes(pc, ncols) of
// it for pc_apply.
// out = v + U (coef . (U^T v)) with coef = d (P^{-1}) or e (P).
size_t pc_ws_bytes(nys_pc pc, int64_t ncols);
template <class T>
nys_status pc_apply(nys_pc pc, bool inverse, const T* v, T* out, int64_t ncols, hipStream_t st);
// cd[col][k] = coef_k (U^T v_col)_k in FP64 (coef = d or e).
template <class T>
nys_status pc_coeffs(nys_pc pc, bool inverse, const T* v, int64_t ncols, double* cd,
                     hipStream_t st);
// The same with the rows of U replaced by those of B (ell_pad rows of len
// values, pitch ldb; v: ncols columns of len).  With B = A U (the operator
// applied to U's rows) and v = psi, B^T psi = U^T (A^T psi): the coefficients
// of P^{-1} A^T psi from a pass over the measurements instead of the image.
template <class T>
nys_status pc_coeffs_on(nys_pc pc, const T* B, int64_t ldb, int64_t len, bool inverse, const T* v,
                        int64_t ncols, double* cd, hipStream_t st);
// Its two stages: block partials of B^T v (FP64, nblk x ell_pad per column,
// taken from the bound workspace and left there for the caller), then their
// sums times the coefficients.
struct CoefPartials {
  const double* part = nullptr;
  int nblk = 0, ncols = 0;
};
template <class T>
nys_status pc_partials_on(nys_pc pc, const T* B, int64_t ldb, int64_t len, const T* v,
                          int64_t ncols, CoefPartials* out, hipStream_t st);
nys_status pc_tail(nys_pc pc, bool inverse, const CoefPartials& cp, double* cd, hipStream_t st);

// s = u - alpha P^{-1} g for one column, one pass over U after the
// coefficients (pinv.hip).
template <class T>
nys_status pc_step(nys_pc pc, const T* u, const T* g, double alpha, T* s, hipStream_t st);

// x = s - lam (t + U cd) for one column (pinv.hip).
template <class T>
nys_status pc_x_from_pinv(nys_pc pc, const T* s, const T* t, const double* cd, double lam, T* x,
                          hipStream_t st);
// Prox centre given by the preconditioned gradient step s = u - alpha (g + U cd)
// (cd: FP64 coefficients d . U^T g from pc_coeffs).
struct SsnStep {
  const void* u;
  const void* g;
  double alpha;
  CoefPartials cp;   // partials of U^T g (one column)
  double* cd;        // ell FP64 of device workspace for cd where it is stored
};
// P-weighted l1 prox by semismooth Newton (Thm. 1, pinv.hip); gamma_state
// (ell FP64, may be null) is the warm start and receives the root.  With
// `step`, s is an output buffer: the step is formed into it (by the first
// evaluation pass where possible).
// With `box`, h is the indicator of C = {lo <= x <= hi} instead of
// lam_bar ||.||_1 (lam_bar unused): x = prox^P_{delta_C}(s), the P-weighted
// projection onto the box, by the same iteration with the clip in place of
// the soft threshold.
struct SsnBox {
  double lo, hi;
};
// A box constraint needs a TV or Hessian prior and lo <= hi (not NaN).
inline nys_status check_box(const nys_reg_desc& r) {
  if (!r.box) return NYS_OK;
  NYS_REQUIRE(r.kind != NYS_REG_L1, "box constraint: needs a TV or Hessian prior");
  NYS_REQUIRE(r.lo <= r.hi, "box constraint: lo must be <= hi");
  return NYS_OK;
}
// Bytes of the preconditioner's semismooth Newton buffer (state, partials,
// stored factors) for N pixels, L columns and es-byte values.
size_t ssn_ws_bytes(int64_t N, int L, size_t es);
template <class T>
nys_status ssn_prox(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                    double* gamma_state, hipStream_t st, int* trials_out = nullptr,
                    const SsnStep* step = nullptr, const SsnBox* box = nullptr);

// Layout of the FP64 metadata block of a preconditioner (pc->meta).
struct PcMeta {
  static constexpr int kMaxEll = 128;
  // offsets in doubles
  static constexpr int kShat = 0;              // ell
  static constexpr int kD = kMaxEll;           // ell: P^{-1} coefficients
  static constexpr int kE = 2 * kMaxEll;       // ell: P coefficients
  static constexpr int kScalars = 3 * kMaxEll; // nu, sK, mu, pinv_norm, k_eff, status
  static constexpr int kNu = kScalars + 0;
  static constexpr int kSK = kScalars + 1;
  static constexpr int kMu = kScalars + 2;
  static constexpr int kPinvNorm = kScalars + 3;
  static constexpr int kKeff = kScalars + 4;
  static constexpr int kStatus = kScalars + 5;
  static constexpr int kEscal = kScalars + 6;
  static constexpr int kSweeps0 = kScalars + 7;   // Jacobi sweeps: shift estimate
  static constexpr int kSweeps1 = kScalars + 8;   // Jacobi sweeps: B^T B
  static constexpr int kTotal = kScalars + 16;
};

// p[0:n] = 0 by a fill kernel on the stream (prox.hip).
template <class T> nys_status fill_zero(T* p, size_t n, hipStream_t st);

// Scratch bytes of Alg. 1 steps 3-8 for N pixels and L columns (factor.hip).
size_t factor_ws_bytes(int64_t N, int L);

// A preconditioner handle with its buffers (U zeroed on st), before any
// factorisation (factor.hip).
nys_status pc_create(int64_t N, int64_t ell, const nys_factor_opts& o, nys_pc* out,
                     hipStream_t st);

// Alg. 1 steps 3-8 on an existing handle of the same N, ell and dtype
// (factor.hip); its scratch comes from the workspace bound to pc.
nys_status factor_refresh(nys_pc pc, const void* omega, const void* Y, nys_dtype in_dt,
                          const nys_factor_opts& o, hipStream_t st);

// Weighted prox (prox.hip).  state as in prox_weighted; work: prox_ws_bytes
// of device memory (the dual iteration's buffers); a preconditioner's
// applications take their scratch from the workspace bound to pc.
// c_kept: the work buffer's leading coefficients already hold d . U^T L^T Q
// for the state's Q with this pc (the previous call on the same state and
// work left them there, or they were cleared with Q = 0); the fused path
// then starts from them instead of a pass over U.
template <class T>
nys_status prox_run(const nys_reg_desc& reg, double lam_bar, nys_pc pc, const T* s, T* x,
                    void* state, hipStream_t st, void* work, bool c_kept = false);
template <class T> size_t prox_ws_bytes(const nys_reg_desc& reg);

}  // namespace nys
