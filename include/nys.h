/*
 * nys.h - C ABI of the MI355X (gfx950) implementation of randomized-Nystrom
 * preconditioned variational image reconstruction (Hong, Xu, Hu, Fessler,
 * "On adapting randomized Nystrom preconditioners to accelerate variational
 * image reconstruction").
 *
 * Conventions shared by every entry point
 * - Array pointers are DEVICE pointers unless a comment says "host".  They are
 *   owned by the caller; the library never frees or keeps them past the call
 *   (handles copy what they need).
 * - Workspaces: every call that needs device scratch takes `ws` / `ws_bytes`,
 *   a caller-owned device buffer (256-byte aligned) of at least the size its
 *   *_workspace_size query returns for the same arguments.  The library
 *   allocates device memory only when a handle is created (nys_op_create,
 *   nys_factor, batch_solve_create; irm_solve with a sketch creates one
 *   preconditioner handle per call) and frees it in the handle's destroy
 *   call.  A workspace may be reused once the work enqueued with it has run;
 *   two calls whose work may overlap need two workspaces.  Too small a
 *   workspace is EINVAL, returned before anything is enqueued.
 * - Images are row-major n1 x n2; a stack of `ncols` images is contiguous
 *   ([col][n1][n2]).  The tall N x K matrices of the paper (Omega, Y, U) are
 *   stored column by column, i.e. as K images.  Sinograms are [view][bin].
 * - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *   enqueue work and return; argument errors are returned synchronously before
 *   anything is enqueued.  Numerical failures are recorded in device status
 *   words (the preconditioner's, read by nys_pc_info; the solve's, the first
 *   int32 of its workspace) and returned by the calls that synchronise.
 * - Storage types: NYS_F64, NYS_F32, NYS_BF16 (bfloat16, FP32 accumulation).
 * - Handles are not safe for concurrent use from several streams.
 * - On any non-OK status, nys_last_error() returns a message (thread-local).
 */
#ifndef NYS_H_
#define NYS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NYS_OK = 0,
  NYS_EINVAL = 1,      /* bad argument, shape or dtype */
  NYS_ENOMEM = 2,      /* device allocation failed */
  NYS_ENOTPD = 3,      /* Cholesky failed after every shift escalation */
  NYS_ENOTFINITE = 4,  /* NaN/Inf met on the device */
  NYS_ENOCONV = 5,     /* semismooth Newton hit its iteration cap */
  NYS_EHIP = 6         /* a HIP runtime call failed */
} nys_status;

typedef enum { NYS_F64 = 0, NYS_F32 = 1, NYS_BF16 = 2 } nys_dtype;

typedef enum {
  NYS_OP_BLUR = 0,           /* periodic k x k blur, n1 x n2 -> n1 x n2 */
  NYS_OP_BLURDOWN = 1,       /* blur then keep every factor-th row/column */
  NYS_OP_PARALLEL_BEAM = 2,  /* Joseph projector, n x n -> views x bins */
  NYS_OP_IDENTITY = 3,       /* A = I (with wavelet_levels: A = W^T) */
  NYS_OP_FAN_BEAM = 4        /* Joseph projector, fan beam, flat detector, n x n -> views x bins */
} nys_op_kind;

typedef enum {
  NYS_REG_TV = 0,        /* isotropic TV, l_{1,2} of first differences */
  NYS_REG_TV_ANISO = 1,  /* anisotropic TV, l_{1,1} */
  NYS_REG_HS1 = 2,       /* Hessian Schatten-1 (sum of |eigenvalues| of each 2x2 Hessian) */
  NYS_REG_L1 = 3,        /* l1 of the unknown itself (wavelet coefficients) */
  NYS_REG_HS2 = 4,       /* Hessian Schatten-2 (Frobenius norm of each 2x2 Hessian) */
  NYS_REG_HSINF = 5      /* Hessian Schatten-inf (spectral norm of each 2x2 Hessian) */
} nys_reg_kind;

typedef enum { NYS_LOSS_LS = 0, NYS_LOSS_HUBER = 1 } nys_loss_kind;

/* ---------------------------------------------------------------------------
 * Operators A (problem statement eq. (4); the method touches A only through
 * A x and A^T y).  Geometry:
 *  BLUR / BLURDOWN: (H x)[i,j] = sum_{a,b} psf[a,b] x[(i+c-a) mod n1,
 *    (j+c-b) mod n2], c = (k-1)/2; BLURDOWN keeps samples (f i, f j).
 *  PARALLEL_BEAM: n1 = n2 = n unit pixels centred at the origin, pixel (i,j)
 *    at (j-c, i-c); bin b at s = b-(B-1)/2; view v at theta = v*pi/V; each
 *    ray is sampled once per row (|cos| >= |sin|) or per column with linear
 *    interpolation and weight 1/max(|cos|,|sin|) (ray-driven, Joseph).  The
 *    adjoint is the exact transpose, computed in gather form.
 *  wavelet_levels > 0 composes A with a wavelet synthesis: the unknown is
 *    the coefficient array xbar, x = W^T xbar (invertible-L reparametrisation,
 *    Sec. III-B).  wavelet = NYS_WAVELET_HAAR: orthonormal Haar, 1..3 levels,
 *    in-place layout (each level writes LL, HL / LH, HH at the positions of
 *    its 2 x 2 group).  wavelet = NYS_WAVELET_DB4: the periodised orthonormal
 *    Daubechies wavelet with four vanishing moments (8 taps, the "daub4" of
 *    the CT experiments), 1..6 levels, quadrant layout (level j transforms the
 *    top-left (n1 / 2^j) x (n2 / 2^j) band, rows then columns, into
 *    [LL | HL ; LH | HH]).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t kind;            /* nys_op_kind */
  int32_t n1, n2;          /* unknown image size */
  int32_t psf_size;        /* k, odd, <= 31 (blur kinds) */
  const double* psf;       /* host, k*k row-major; copied at create */
  int32_t factor;          /* decimation factor (BLURDOWN), >= 1 */
  int32_t n_views, n_bins; /* PARALLEL_BEAM */
  int32_t wavelet_levels;  /* 0 or wavelet levels; n1, n2 divisible by 2^levels */
  int32_t wavelet;         /* NYS_WAVELET_HAAR (0) or NYS_WAVELET_DB4 (1) */
  /* FAN_BEAM, in pixel units: view v at theta = 2 pi v / views; source at
   * fan_src from the centre opposite the central ray direction (-sin, cos);
   * a flat detector at fan_det past the centre, perpendicular to it; bin b at
   * u = (b - (bins - 1) / 2) fan_du along (cos, sin).  Every ray, a line
   * n . p = s, is sampled as in PARALLEL_BEAM with its own normal n and
   * offset s; the adjoint is the exact transpose, gathered per pixel (no
   * atomics) when the source lies outside the image's circumscribed circle,
   * else scattered with atomic additions (summation order not fixed). */
  double fan_src, fan_det, fan_du;
} nys_op_desc;

enum { NYS_WAVELET_HAAR = 0, NYS_WAVELET_DB4 = 1 };

typedef struct nys_op_s* nys_op;
typedef struct nys_pc_s* nys_pc;

/* Create/destroy an operator handle.  EINVAL on inconsistent sizes. */
nys_status nys_op_create(const nys_op_desc* desc, nys_op* out);
void nys_op_destroy(nys_op op);
/* Number of unknowns N and of measurements M of one column (host out). */
nys_status nys_op_shape(nys_op op, int64_t* n_unknowns, int64_t* n_meas);

/* Workspace bytes of op_forward / op_adjoint on `ncols` columns of dtype dt
 * (host out; 0 when the operator needs none). */
nys_status nys_op_workspace_size(nys_op op, nys_dtype dt, int64_t ncols, size_t* bytes);
/* y = A x for `ncols` stacked columns; x: ncols*N, y: ncols*M, dtype F64 or
 * F32.  x and y must not overlap. */
nys_status op_forward(nys_op op, nys_dtype dt, const void* x, void* y,
                      int64_t ncols, void* ws, size_t ws_bytes, void* stream);
/* x = A^T y for `ncols` stacked columns. */
nys_status op_adjoint(nys_op op, nys_dtype dt, const void* y, void* x,
                      int64_t ncols, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Sketch, Alg. 1 step 2 (and Sec. III-C, on-the-fly batched evaluation):
 * Y = Phi Omega with Phi = A^T A (with the wavelet composition,
 * Phi = W A^T A W^T), all `ell` columns in one batched launch sequence.
 * omega, Y: ell*N in dtype `dt`; BF16 keeps FP32 accumulation inside.
 * ------------------------------------------------------------------------- */
nys_status nys_sketch_workspace_size(nys_op op, nys_dtype dt, int64_t ell, size_t* bytes);
nys_status nys_sketch(nys_op op, nys_dtype dt, const void* omega, void* Y,
                      int64_t ell, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Nystrom factorisation, Alg. 1 steps 3-8, and the preconditioner of eq. (11):
 *   nu; Y_nu = Y + nu Omega; C = chol(Omega^T Y_nu) (lower, symmetrised);
 *   B = Y_nu C^{-T}; [U, S] = svd(B); shat = max(0, S^2 - nu).
 * B is not formed: the ell x ell FP64 matrix C^{-1} Y_nu^T Y_nu C^{-T} is
 * diagonalised (Jacobi) and U = Y_nu C^{-T} V S^{-1} is written in one pass.
 * Columns with shat = 0 are kept in U but left unscaled by P (equivalent to
 * dropping them).  If Cholesky fails, nu is multiplied by 10 and the steps are
 * repeated up to max_escalations times; then the status word is ENOTPD.
 * P^{-1} = (s_K + mu) U (S + mu I)^{-1} U^T + (I - U U^T), where s_K is the
 * smallest retained shat, or its square root with tail = 0 (the paper's
 * heuristic, Sec. III-B).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t nu_mode;         /* 0: sqrt(N) eps ||Y||_2 ; 1: eps ||Omega||_F */
  int32_t tail;            /* 0: s_K <- sqrt(s_K) (paper) ; 1: s_K */
  double mu;               /* < 0: mu = nu */
  int32_t max_escalations; /* < 0: 6 */
  int32_t u_dtype;         /* storage of U: NYS_F64 or NYS_F32 */
} nys_factor_opts;

/* omega, Y: ell*N in dtype in_dt (F64, F32 or BF16).  ell <= 128.
 * The handle owns U (ell*N in u_dtype), the FP64 spectrum and the semismooth
 * Newton buffers, allocated here; the factorisation's scratch (Gram partials,
 * the 2 ell x 2 ell Gram, the ell x ell FP64 matrices) is the workspace. */
nys_status nys_factor_workspace_size(int64_t N, int64_t ell, size_t* bytes);
nys_status nys_factor(const void* omega, const void* Y, nys_dtype in_dt,
                      int64_t N, int64_t ell, const nys_factor_opts* opts,
                      void* ws, size_t ws_bytes, nys_pc* out, void* stream);
void nys_pc_destroy(nys_pc pc);

/* Synchronises `stream` and copies to host: shat (ell values, descending,
 * 0 for dropped columns), nu used, number of retained columns, status word
 * (nys_status of the device-side factorisation).  Any pointer may be NULL. */
nys_status nys_pc_info(nys_pc pc, double* shat, double* nu, int32_t* k_eff,
                       int32_t* status, void* stream);
/* Diagnostics of the factorisation (host out, synchronises `stream`): up to
 * n (<= 16) doubles: [0] nu used, [1] s_K value used in P, [2] mu,
 * [3] ||P^{-1}||_2, [4] retained columns, [5] status word, [6] shift
 * escalations, [7] Jacobi sweeps of the shift estimate, [8] Jacobi sweeps of
 * the ell x ell eigenproblem, [9..15] device timestamps of the factor kernel's
 * phases (100 MHz wall clock). */
nys_status nys_pc_diag(nys_pc pc, double* out, int32_t n, void* stream);

/* Device pointer to U and its sizes: column k of U starts at element k * ldu
 * (ldu >= N; the library pads the pitch), dtype u_dtype. */
nys_status nys_pc_u(nys_pc pc, const void** u, int64_t* N, int64_t* ell, int64_t* ldu,
                    int32_t* u_dtype);

/* Copies U into the caller's device buffer `dst`, packed as ell*N (u_dtype). */
nys_status nys_pc_copy_u(nys_pc pc, void* dst, void* stream);

/* out = P^{-1} v (inverse != 0) or P v (eq. (11)), for `ncols` stacked
 * vectors of length N, dtype = the pc's u_dtype.  out may equal v.  The
 * workspace holds the coefficients and the block partials of U^T v. */
nys_status nys_apply_workspace_size(nys_pc pc, int64_t ncols, size_t* bytes);
nys_status nys_apply(nys_pc pc, int32_t inverse, nys_dtype dt, const void* v,
                     void* out, int64_t ncols, void* ws, size_t ws_bytes, void* stream);

/* nys_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and results, with the coefficients and the block partials of
 * U^T v in a file-scope device array of 2 MiB per GPU (held by each GPU the
 * library runs on until the process ends) instead of a workspace.  ncols <= 8
 * (EINVAL beyond); no allocation of any kind.  Every call on one GPU shares
 * that GPU's array: calls whose work may overlap (several streams or host
 * threads) race. */
nys_status nys_apply_static(nys_pc pc, int32_t inverse, nys_dtype dt, const void* v,
                            void* out, int64_t ncols, void* stream);

/* Squared P-norm of a difference, the metric of the WAPG rate bound
 * 2 L_f^P ||x^1 - x^*||_P^2 / (k + 1)^2 stated after eq. (20) (Sec. III-B):
 * *out (one device double, written on `stream`) = (a - b)^T P (a - b), or
 * (a - b)^T P^{-1} (a - b) when inverse != 0; pc = NULL gives P = I.  a, b:
 * n device values (n = the pc's N, dtype = its u_dtype; F64 or F32 without
 * a pc); b may be NULL (b = 0).  With a pc the difference and P (a - b) are
 * rounded to dt; the dot product accumulates in FP64 block partials summed
 * in a fixed order. */
nys_status nys_pnorm2_workspace_size(nys_pc pc, int64_t n, nys_dtype dt, size_t* bytes);
nys_status nys_pnorm2(nys_pc pc, int64_t n, int32_t inverse, nys_dtype dt, const void* a,
                      const void* b, double* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Weighted proximal map (eq. (5), Sec. I-D):
 *   x = argmin_u  lambda_bar g(u) + 1/2 ||u - s||_P^2,   C = R^N,
 * P = I when pc is NULL.
 *  TV / TV_ANISO / HS1 / HS2 / HSINF: dual accelerated projected gradient on
 *   Q for n_inner iterations (eqs. (21)-(29)); x(Q) = s - lambda_bar P^{-1}
 *   L^T Q; the step is 1 / (lambda_bar ||L||^2 ||P^{-1}||).  The dual ball of
 *   eq. (23) is per group: the unit l2 ball (TV), [-1, 1] (TV_ANISO), and for
 *   the Hessian groups the unit Schatten-inf, -2, -1 ball (HS1, HS2, HSINF).
 *   `state` holds Q (2*N values for TV, 3*N for the Hessian kinds, dtype dt)
 *   and is used as the warm start and updated.
 *  L1: Thm. 1 with P = I + U diag(e) U^T: gamma solves
 *   gamma = diag(e) U^T (soft(s - U gamma) - s), semismooth Newton with
 *   backtracking on ||F||; x = soft(s - U gamma).  `state` holds gamma
 *   (ell FP64 values) as warm start.  P = I gives x = soft(s).  The call
 *   waits for the device's Newton decisions and returns NYS_ENOTFINITE when
 *   ||F|| is not finite (the warm start is then left as it was) and
 *   NYS_ENOCONV when max_newton trial points end without convergence (x and
 *   the warm start then hold the last accepted point).
 * state may be NULL (cold start, not kept).  x may be s (in place); no other
 * overlap of s and x is allowed.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t kind;        /* nys_reg_kind */
  int32_t n1, n2;
  double lnorm2;       /* ||L||^2 bound for the dual step; <= 0: 8 (TV), 34 (Hessian kinds) */
  int32_t n_inner;     /* dual iterations (TV and Hessian kinds) */
  int32_t max_newton;  /* SSN trial points (L1); <= 0: 60 */
  double newton_tol;   /* ||F|| <= tol (1 + ||gamma||); <= 0: 1e-12 / 1e-6 */
  int32_t box;         /* != 0: x restricted to C = {lo <= x_i <= hi} (TV and
                          Hessian kinds only): x(Q) = prox^P_{delta_C}(s -
                          lambda_bar P^{-1} L^T Q) in every dual iteration
                          (eqs. (26), (29)), the P-weighted projection by Thm. 1
                          with the clip in place of the soft threshold (the
                          clip itself when P = I); 0: C = R^N */
  double lo, hi;       /* the box (lo <= hi; hi may be +inf) */
} nys_reg_desc;

nys_status nys_prox_workspace_size(const nys_reg_desc* reg, nys_pc pc, nys_dtype dt,
                                   size_t* bytes);
nys_status prox_weighted(const nys_reg_desc* reg, double lambda_bar, nys_pc pc,
                         nys_dtype dt, const void* s, void* x, void* state,
                         void* ws, size_t ws_bytes, void* stream);
/* Bytes of `state` for prox_weighted (host out). */
nys_status nys_prox_state_bytes(const nys_reg_desc* reg, nys_pc pc,
                                nys_dtype dt, size_t* bytes);

/* ---------------------------------------------------------------------------
 * Solve min_x f(x) + lambda g(x) with WAPG (Alg. 3): x^1 = u^1 = 0, t^0 = 1,
 *   x^{k+1} = prox^P_{alpha lambda g}(u^k - alpha P^{-1} grad f(u^k)),
 *   t^k = (1 + sqrt(1 + 4 (t^{k-1})^2)) / 2,
 *   u^{k+1} = x^{k+1} + ((t^{k-1} - 1) / t^k) (x^{k+1} - x^k).
 * f = 1/2 ||A x - y||^2 or sum h_delta(A x - y) (Huber: r^2/(2 delta) for
 * |r| <= delta, |r| - delta/2 otherwise).  pc = NULL gives plain APG.
 * alpha <= 0 selects alpha = 1 / (safety * L), L = lambda_max(P^{-1} A^T A) *
 * curvature by `power_iters` power-method steps from `power_v0` (N values).
 * ------------------------------------------------------------------------- */
typedef struct {
  nys_op op;
  int32_t loss;        /* nys_loss_kind */
  double delta;        /* Huber parameter */
  nys_reg_desc reg;
  double lambda;
  const void* y;       /* M measurements, solver dtype */
} nys_problem;

typedef struct {
  int32_t max_iter;        /* outer iterations */
  double alpha;            /* step; <= 0: from the power method */
  double safety;           /* alpha = 1 / (safety L); <= 0: 1.01 */
  int32_t power_iters;     /* power-method steps (alpha <= 0) */
  const void* power_v0;    /* N start values, solver dtype (alpha <= 0) */
  int32_t warm_start;      /* keep Q / gamma across outer iterations */
} nys_solve_opts;

/* x_out: N values (solver dtype dt = F64 or F32).  costs: device, max_iter
 * FP64 values F(x^{k+1}) or NULL.  info (host, 8 doubles, may be NULL):
 * [0] alpha used, [1] L estimate, [2] status, [3] reserved.
 * The first int32 of the workspace is the solve's device status word: 0, or
 * NYS_ENOTFINITE when x_out holds a NaN or infinity at the end (set by the
 * last kernel of the call).  With info != NULL the stream is synchronised and
 * the call returns that status (NYS_ENOTFINITE) or NYS_ENOCONV when an l1
 * prox ran out of Newton trial points (the iteration goes on from its last
 * accepted point); without info it returns NYS_ENOCONV in that case and the
 * word is left for the caller to read.  A power method that meets non-finite
 * values returns NYS_ENOTFINITE before the iteration starts. */
nys_status nys_workspace_size(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                              size_t* bytes);
nys_status solve(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                 const nys_solve_opts* opts, void* x_out, double* costs,
                 double* info, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * The same fixed-count solve (Alg. 3, opts->max_iter iterations) captured
 * once as HIP graphs and replayed with no host work inside the loop: the
 * start, a chunk of 16 iterations launched max_iter / 16 times, the remaining
 * iterations and the final finite check, all enqueued by nys_solve_plan_run
 * on the caller's stream.  Each iteration finds its momentum weight and cost
 * slot through a device counter; the results are those of solve with the
 * same arguments (the same kernels and step) for the TV / Hessian priors and
 * for every prior without a preconditioner.  The P-weighted l1 prox (Thm. 1,
 * FP32 with ell <= 64) runs a fixed sequence of semismooth Newton trials
 * whose kernels skip themselves once the device state has converged: the
 * first two trials of solve, then 2 rounds of a Newton step and a trial; a
 * call that has not converged by then goes on from its last accepted point
 * and sets the second int32 of ws to NYS_ENOCONV (solve allows max_newton
 * trials instead).  The P-weighted box projection decides on the host and is
 * EINVAL here.
 * create: alpha <= 0 runs the power method on `stream` and synchronises; the
 * plan keeps prob->y, x_out, costs (device, max_iter values, or NULL), ws
 * (nys_workspace_size bytes) and pc by address: they must stay allocated and
 * unmoved while the plan lives.  info (host, 8 doubles, may be NULL): [0]
 * alpha, [1] L estimate.  The first int32 of ws is the status word of each
 * run (NYS_ENOTFINITE when x_out holds a NaN or infinity at its end, or a
 * Newton trial met one), the second NYS_ENOCONV as above.  With the l1 prior
 * and a preconditioner whose Newton factors are not stored yet, create runs
 * one iteration on `stream` first and synchronises.
 * destroy: only once the runs have completed (synchronise their streams).
 * Allocates the plan, its graphs and max_iter + 1 doubles of device memory.
 * ------------------------------------------------------------------------- */
typedef struct nys_solve_plan_s* nys_solve_plan;
nys_status nys_solve_plan_create(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                 const nys_solve_opts* opts, void* x_out, double* costs,
                                 void* ws, size_t ws_bytes, void* stream, double* info,
                                 nys_solve_plan* out);
nys_status nys_solve_plan_run(nys_solve_plan plan, void* stream);
void nys_solve_plan_destroy(nys_solve_plan plan);

/* ---------------------------------------------------------------------------
 * Unrolled, differentiable WAPG (Alg. 3) with the P-weighted TV prox (dual
 * FISTA of eqs. (21)-(29), warm-started across outer iterations): a fixed
 * number n_outer of outer and n_inner of inner iterations, a fixed step
 * alpha, u^1 = x^1 = 0, Q = 0.  The forward keeps u_k and the dual Q_k of
 * every outer iteration in the workspace; the backward recomputes one outer
 * iteration at a time from them and returns the exact vector-Jacobian
 * products with respect to the measurements y and the weight lambda (the
 * projection onto the dual ball is differentiated where it is smooth).
 * Operator, preconditioner (U, Lambda depend on A only) and alpha are
 * constants of the map.  Least-squares data term; reg TV or TV_ANISO.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_outer;   /* unrolled outer iterations K */
  int32_t n_inner;   /* dual iterations per outer iteration */
  double alpha;      /* step, > 0 */
} nys_unroll_opts;

/* Bytes of device workspace for `batch` instances (host out). */
nys_status nys_unrolled_workspace(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                                  const nys_unroll_opts* opts, int32_t batch, size_t* bytes);

/* x[b] (N values) = K unrolled iterations on y[b] (M values) with weight
 * lambda[b] (host array), b < batch; prob->y and prob->lambda are ignored.
 * ws: device workspace of ws_bytes >= nys_unrolled_workspace(...), kept for
 * the backward. */
nys_status unrolled_forward(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                            const nys_unroll_opts* opts, int32_t batch, const void* y,
                            const double* lambda, void* x, void* ws, size_t ws_bytes,
                            void* stream);

/* Given bar_x = dLoss/dx (batch x N), writes bar_y = dLoss/dy (batch x M,
 * device) and bar_lambda (host, batch doubles; the stream is synchronised).
 * Same arguments and workspace as the forward call. */
nys_status unrolled_backward(const nys_problem* prob, nys_pc pc, nys_dtype dt,
                             const nys_unroll_opts* opts, int32_t batch, const void* y,
                             const double* lambda, const void* bar_x, void* bar_y,
                             double* bar_lambda, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched reconstruction: many periodic-blur problems of different sizes
 * solved together, every step of every instance in shared launches that are
 * captured once into a HIP graph.  Instance i solves eq. (4) with
 * f = 1/2 ||h_i * x - y_i||^2 and lambda_i g(x), g = TV, anisotropic TV or
 * a Hessian Schatten prior HS1 / HS2 / HSINF (one kind for the batch), by
 * WAPG (Alg. 3) from x = u = 0 with the
 * P-weighted prox of the dual iterations (eqs. (21)-(29)).  With
 * precondition = 1, P is the Nystrom preconditioner of eq. (11) built from the
 * sketch Y = A^T A Omega (Alg. 1, step 2) and the shifted factorisation
 * (Alg. 1, steps 3-7); with precondition = 0, P = I (plain APG).  The step is
 * 1 / (safety L) with L from power_iters power-method steps on P^{-1} A^T A
 * (the constant of eq. (20)).  Images, sketches and iterates are FP32, the
 * factorisation and all reductions FP64.
 *
 * batch_solve_create checks the items, allocates every buffer of the batch,
 * times the stencil tile heights (tune = 1; the table is kept per process),
 * and captures the pipeline into a graph; it synchronises `stream`.  The graph
 * keeps the item pointers: y, omega, v0, x and costs must stay valid and may
 * be refilled between runs.  batch_solve_run enqueues one graph launch on
 * `stream`; runs of one plan must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct nys_batch_s* nys_batch;

typedef struct {
  int32_t n1, n2;         /* image rows and columns; n1 * n2 a multiple of 4 */
  int32_t psf_k;          /* PSF size, odd, 1..31 */
  const double* psf;      /* host, psf_k x psf_k row-major, centre (k-1)/2,
                             separable (rank 1, e.g. Gaussian); copied */
  int32_t ell;            /* sketch size 1..64 (ignored when precondition = 0) */
  double lambda;          /* regularisation weight, >= 0 */
  const float* y;         /* n1 x n2 measurements */
  const float* omega;     /* ell x n1 x n2 test images, 16-byte aligned */
  const float* v0;        /* n1 x n2 power-method start (not all zero) */
  float* x;               /* n1 x n2 reconstruction (written by each run) */
  double* costs;          /* max_iter FP64 costs F(x_k), or NULL */
} nys_batch_item;

typedef struct {
  int32_t reg;            /* NYS_REG_TV, NYS_REG_TV_ANISO, NYS_REG_HS1, _HS2 or _HSINF */
  int32_t max_iter;       /* outer WAPG iterations */
  int32_t n_inner;        /* dual iterations per prox */
  int32_t power_iters;    /* >= 1 */
  int32_t precondition;   /* 1: Nystrom P; 0: P = I */
  int32_t warm_start;     /* 1: dual variable kept across outer iterations */
  int32_t nu_mode, tail;  /* shift and tail rules as in nys_factor_opts */
  double mu;              /* < 0: mu = nu */
  double safety;          /* <= 0: 1.01 */
  int32_t tune;           /* 1: run the tile autotuner */
} nys_batch_opts;

nys_status batch_solve_create(const nys_batch_item* items, int32_t count,
                              const nys_batch_opts* opts, nys_batch* out, void* stream);
nys_status batch_solve_run(nys_batch b, void* stream);
/* Enqueues only the sketches Y_i = A_i^T A_i Omega_i of every instance (the
 * first step of a run) on `stream`; the plan must have a preconditioner.  It
 * shares the plan's work-queue counters with batch_solve_run: the two must
 * not overlap. */
nys_status batch_solve_sketch(nys_batch b, void* stream);
/* Host out[6] for instance i after a run (synchronises `stream`): alpha, L,
 * ||P^{-1}||, nu, factorisation status (nys_status), k_eff. */
nys_status batch_solve_info(nys_batch b, int32_t i, double* out, void* stream);
/* Host shat[ell_i]: the Nystrom eigenvalue estimates of instance i. */
nys_status batch_solve_shat(nys_batch b, int32_t i, double* shat, void* stream);
/* Device views of instance i's sketch Y (ell x N) and U (ell columns of
 * pitch *ldu); NULL without a preconditioner.  Owned by the plan. */
nys_status batch_solve_buffers(nys_batch b, int32_t i, const float** Y, const float** U,
                               int64_t* ldu);
/* Copies instance i's sketch Y (what = 0) or U (what = 1), ell x N compact,
 * into dst (device, ell * N floats) on `stream`. */
nys_status batch_solve_copy(nys_batch b, int32_t i, int32_t what, float* dst, void* stream);
/* Tile table of the plan's stencil classes: row taps, column taps, tile rows
 * (host arrays of `cap` entries, NULL allowed); *count = number of classes. */
nys_status batch_solve_tiles(nys_batch b, int32_t* nt_r, int32_t* nt_c, int32_t* ty,
                             int32_t cap, int32_t* count);
void batch_solve_destroy(nys_batch b);

/* ---------------------------------------------------------------------------
 * l_p - l_q reconstruction by the alternating minimisation method (Alg. 2):
 *   min_x 1/p sum_m |(A x - y)_m|^p + lambda/q sum_l |(L x)_l|^q
 * with L the first differences of the TV regulariser (each component its own
 * group; prob->reg is not used) and |r| smoothed to sqrt(r^2 + eps).  Outer
 * iteration k sets W_f = |A x - y|^{p-2}, W_g = |L x|^{q-2} (element-wise) at
 * the previous iterate and solves Phi_k x = A^T W_f y,
 * Phi_k = A^T W_f A + lambda L^T W_g L, by conjugate gradients from the
 * previous iterate until ||b - Phi_k x|| <= cg_tol ||b|| or max_cg steps.  With
 * ell > 0 the CG is preconditioned by the Nystrom P of eq. (11), rebuilt at
 * every outer iteration from Y = Phi_k Omega (Alg. 1).  Stops after
 * max_outer iterations or when ||x_k - x_{k-1}|| <= outer_tol ||x_k||.
 * Synchronises `stream` (CG scalars are read back every step).
 * ------------------------------------------------------------------------- */
typedef struct {
  double p, q;          /* exponents of the data and regulariser terms, in (0, 2] */
  double eps;           /* smoothing, > 0 */
  int32_t max_outer;    /* outer (IRM) iterations */
  double outer_tol;     /* relative change that stops the outer loop (0: never) */
  int32_t max_cg;       /* CG steps per outer iteration */
  double cg_tol;        /* relative residual of the x-update */
  int32_t nu_mode;      /* as nys_factor_opts */
  int32_t tail;         /* as nys_factor_opts; 1 = s_K as printed in eq. (11) */
  double mu;            /* < 0: mu = nu */
} nys_irm_opts;

/* x (N values, dtype dt = F64 or F32) from x0 (N values, or NULL for 0);
 * omega: ell x N test images (dtype dt) or NULL with ell = 0 (plain CG).
 * cg_iters (host, max_outer entries, may be NULL) receives the CG steps of
 * every outer iteration and *outer_done (host, may be NULL) their count;
 * info (host, 3 * max_outer doubles, may be NULL) receives per outer
 * iteration the factorisation status (nys_status), k_eff and the shift nu. */
nys_status irm_workspace_size(const nys_problem* prob, nys_dtype dt, int64_t ell,
                              size_t* bytes);
nys_status irm_solve(const nys_problem* prob, nys_dtype dt, const nys_irm_opts* opts,
                     const void* omega, int64_t ell, const void* x0, void* x,
                     int32_t* cg_iters, int32_t* outer_done, double* info, void* ws,
                     size_t ws_bytes, void* stream);

/* F(x) = f(x) + lambda g(x) for one column, FP64 accumulation, written to the
 * device double `cost`. */
nys_status nys_cost_workspace_size(const nys_problem* prob, nys_dtype dt, size_t* bytes);
nys_status nys_cost(const nys_problem* prob, nys_dtype dt, const void* x,
                    double* cost, void* ws, size_t ws_bytes, void* stream);

/* Message of the last non-OK status on this thread. */
const char* nys_last_error(void);
/* Library version string. */
const char* nys_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NYS_H_ */
