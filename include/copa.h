/*
 * copa.h - C ABI of libcopa.so: COPA, constrained PARAFAC2 fitted by AO-ADMM, on one AMD GPU
 * (gfx950 / MI355X).
 *
 * Model (Background, "Original PARAFAC2 model"; Section "General Framework", eq.
 * PARAFAC2_obj_func): each subject k has a sparse count matrix X_k (I_k visits x J features) and
 *     X_k ~= U_k S_k V^T,  U_k = Q_k H,  Q_k^T Q_k = I,  S_k = diag(W(k,:)),
 * fitted by Algorithm 1 (COPA): per outer iteration a Procrustes step gives Q_k (eq. solv_Q),
 * then one ADMM block per factor H, W, V (update rules after eq. Solve_W) with a proximity
 * operator per factor (Section "Examples of useful constraints"). With temporal smoothing
 * (Section "Smoothness on U_k") every subject's U_k lies in the span of a cubic spline basis
 * M_k evaluated at its visit days; the fit then runs on C_k^T X_k with C_k an orthonormal basis
 * of span(M_k), and U_k = C_k Q_k H.
 *
 * Conventions
 *  - Every pointer named "device" is GPU memory on the current HIP device; "host" is CPU memory.
 *  - Matrices are row-major: H is R x R, V is J x R, W is K x R, Qtilde is S x R (row i belongs
 *    to visit row i of the input; U_k = Qtilde_k H).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). All GPU work is
 *    ordered on it. Calls return after enqueueing, except where a call says it synchronises.
 *  - Errors: every call returns a copa_status and never aborts; copa_last_error() gives a
 *    thread-local message for the last failure of the calling thread.
 */
#ifndef COPA_H
#define COPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  COPA_OK = 0,
  COPA_EINVAL = -1,        /* bad argument, shape or input content (checked before any update) */
  COPA_ENOMEM = -2,        /* device allocation failed */
  COPA_EDEVICE = -3,       /* a HIP runtime call failed */
  COPA_ENUMERIC = -4,      /* non-finite value or failed Cholesky during the fit */
  COPA_EUNSUPPORTED = -5   /* a size outside what this build supports (R, l) */
} copa_status;

/* Proximity operators (Section "Examples of useful constraints"). The prox argument is
 * x = Z - D (Algorithm 1 inner loop) and rho is the mode's ADMM step size.
 *   NONE       x                            (unconstrained)
 *   NONNEG     max(0, x)                    (non-negativity)
 *   L1         sign(x) max(|x| - lam/rho, 0)   (l1 sparsity, soft threshold)
 *   L0         x if x*x > lam else 0        (l0 sparsity, hard threshold; lam plays mu)
 *   NONNEG_L1  max(0, x - lam/rho)                                                         */
typedef enum {
  COPA_PROX_NONE = 0,
  COPA_PROX_NONNEG = 1,
  COPA_PROX_L1 = 2,
  COPA_PROX_L0 = 3,
  COPA_PROX_NONNEG_L1 = 4
} copa_prox;

/* The irregular tensor {X_k}: CSR by subject (Algorithm 1 input). All arrays are device memory
 * owned by the caller; copa_plan_create copies what it needs, so they may be freed afterwards.
 *   subj_ptr [K+1]  visit-row offsets: subject k owns rows [subj_ptr[k], subj_ptr[k+1]),
 *                   subj_ptr[0] = 0, non-decreasing, subj_ptr[K] = S (a subject may have 0 rows)
 *   row_ptr  [S+1]  nonzero offsets per visit row, row_ptr[0] = 0, row_ptr[S] = nnz
 *   col      [nnz]  feature ids in [0, J), strictly increasing within a row
 *   val      [nnz]  finite values (counts in the paper's use)
 *   days     [S]    visit day of each row (finite); with l > 0 and basis == NULL the library
 *                   evaluates the cubic spline basis at these days (Section "Smoothness on U_k":
 *                   clamped knots, l - 4 equally spaced interior knots on the subject's span)
 *   basis    [S*l]  optional caller basis, FP64 row-major: row i holds M_k(i, :) of the subject
 *                   that owns visit row i (for example a basis on knots the caller placed);
 *                   when given, days is not read. Only span(M_k) enters the fit.
 * Limits: S and nnz below 2^31; J below 2^31.                                              */
typedef struct copa_tensor {
  int64_t K, J, S, nnz;
  const int64_t *subj_ptr;
  const int64_t *row_ptr;
  const int32_t *col;
  const float *val;
  const double *days;
  int32_t l; /* spline basis functions per subject; 0 = no smoothing; this build: 0 or 1..8 */
  const double *basis;
} copa_tensor;

/* Arithmetic of the streaming passes (copa_options.precision).
 *   FP32   the MTTKRP and SpMM inputs (nonzeros, basis rows or the projected data C_k^T X_k, and
 *          the factor rows) in FP32, FP32 accumulation; the Procrustes eigenproblems, Grams and
 *          ADMM systems in FP64
 *   MIXED  the projected data C_k^T X_k held a second time as bfloat16 (16-byte records, half
 *          the bytes each pass streams) with FP32 accumulation; the last mixed_refine iterations
 *          of each copa_fit call stream the FP32 records again (refinement), so that the returned
 *          factors, MTTKRPs and FIT come from FP32 inputs. Needs smoothing with l <= 7, J <= 65536
 *          and at most two nonzeros per visit row on average (COPA_EUNSUPPORTED otherwise).   */
typedef enum { COPA_PREC_FP32 = 0, COPA_PREC_MIXED = 1 } copa_precision;

/* Block order of one outer iteration (copa_options.order). Algorithm 1 updates its blocks
 * Z1 = H, Z2 = W (the diagonals of S_k), Z3 = V in that order (HWV). WHV updates W first, with
 * the H of the previous outer iteration, then H with the new W, then V: the same blocks and the
 * same fixed points, different iterates. On the GPU it lets the W update share one pass over the
 * Procrustes outputs with the H block's MTTKRP, instead of two passes and a written M row set
 * that is read again.                                                                           */
typedef enum { COPA_ORDER_HWV = 0, COPA_ORDER_WHV = 1 } copa_order;

/* Fit options. R: target rank (this build: 1..64 from the list copa_rank_supported accepts).
 * inner_iters: ADMM steps per factor per outer iteration (>= 1). rank_rtol: Procrustes
 * truncation - singular values of X_k' V S_k H^T at or below rank_rtol * sigma_1 are dropped
 * (default 1e-6 when <= 0). basis_rtol: rank tolerance of the smoothing basis M_k (default 1e-10
 * when <= 0). lambda_*: penalty weight of each factor's prox (see copa_prox).                */
typedef struct copa_options {
  int32_t R;
  int32_t inner_iters;
  int32_t prox_H, prox_W, prox_V;
  double lambda_H, lambda_W, lambda_V;
  double rank_rtol;
  double basis_rtol;
  /* Optional stop: when stop_tol > 0, copa_fit evaluates the stationarity residual (see
   * copa_stationarity) every check_every outer iterations (default 10 when <= 0) and returns
   * early once its largest block value is below stop_tol. 0 = fixed iteration count.          */
  double stop_tol;
  int32_t check_every;
  int32_t precision;     /* copa_precision; 0 = FP32                                          */
  int32_t mixed_refine;  /* MIXED: final iterations per copa_fit call on FP32 records (>= 0)  */
  /* 1: every reduction in a fixed order (no floating-point atomics), so that two runs on the
   * same inputs give bitwise equal results. Needs the chunked pass 2 (J <= 65536 and a F_V tile
   * that fits LDS); the plan is refused with COPA_EUNSUPPORTED otherwise.                     */
  int32_t deterministic;
  /* 1: the workspace also holds the buffers of copa_loss_grad and copa_stationarity (2 S R +
   * J R floats and S R floats more). Implied by stop_tol > 0.                                 */
  int32_t adjoint;
  /* 1: the first copa_fit on the plan picks the launch shapes (pass-1 blocks per compute unit,
   * the Procrustes kernel variant for smoothed R > 16, row-Gram blocks, pass-2 grid width) by
   * timing the candidates on the fit's starting point, or reads them from the file named by the
   * environment variable COPA_TUNE_CACHE (lines "<J> <R> <l> <projected> <precision> <log2 K>
   * <compute units> : <four shapes>"; tuned shapes are appended there). Not with deterministic
   * = 1, whose fixed summation order needs fixed shapes. 0: fixed default shapes.            */
  int32_t autotune;
  int32_t order;  /* copa_order; 0 = Algorithm 1's H -> W -> V                              */
} copa_options;

/* Fit state, device memory owned by the caller, FP32 row-major. In: the starting point
 * (auxiliary variables Hbar = H, Wbar = W, Vbar = V and duals D_*; D_* = 0 for a fresh start).
 * Out: the state after the last iteration (Algorithm 1 output H = Hbar_1, W = Hbar_2,
 * V = Hbar_3).
 *   H, D_H: R x R;  W, D_W: K x R;  V, D_V: J x R
 * iter (host field): outer iterations this state has been through; 0 marks a fresh start.
 * copa_fit adds the iterations it ran. When a call continues the state that the plan's previous
 * copa_fit returned (same buffers, iter unchanged since), it also continues the Procrustes warm
 * start, so that n + m iterations in two calls give the same numbers as n + m in one call (bitwise
 * with deterministic = 1). Any other state starts the warm start afresh.                     */
typedef struct copa_state {
  float *H, *W, *V;
  float *D_H, *D_W, *D_V;
  int32_t iter;
} copa_state;

/* Fit report (host memory). fit_history / objective_history are optional host arrays of
 * length `iters` (NULL to skip). FIT = 1 - sum_k ||X_k - U_k S_k V^T||^2 / sum_k ||X_k||^2
 * (Section "Evaluation Metrics"); objective = 1/2 sum_k ||X_k - U_k S_k V^T||^2 plus the
 * l1 penalties; sparsity_V = share of exact zeros in V (SPARSITY metric).
 * rank_deficient: subjects whose Procrustes rank was below min(rows, R) in the last iteration
 * (zero entries of W, rank-deficient smoothing bases, ...). stationarity: the largest block
 * stationarity residual at the last check (stop_tol > 0), else -1.                           */
typedef struct copa_report {
  int32_t iters_done;
  int32_t fail_iter; /* first iteration with a non-finite value or a failed ADMM system, or -1 */
  double fit;
  double objective;
  double sparsity_V;
  int64_t rank_deficient;
  double *fit_history;
  double *objective_history;
  double stationarity;
} copa_report;

typedef struct copa_plan copa_plan;

/* Device memory of a plan: every buffer the plan uses (packed tensor, smoothing basis, iteration
 * row spaces, pass-2 layout, Gram partials, and with opt->adjoint the adjoint's buffers) lives in
 * one workspace of *bytes bytes, sized here from the shapes and options alone (a bound where the
 * layout depends on the data). Reads no device memory.                                       */
copa_status copa_workspace_bytes(const copa_tensor *X, const copa_options *opt, size_t *bytes);

/* Validates the tensor (shapes on the host, CSR content on the device), packs it into the
 * workspace, builds the per-subject smoothing bases (l > 0) and lays out every buffer the fit
 * needs. workspace: device memory of at least copa_workspace_bytes bytes, 256-byte aligned,
 * owned by the caller and not touched by anyone else until copa_plan_destroy; or NULL, and the
 * library allocates it (one hipMalloc) and frees it in copa_plan_destroy. No later call on the
 * plan allocates device memory. Synchronises `stream`. Returns COPA_EINVAL for bad shapes or
 * content or a workspace that is too small or misaligned, COPA_EUNSUPPORTED for R, l or options
 * outside this build, COPA_ENOMEM when the library's own allocation fails.                   */
copa_status copa_plan_create(const copa_tensor *X, const copa_options *opt, void *workspace,
                             size_t workspace_bytes, void *stream, copa_plan **out);

/* Runs `iters` outer iterations of Algorithm 1 from `state` (updated in place, state->iter
 * advanced). Qtilde (device, S x R, may be NULL) receives C_k Q_k of the last iteration (Q_k
 * without smoothing), so that U_k = Qtilde_k H. `rep` (host, may be NULL) receives the report.
 * Synchronises `stream` at the end, and every check_every iterations when stop_tol > 0.
 * Allocates nothing. Returns COPA_ENUMERIC (and sets rep->fail_iter) when a non-finite value or
 * a non-positive pivot of an ADMM system occurred; iterations are then run in chunks of up to
 * 1024 (the whole call when it is shorter), so the state holds the values at the end of the
 * chunk in which the failure happened. iters = 0 is valid and only refreshes Qtilde/rep.     */
copa_status copa_fit(copa_plan *plan, copa_state *state, int32_t iters, float *Qtilde,
                     copa_report *rep, void *stream);

/* MTTKRPs of the last completed iteration (Algorithm 1, "F" of each mode): F_H (R x R),
 * F_W (K x R), F_V (J x R), device, FP32; any may be NULL. Enqueued on `stream`.             */
copa_status copa_mttkrp_last(copa_plan *plan, float *F_H, float *F_W, float *F_V, void *stream);

/* The smoothing basis the plan built: C (device, S x l, FP32; row i of subject k holds row i
 * of C_k, columns >= r_k are zero) and rank (device, K, int32: r_k). Only when l > 0.      */
copa_status copa_plan_basis(copa_plan *plan, float *C, int32_t *rank, void *stream);

/* Reconstruction loss of eq. Classic_PARAFAC2_obj_func with U_k = Qtilde_k H, Qtilde held fixed:
 *   L = 1/2 sum_k ||X_k - Qtilde_k H S_k V^T||_F^2,  S_k = diag(W(k,:)),
 * and its gradient: dH (R x R), dV (J x R), dW (K x R), optional dS (K x R x R, the full
 * dL/dS_k; may be NULL). Inputs and outputs are device FP32; *loss is written to host memory
 * (the call synchronises `stream`). Needs a plan created with opt->adjoint = 1 (or stop_tol >
 * 0): COPA_EINVAL otherwise. Allocates nothing.                                              */
copa_status copa_loss_grad(copa_plan *plan, const float *H, const float *V, const float *W,
                           const float *Qtilde, float *dH, float *dV, float *dW, float *dS,
                           double *loss, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc), also on plans created without opt->adjoint: the same
 * loss and gradient as copa_loss_grad, with the adjoint's work memory (2 S R + J R floats plus 4
 * per 256 subjects' rows block) taken from a static device array of 64 MiB (16 Mi floats) that
 * the library holds on each GPU it runs on until the process ends. Larger problems return
 * COPA_EINVAL. Allocates nothing. Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU race (issue them on one stream, or serialise them). Synchronises `stream`. */
copa_status copa_loss_grad_static(copa_plan *plan, const float *H, const float *V, const float *W,
                                  const float *Qt, float *dH, float *dV, float *dW, float *dS,
                                  double *loss, void *stream);

/* Frees every device buffer of the plan (synchronises its device first). NULL is a no-op.   */
void copa_plan_destroy(copa_plan *plan);

/* copa_fit replays each outer iteration from one hipGraph (captured on a stream of the plan on
 * the first call and again when the state buffers change), which removes the per-kernel launch
 * cost. copa_set_graph(plan, 0) launches the kernels one by one instead (as does per-kernel
 * timing). Default: enabled.                                                                 */
copa_status copa_set_graph(copa_plan *plan, int32_t enable);

/* Stationarity residual of each factor block of the penalised reconstruction loss at (H, V, W)
 * with Qtilde fixed (the adjoint of copa_loss_grad supplies the gradient):
 *   r_n = || Z_n - prox_n(Z_n - dL/dZ_n / rho_n) ||_F / || Z_n ||_F,   n = H, W, V,
 * with each block's proximity operator and weight from the plan's options and rho_n =
 * trace(G_n) / R (G_H = W^TW * V^TV, G_W = H^TH * V^TV, G_V = H^TH * W^TW, the steps of
 * Algorithm 1). r_n = 0 exactly at a first-order stationary point of the block. Arguments as
 * for copa_loss_grad (device memory); res: 3 doubles (host) in the order H, W, V. Needs a plan
 * created with opt->adjoint = 1 (or stop_tol > 0); synchronises `stream`. Where Q_k^T Q_k != I (subjects with fewer
 * rows than R, or a basis of rank below R) the ADMM blocks fit Q_k^T X_k rather than X_k, and
 * the residual of the reconstruction loss need not vanish at the fit's fixed point.          */
copa_status copa_stationarity(copa_plan *plan, const float *H, const float *V, const float *W,
                              const float *Qtilde, double *res, void *stream);

/* Per-kernel GPU timing of copa_fit for benchmarking. copa_set_timing(plan, 1) makes later
 * copa_fit calls record a HIP event pair on `stream` around every kernel launch (events are
 * created here, once per plan; copa_fit then synchronises every 64 iterations to read them).
 * copa_read_timing writes, per kernel id in [0, COPA_NUM_KERNELS), the summed milliseconds
 * (`ms`, host) and launch counts (`launches`, host) since the previous read, then resets them.
 * copa_kernel_name(id) names the kernel.                                                     */
#define COPA_NUM_KERNELS 14
copa_status copa_set_timing(copa_plan *plan, int32_t enable);
copa_status copa_read_timing(copa_plan *plan, double *ms, int64_t *launches);
const char *copa_kernel_name(int32_t id);

/* Facts about a plan's device layout, for reports and tests: `what` is one of
 *   COPA_QUERY_COMPACT  1 if pass 1 streams the compact nonzeros (feature id below 2^16 and every
 *                       value exactly representable as bfloat16, so the 4-byte form is lossless),
 *   COPA_QUERY_CHUNKS   number of pass-2 chunks (0 if pass 2 uses its unchunked form),
 *   COPA_QUERY_WAVES    number of pass-1 wave entries,
 *   COPA_QUERY_PAIRS    number of (subject, feature) pairs of the projected data C_k^T X_k that
 *                       the passes stream (smoothed plans with at most two nonzeros per visit
 *                       row on average), or 0 when they stream the nonzeros and basis rows,
 *   COPA_QUERY_TUNED    0 launch shapes not tuned (yet), 1 timed on this plan, 2 read from the
 *                       tuning cache file,
 *   COPA_QUERY_PASS1_BLOCKS_PER_CU, COPA_QUERY_PROCRUSTES_VARIANT, COPA_QUERY_GRAM_BLOCKS,
 *   COPA_QUERY_PASS2_BLOCKS   the launch shapes in use (see copa_options.autotune),
 *   COPA_QUERY_WFIRST_BLOCKS, COPA_QUERY_MROWS_BLOCKS   block order W -> H -> V: blocks of the
 *                       persistent W-block and M-row launches (0 before the first fit).
 * *out (host) receives the value. COPA_EINVAL for a NULL argument or an unknown `what`.       */
#define COPA_QUERY_COMPACT 0
#define COPA_QUERY_CHUNKS 1
#define COPA_QUERY_WAVES 2
#define COPA_QUERY_PAIRS 3
#define COPA_QUERY_TUNED 4
#define COPA_QUERY_PASS1_BLOCKS_PER_CU 5
#define COPA_QUERY_PROCRUSTES_VARIANT 6
#define COPA_QUERY_GRAM_BLOCKS 7
#define COPA_QUERY_PASS2_BLOCKS 8
#define COPA_QUERY_WFIRST_BLOCKS 9
#define COPA_QUERY_MROWS_BLOCKS 10
copa_status copa_plan_query(const copa_plan *plan, int32_t what, int64_t *out);

/* 1 if this build has kernels for rank R, else 0.                                           */
int32_t copa_rank_supported(int32_t R);

const char *copa_status_string(copa_status status);
const char *copa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* COPA_H */
