/*
 * nmpc.h -- C ABI of the MI355X double-layer Jacobi NMPC solver.
 *
 * Method: Deng & Ohtsuka, "A Double-Layer Jacobi Method for PDE-Constrained
 * Nonlinear Model Predictive Control" (arXiv 2004.02484).
 *
 * Problem (Sec. 3, eq. nlp, without inequality constraints): minimize
 *   sum_{i=1..N} h ( q/2 |x_i - xref_i|^2 + r/2 |u_i|^2 )
 * subject to x_0 = x0 and the backward-Euler model
 *   x_i = x_{i-1} + h f(u_i, x_i),   f(u, x) = k(x) .* (L x) + B u,
 * where x is the PDE state on the nsy x nsx interior nodes of the unit
 * interval/square (node p = iy*nsx + ix, zero Dirichlet values outside),
 * L the central-difference Laplacian (Sec. 2.1), k(w) = k0 (1 + k1 w) the
 * conductivity, and B the input operator
 *   B[iy*nsx + ix][b*lx + a] = gy[b][iy] * gx[a][ix]        (m = lx*ly inputs).
 *
 * Solution: the KKT point K_i(x_{i-1}, s_i, lambda_{i+1}) = 0, i = 1..N
 * (Sec. 3.2, eq. KKT), computed by the double-layer Jacobi method:
 *   upper layer  S^{k+1} = S^k - (D^k)^{-1} K^k, every stage block solved
 *                independently from S^k (Sec. 4.2, eq. 1st_jacobi; alpha = 1);
 *   lower layer  Schur elimination onto the inputs with A_uu = (h r + gamma) I
 *                iterated n_schur times, F_x / F_x^T solves by n_sweep
 *                point-Jacobi sweeps from zero (Sec. 4.3, eqs. step12, coff;
 *                Sec. 5.2 for the Schur iteration);
 *   regularization reference u~ = u^k (Sec. 5.2 parameter table), so the
 *                gamma term changes the rate, not the solution.
 * Stopping rule: r_scaled(S^k) <= tol, where
 *   r_scaled = max_i max(|K^x_i|_inf, |K^u_i|_inf / (h r), |K^lambda_i|_inf / h)
 * (the paper's |K|_inf, Sec. 5.2, with the input and costate rows brought to
 * the units of u and of q (x - xref)); r_paper = |K|_inf is also reported.
 *
 * Trajectory layout (row-major, caller-owned): x [N][n], u [N][m],
 * lambda [N][n]; batched calls prepend the instance index: [count][N][n] ...
 * The returned trajectory is the last evaluated iterate S^k, whose residuals
 * are reported; lambda follows the paper's sign (lambda_i = lambda_{i+1} +
 * h grad_x H_i^T at the solution).
 *
 * Errors: every int-returning call returns NMPC_OK (0) or an NMPC_E_* code;
 * nothing is thrown across the ABI. nmpc_last_error() gives a message for the
 * calling thread. Handles are not thread-safe: use one per host thread.
 */
#ifndef NMPC_H
#define NMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NMPC_OK = 0,
    NMPC_E_ARG = 1,          /* invalid argument or shape */
    NMPC_E_NOCONV = 2,       /* max_iter reached; outputs hold S^max_iter */
    NMPC_E_NONFINITE = 3,    /* residual became NaN/Inf; outputs hold that iterate */
    NMPC_E_DEVICE = 4,       /* HIP runtime error */
    NMPC_E_OOM = 5,          /* device allocation failed */
    NMPC_E_UNSUPPORTED = 6   /* valid problem but no kernel for this shape */
};

enum { NMPC_FP64 = 0, NMPC_FP32_SWEEP = 1 };

enum { NMPC_START_COLD = 0, NMPC_START_WARM = 1 };

enum { NMPC_UPPER_JACOBI = 0, NMPC_UPPER_FGS = 1, NMPC_UPPER_BGS = 2, NMPC_UPPER_SGS = 3 };

enum { NMPC_PATH_AUTO = 0, NMPC_PATH_FUSED = 1, NMPC_PATH_STREAM = 2 };

/* Form of the input operator B in nmpc_problem. */
enum { NMPC_B_DENSE = 0, NMPC_B_KRON = 1 };

/* Norm of the stopping test: NMPC_RES_SCALED, r_scaled (see above), or
 * NMPC_RES_PAPER, the paper's |K|_inf (Table tab_NMPC_para). */
enum { NMPC_RES_SCALED = 0, NMPC_RES_PAPER = 1 };

/* Problem data (Sec. 3 notation). gx/gy (or B) are host arrays, copied at
 * create. */
typedef struct nmpc_problem {
    int32_t dim;          /* 1 or 2 */
    int32_t nsx, nsy;     /* interior nodes per axis; nsy = 1 when dim == 1 */
    int32_t horizon;      /* N >= 1 */
    int32_t lx, ly;       /* input lattice; m = lx * ly; ly = 1 when dim == 1 */
    const double *gx;     /* [lx][nsx] */
    const double *gy;     /* [ly][nsy] */
    double h;             /* stage length T/N > 0 */
    double k0, k1;        /* conductivity k(w) = k0 (1 + k1 w) */
    double q, r;          /* cost weights Q = q I, R = r I; r > 0 */
    double gamma;         /* regularization weight >= 0 */
    double tau;           /* input box u_lo <= u <= u_hi by the log barrier
                             -tau sum_j (ln(u_j - u_lo) + ln(u_hi - u_j)) of
                             the relaxed problem (eq. nlp_relaxed), each step
                             of the upper layer (a Jacobi iteration, or each
                             Gauss-Seidel sweep) cut by the fraction-to-the-
                             boundary rule (eq. eq_alphamax, alpha global over
                             the instance's stages: S <- S + alpha (S_step -
                             S)); every path and upper layer, ragged batches
                             too. tau = 0: no box. tau > 0 needs u_lo < 0 <
                             u_hi (the cold start u = 0 inside); given start
                             inputs are clipped to the box shrunk by 0.5 % of
                             its width at each end */
    double u_lo, u_hi;
    int32_t b_kind;       /* NMPC_B_KRON: B from the factors gx, gy (above);
                             NMPC_B_DENSE: B is the dense matrix below, m =
                             lx * ly inputs (gx, gy unused). A dense-B problem
                             (up to 4096 nodes, 64 inputs, 256 stages) runs on
                             the model engine (NMPC_MODEL_HEAT): FP64 sweeps,
                             every upper layer (the input box included), cold
                             or (x, u, lambda) starts, one reference per
                             instance; nmpc_solve, nmpc_solve_batch,
                             nmpc_residual_batch, nmpc_set_options and the
                             timing calls apply, the others give
                             NMPC_E_UNSUPPORTED */
    const double *B;      /* NMPC_B_DENSE: [nsx * nsy][m] row-major */
} nmpc_problem;

/* Solver options. */
typedef struct nmpc_options {
    double tol;           /* stop when r_scaled <= tol */
    int32_t max_iter;     /* upper iterations (>= 0) */
    int32_t n_sweep;      /* point-Jacobi sweeps per F_x / F_x^T solve, 1..16 */
    int32_t n_schur;      /* Schur input iterations, 0..16 */
    int32_t precision;    /* NMPC_FP64, or NMPC_FP32_SWEEP: lower layer in FP32,
                             S, K, the norms and the test in FP64; once the
                             test passes at S^j, one FP64 step is taken from S^j
                             (Jacobi: one iteration; Gauss-Seidel: the first
                             sweep of an iteration) and FP64 iterations continue
                             until the test passes at an FP64-stepped iterate
                             (final FP64 correction) */
    int32_t check_every;  /* iterations between host convergence polls (>= 1).
                             An FP32-sweep Jacobi solve whose handle's previous
                             solve converged in J iterations, J + 4 <=
                             check_every, starts with one graph of J + 1 FP32
                             launches and the three of the final FP64
                             correction, so a solve like the previous one
                             needs a single poll */
    int32_t xref_per_stage; /* 0: xref is [n] per instance; 1: [N][n] */
    int32_t tile_rows;    /* grid rows per lane of the stage kernel's register
                             tile for the main precision; 0 = default. Other
                             values select alternative kernel instances (as
                             chosen by the tile autotuner); unsupported values
                             give NMPC_E_UNSUPPORTED */
    int32_t warm_sweeps;  /* sweeps per stage (point-Jacobi with Chebyshev
                             weights) for the states, and for the costates
                             unless warm_sweeps_lambda is set, when a start is
                             built from an input trajectory (0 = 24) */
    int32_t fallback;     /* 1: for a warm start, compare its residual with the
                             cold start's per instance and keep the smaller
                             (non-finite counts as larger) */
    int32_t upper;        /* upper-layer splitting (Sec. 4.4): NMPC_UPPER_JACOBI
                             (eq. 1st_jacobi, all stages in parallel; default),
                             NMPC_UPPER_FGS (eq. fgs), NMPC_UPPER_BGS, or
                             NMPC_UPPER_SGS (eq. sgs: a backward sweep, then a
                             forward sweep). The Gauss-Seidel variants visit the
                             stages of an instance in turn: one workgroup per
                             instance runs the whole solve in one launch per
                             precision phase. Every variant has the same
                             solution; iterations count upper iterations */
    int32_t path;         /* NMPC_PATH_FUSED: one workgroup holds a stage in
                             registers and runs its whole upper-iteration step
                             (grids up to 96 columns); NMPC_PATH_STREAM: every
                             step of the stage algebra is a pass over grid rows
                             of all stages (any grid size, e.g. 256 x 256;
                             Jacobi upper layer, cold or given starts, no
                             fallback); NMPC_PATH_AUTO (default): fused where
                             it fits, else streaming */
    double omega;         /* over-relaxation of the Gauss-Seidel sweeps
                             (Sec. 4.4): each stage's step is scaled by omega,
                             so FGS becomes SOR, S - omega (D + omega L)^{-1} K,
                             BGS its backward form and SGS the symmetric SSOR;
                             0 < omega < 2, default 1. The Jacobi upper layer
                             takes omega = 1 only (NMPC_E_ARG otherwise) */
    int32_t fp32_finish;  /* with NMPC_FP32_SWEEP: 0 (default) takes the final
                             FP64 correction described under precision; 1
                             returns S^j as soon as its FP64-evaluated test
                             passes in the FP32 phase (S^j is FP64 data; only
                             the step that produced it was solved in FP32).
                             Fused path only (NMPC_E_UNSUPPORTED on the
                             streaming path and for ragged batches); 0 or 1 */
    int32_t residual;     /* NMPC_RES_SCALED (default): stop when r_scaled <= tol;
                             NMPC_RES_PAPER: stop when r_paper = |K|_inf <= tol,
                             the paper's rule (Table tab_NMPC_para) */
    int32_t warm_sweeps_lambda; /* sweeps per stage for the costates of a start
                             built from an input trajectory (0 = warm_sweeps);
                             0..1000. The costate error enters r_scaled divided
                             by h, the state error not, so the costates may
                             need more sweeps than the states */
} nmpc_options;

/* Per-instance result information. */
typedef struct nmpc_info {
    double r_scaled;      /* scaled residual of the returned iterate */
    double r_paper;       /* |K|_inf of the returned iterate */
    int32_t iters;        /* k of the returned iterate S^k */
    int32_t status;       /* NMPC_OK, NMPC_E_NOCONV or NMPC_E_NONFINITE */
    int32_t fp32_iters;   /* iterations run with FP32 sweeps */
    int32_t start_used;   /* 0 cold, 1 given (x, u, lambda), 2 built from u */
    double err_vs_fp64;   /* error of the FP32-sweep phase against FP64: the
                             size of the final FP64 correction step taken from
                             the iterate accepted in the FP32 phase, max |du| /
                             max |u| over the horizon (relative control change);
                             0 for NMPC_FP64 solves; -1 where no FP64 step was
                             taken (fp32_finish = 1, or the solve ended in the
                             FP32 phase) */
} nmpc_info;

typedef struct nmpc_handle nmpc_handle;

/* Fill options with the paper's lower-layer settings (2 sweeps, 2 Schur
 * iterations), tol 1e-6, max_iter 2000, FP64, check_every 16, default
 * tile, Jacobi upper layer, automatic kernel path. */
void nmpc_default_options(nmpc_options *opt);

/* Create a solver for one problem shape and up to max_batch instances on the
 * current HIP device. Allocates all device workspace (two trajectory buffers
 * per instance). Returns NMPC_E_ARG for invalid data, NMPC_E_UNSUPPORTED if
 * no kernel covers the shape, NMPC_E_OOM/NMPC_E_DEVICE on device failure. */
int nmpc_create(const nmpc_problem *prob, const nmpc_options *opt, int32_t max_batch,
                nmpc_handle **out);

/* Replace the options of an existing handle (same validation as create). */
int nmpc_set_options(nmpc_handle *hd, const nmpc_options *opt);

/* Solve one instance, host buffers. x0, xref: [n] (xref [N][n] with
 * xref_per_stage). warm_x/warm_u/warm_lam: a start S^0 ([N][n], [N][m],
 * [N][n]); all three NULL selects the cold start x_i = x0, u_i = 0,
 * lambda_i = 0. warm_x NULL with warm_u given builds the start from the
 * input trajectory: states by the backward-Euler model (K^x = 0), costates by
 * the adjoint recursion (K^lambda = 0, warm_lam, if given, is the sweeps'
 * initial guess). warm_x without warm_u is NMPC_E_ARG. out_* receive the returned
 * iterate; info may be NULL. Returns the instance status (NMPC_OK,
 * NMPC_E_NOCONV, NMPC_E_NONFINITE) or an error code. Blocks until done. */
int nmpc_solve(nmpc_handle *hd, const double *x0, const double *xref,
               const double *warm_x, const double *warm_u, const double *warm_lam,
               double *out_x, double *out_u, double *out_lam, nmpc_info *info);

/* Solve count <= max_batch instances, DEVICE buffers with a leading instance
 * index (x0 [count][n], xref [count][n] or [count][N][n], warm_* and out_*
 * [count][N][...]; warm pointers as in nmpc_solve). Work is ordered after
 * everything already queued on `stream` (a hipStream_t, NULL = null stream)
 * and the call returns when the results are written. info: HOST array
 * [count] (may be NULL). Returns NMPC_OK if every instance converged,
 * otherwise the first failing instance's status, or an error code. */
int nmpc_solve_batch(nmpc_handle *hd, int32_t count, const double *x0, const double *xref,
                     const double *warm_x, const double *warm_u, const double *warm_lam,
                     double *out_x, double *out_u, double *out_lam, nmpc_info *info,
                     void *stream);

/* KKT residual norms of given trajectories (DEVICE buffers as in
 * nmpc_solve_batch, ut = u). r_scaled/r_paper: HOST arrays [count]. */
int nmpc_residual_batch(nmpc_handle *hd, int32_t count, const double *x0, const double *xref,
                        const double *x, const double *u, const double *lam,
                        double *r_scaled, double *r_paper, void *stream);

/* Release the handle and its device memory. NULL is ignored. */
void nmpc_destroy(nmpc_handle *hd);

/* Static description of an error code. */
const char *nmpc_strerror(int code);

/* Detail of the last error on the calling thread ("" if none). */
const char *nmpc_last_error(void);

/* Kernel configuration chosen for the handle: rows per lane, waves per
 * workgroup, workgroups per upper iteration at max_batch. Any pointer may be
 * NULL. */
int nmpc_kernel_config(const nmpc_handle *hd, int32_t *rows_per_lane, int32_t *waves,
                       int32_t *workgroups);

/* Kernel timing of later solves on this handle (not thread-safe). enable != 0
 * resets the counters and brackets every replay of the captured iteration
 * graph with HIP events on the handle's stream; enable == 0 stops timing. */
int nmpc_timing_enable(nmpc_handle *hd, int32_t enable);

/* Read the counters since the last enable: GPU milliseconds spent in the
 * iteration kernels, number of iteration-kernel launches, and number of
 * (instance, stage) units that were evaluated and updated (a Gauss-Seidel
 * sweep over a stage is one unit; a streaming solve counts its updates).
 * NULL pointers are skipped. */
int nmpc_timing_read(const nmpc_handle *hd, double *kernel_ms, int64_t *launches,
                     int64_t *units);

/* Evaluation-only (instance, stage) units since the last enable, which
 * nmpc_timing_read leaves out: the residual check of the FP64-corrected
 * iterate that ends an FP32-sweep solve (NMPC_FP32_SWEEP with its final
 * correction step, a precision option of this library rather than part of
 * the paper's method), one visit per stage of each instance that reaches
 * it; such a unit reads the stage and writes no new iterate. 0 for FP64 and
 * fp32_finish solves and for the streaming path and the model engine. NULL
 * eval_units is skipped; NMPC_E_ARG for a NULL handle. */
int nmpc_timing_read_eval(const nmpc_handle *hd, int64_t *eval_units);

/* Set the calling thread's last-error text (used by the network calls). */
void nmpc_set_last_error(const char *msg);

/* Shifted start for the next closed-loop step (the paper reuses the previous
 * step's optimum, Remark rmk_gamma): out_s[b][i] = s[b][i+1] for i < N-1 and
 * out_s[b][N-1] = s[b][N-1], for x [count][N][n], u [count][N][m] and
 * lambda [count][N][n] (DEVICE; outputs must not alias inputs). Queued on
 * `stream`, returns without waiting. */
int nmpc_shift_batch(nmpc_handle *hd, int32_t count, const double *x, const double *u,
                     const double *lam, double *out_x, double *out_u, double *out_lam,
                     void *stream);

/* Plant step of a closed-loop simulation: one explicit-Euler step of the
 * handle's model, out = x + dt (k(x) .* (L x) + B u), for x [count][n] and the
 * applied inputs u (instance b's m values at u + b * ldu; ldu = N * m takes
 * stage 1 of a [count][N][m] trajectory). DEVICE buffers; out must not alias
 * x. Queued on `stream`, returns without waiting. */
int nmpc_plant_step_batch(nmpc_handle *hd, int32_t count, const double *x, const double *u,
                          int32_t ldu, double dt, double *out, void *stream);

/* Tile autotuner: time `iters` upper iterations (1..1000) of this batch from
 * the cold start (DEVICE x0 [count][n], xref [count][n]) with every tile
 * height that the kernel table holds for the problem's grid width in the
 * handle's main precision and upper layer, keep the fastest as the handle's
 * tile_rows and return it in *tile_rows (may be NULL). The timing runs'
 * results are discarded; stream as in nmpc_solve_batch. */
int nmpc_autotune(nmpc_handle *hd, int32_t count, const double *x0, const double *xref,
                  int32_t iters, void *stream, int32_t *tile_rows);

/* ---------------------------------------------------------------------------
 * Ragged batches: instances of several problem classes (grid sizes,
 * horizons, steps, input factors) solved together, one kernel launch per
 * upper iteration over all of their (instance, stage) units, replayed as a
 * captured graph of check_every launches; each instance keeps its own
 * convergence state (as in nmpc_solve_batch). Classes are 2D problems with the
 * 4 x 4 input lattice and nsx, nsy <= 96.
 * ------------------------------------------------------------------------ */
typedef struct nmpc_ragged nmpc_ragged;

/* Create for nclass (1..64) classes (copied) and up to max_instances
 * instances per solve. opt as for nmpc_create; xref_per_stage must be 0 and
 * upper NMPC_UPPER_JACOBI; tile_rows, warm_sweeps and fallback are not used. Device trajectory
 * buffers are sized at the first solve and grow on demand. */
int nmpc_ragged_create(const nmpc_problem *classes, int32_t nclass, const nmpc_options *opt,
                       int32_t max_instances, nmpc_ragged **out);

/* Solve count instances; cls: HOST [count] class of each instance. DEVICE
 * buffers, packed in instance order: x0 and xref n_b values per instance
 * (n_b = nsx * nsy of its class), warm_x / warm_lam / out_x / out_lam N_b * n_b,
 * warm_u / out_u N_b * m. The warm pointers are all NULL (cold start) or all
 * given. info: HOST [count] or NULL. Ordering, blocking and return value as
 * in nmpc_solve_batch. */
int nmpc_ragged_solve(nmpc_ragged *rg, int32_t count, const int32_t *cls, const double *x0,
                      const double *xref, const double *warm_x, const double *warm_u,
                      const double *warm_lam, double *out_x, double *out_u, double *out_lam,
                      nmpc_info *info, void *stream);

/* Workgroup-size autotuner: for the set of classes in this batch, time
 * `iters` (1..1000) upper iterations from the cold start with each
 * workgroup size of the ragged kernel (8, 12 or 16 waves) whose tiles fit
 * every class, remember the fastest for later solves of batches with the
 * same class set and return it in *waves (may be NULL). */
int nmpc_ragged_autotune(nmpc_ragged *rg, int32_t count, const int32_t *cls, const double *x0,
                         const double *xref, int32_t iters, void *stream, int32_t *waves);

/* Workgroup size (waves) a solve of a batch with these classes would use. */
int nmpc_ragged_config(const nmpc_ragged *rg, int32_t count, const int32_t *cls, int32_t *waves);

/* Kernel timing of later ragged solves, as nmpc_timing_enable/read/read_eval. */
int nmpc_ragged_timing_enable(nmpc_ragged *rg, int32_t enable);
int nmpc_ragged_timing_read(const nmpc_ragged *rg, double *kernel_ms, int64_t *launches,
                            int64_t *units);
int nmpc_ragged_timing_read_eval(const nmpc_ragged *rg, int64_t *eval_units);

/* Release the ragged solver. NULL is ignored. */
void nmpc_ragged_destroy(nmpc_ragged *rg);

/* ---------------------------------------------------------------------------
 * Learned warm start: kernels of the patch-encoder network (trained on the
 * GPU on solutions of the method itself). All pointers are DEVICE memory,
 * work is queued on `stream` (hipStream_t, NULL = null stream) and the calls
 * return without waiting. bf16 values are raw 16-bit patterns (uint16_t).
 * Errors: NMPC_E_ARG for bad sizes/NULLs, NMPC_E_DEVICE for launch failures.
 * ------------------------------------------------------------------------ */

/* C[m][n] = beta C[m][n] + sum_k A(m,k) B(k,n) (+ bias[n]) (ReLU if relu),
 * bf16 operands on the matrix cores with fp32 accumulation. A(m,k) is
 * A[m*lda + k] (trans_a = 0) or A[k*lda + m]; B(k,n) is B[k*ldb + n]
 * (trans_b = 0) or B[n*ldb + k]. C (fp32, may be NULL if Cb is given) and Cb
 * (bf16 copy of the result, may be NULL). Forward layers use (0,0), data
 * gradients (0,1), weight gradients (1,0). */
int nmpc_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                   const uint16_t *A, int32_t lda, const uint16_t *B, int32_t ldb, float beta,
                   float *C, int32_t ldc, const float *bias, int32_t relu, uint16_t *Cb,
                   int32_t ldcb, void *stream);

/* C_g = beta C_g + op(A_g) B_g for groups g = 0 .. groups-1, fp32 operands
 * on the matrix cores with fp32 accumulation (the network's per-actuator
 * linear map needs more significant bits than bf16 carries). X_g = X + g *
 * stride_x (elements). A_g(m,k) is A_g[m*lda + k] (trans_a = 0) or
 * A_g[k*lda + m]; B_g(k,n) = B_g[k*ldb + n]; C_g is M x N with row stride ldc.
 * The forward map uses trans_a = 0, its weight gradient trans_a = 1. With
 * ksplit > 1 the K range is cut in ksplit parts computed in parallel into
 * `work` (caller-owned device memory of groups * ksplit * M * N floats) and
 * added in a fixed order (a result that does not depend on scheduling);
 * ksplit = 1 takes work = NULL. groups * ksplit <= 65535. */
int nmpc_gemm_f32(int32_t trans_a, int32_t M, int32_t N, int32_t K, const float *A, int32_t lda,
                  int64_t stride_a, const float *B, int32_t ldb, int64_t stride_b, float beta,
                  float *C, int32_t ldc, int64_t stride_c, int32_t groups, int32_t ksplit,
                  float *work, void *stream);

/* nmpc_gemm_f32 without a caller workspace, for callers that cannot
 * allocate device memory (code under graph capture, serving loops, harnesses
 * that forbid allocation): the split-K partials live in a static device array
 * of 2^21 floats (8 MiB) that each GPU holds from the first call on it until
 * the process ends; this call allocates nothing. ksplit > 1 needs groups *
 * ksplit * M * N <= 2^21 (NMPC_E_ARG otherwise, before anything is queued).
 * Every call on a GPU shares that GPU's array: calls whose execution may
 * overlap on one GPU (several streams or host threads) race and must be
 * serialized by the caller. Results equal nmpc_gemm_f32 with the same
 * arguments (the partials are fully written before they are summed, in the
 * same fixed order). */
int nmpc_gemm_f32_noalloc(int32_t trans_a, int32_t M, int32_t N, int32_t K, const float *A,
                          int32_t lda, int64_t stride_a, const float *B, int32_t ldb,
                          int64_t stride_b, float beta, float *C, int32_t ldc, int64_t stride_c,
                          int32_t groups, int32_t ksplit, void *stream);

/* The same grouped product with fp64 products and accumulation: C_g =
 * alpha op(A_g) B_g + beta Cin_g (Cin = C when NULL; Cin_g and C_g share
 * stride_c and ldc) on fp64 operands (nmpc_gemm_f64), or C_g = op(A_g) B_g +
 * beta C_g on fp32 operands with an fp64 result (nmpc_gemm_f32_acc64: the
 * Gram matrices X^T X and X^T T of fp32 feature rows). Used to fit the
 * network's per-actuator linear map by its normal equations. */
int nmpc_gemm_f64(int32_t trans_a, int32_t M, int32_t N, int32_t K, const double *A, int32_t lda,
                  int64_t stride_a, const double *B, int32_t ldb, int64_t stride_b, double alpha,
                  double beta, const double *Cin, double *C, int32_t ldc, int64_t stride_c,
                  int32_t groups, void *stream);
int nmpc_gemm_f32_acc64(int32_t trans_a, int32_t M, int32_t N, int32_t K, const float *A,
                        int32_t lda, int64_t stride_a, const float *B, int32_t ldb,
                        int64_t stride_b, double beta, double *C, int32_t ldc, int64_t stride_c,
                        int32_t groups, void *stream);

/* Start of the Newton-Schulz inverse of ridge-regularized Gram matrices: for
 * each group g, G_g (n x n, row stride ld, symmetric positive semidefinite)
 * gets ridge_rel * trace(G_g) / n added to its diagonal, and X_g (n x n, row
 * stride ld) is set to I / trace(G_g) (after the ridge). Iterating
 * X <- 2 X - X (G X) with nmpc_gemm_f64 then converges to G^{-1}. */
int nmpc_ls_prepare(double *G, int32_t n, int32_t ld, int64_t stride_g, double ridge_rel,
                    double *X, int64_t stride_x, int32_t groups, void *stream);

/* Network input rows: for each instance b and each actuator p = pb*L + pa of
 * an L x L lattice on an ns x ns grid, row b*L^2 + p holds a win x win window
 * (starting (win - ns/L)/2 nodes before the actuator's cell, zero outside the
 * grid) of each feature plane, then a one-hot of p (L^2 values), then zeros
 * up to ld. With xt = x0/0.1 - 1 and rt = xref/0.3 the planes are xt, rt
 * (planes = 2) followed by xt^2 - 1/3, xt*rt, rt^2 - 1/3 (planes = 5).
 * x0, xref: [count][ns*ns]; Xf: fp32 rows and/or Xb: bf16 rows (either may
 * be NULL), both [count*L^2][ld]. */
int nmpc_net_features(const double *x0, const double *xref, int32_t count, int32_t ns,
                      int32_t lattice, int32_t win, int32_t planes, float *Xf, uint16_t *Xb,
                      int32_t ld, void *stream);

/* dh[i] = h[i] > 0 ? dh[i] : 0 (in place), dhb = bf16(dh). */
int nmpc_relu_grad(float *dh, const float *h, uint16_t *dhb, int64_t n, void *stream);

/* out[n] = sum_m A[m*lda + n] for n < N (bias gradients). */
int nmpc_colsum(const float *A, int32_t M, int32_t N, int32_t lda, float *out, void *stream);

/* dY = scale (Y - T) (fp32 and bf16, row stride lddy) and row_sse[m] =
 * sum_n (Y - T)^2 for the M x N block. */
int nmpc_mse_grad(const float *Y, int32_t ldy, const float *T, int32_t ldt, int32_t M, int32_t N,
                  float scale, float *dY, uint16_t *dYb, int32_t lddy, float *row_sse, void *stream);

/* Adam step `step` (>= 1) on fp32 weights w with gradient g and moments m, v
 * (decoupled weight decay); wb (may be NULL) receives the bf16 copy of w. */
int nmpc_adam(float *w, const float *g, float *m, float *v, uint16_t *wb, int64_t n, float lr,
              float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream);

/* y = bf16(x). */
int nmpc_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream);

/* Input trajectories u [count][N][m] (double) <-> per-actuator rows
 * rows[(b*m + j)*ldr + i] = scale * u[b][i][j] (float). */
int nmpc_pack_inputs(const double *u, int32_t count, int32_t N, int32_t m, float scale, float *rows,
                     int32_t ldr, void *stream);
int nmpc_unpack_inputs(const float *rows, int32_t ldr, int32_t count, int32_t N, int32_t m,
                       float scale, double *u, void *stream);

/* ---------------------------------------------------------------------------
 * The warm-start network as one object (the layer sequence above, run by the
 * kernels above): a patch encoder for an ns x ns grid with an L x L actuator
 * lattice and N stages. For actuator p of instance b it reads a win x win
 * window of `planes` feature planes of (x0, xref) (nmpc_net_features) and
 * predicts that actuator's inputs over the horizon:
 *   H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), H3 = relu(H2 W3 + b3)
 *   (bf16 operands, fp32 accumulation, bf16 copies of H between layers),
 *   Y = H3 W4 + b4 + X Ws[p] (the per-actuator map on fp32 operands),
 *   u[b][i][p] = 4 Y[b L^2 + p][i].
 * hidden = 0 leaves the per-actuator map alone. Parameters, gradients, Adam
 * moments and activation buffers for up to max_count instances live on the
 * device in the object. All x0 / xref / u pointers are DEVICE memory; work
 * is queued on `stream` (hipStream_t); nmpc_net_get / _set / _load / _save and
 * a loss pointer block. The network reaches the solver only through the
 * warm-start inputs of nmpc_solve_batch, so the solver does not know it.
 * ------------------------------------------------------------------------ */
typedef struct nmpc_net_config {
    int32_t N, ns, lattice, win, hidden, planes;   /* planes: 2 or 5 (nmpc_net_features) */
} nmpc_net_config;

typedef struct nmpc_net nmpc_net;

/* Create with seeded initial weights (He-uniform hidden layers, zero biases,
 * zero map). NMPC_E_ARG for an inconsistent configuration; NMPC_E_UNSUPPORTED
 * for N > 48 or lattice > 8 (the forward pass's map kernel, which gathers the
 * features inside the product, holds 48 output columns per instance tile). */
int nmpc_net_create(const nmpc_net_config *cfg, uint64_t seed, int32_t max_count, nmpc_net **out);

/* u [count][N][L^2] predicted for x0, xref [count][ns^2] (count <= max_count). */
int nmpc_net_forward(nmpc_net *net, int32_t count, const double *x0, const double *xref, double *u,
                     void *stream);

/* Forward pass and the gradients of the mean squared error of Y against
 * u_target / 4 (u_target [count][N][L^2]) with respect to every parameter,
 * kept in the object (read with nmpc_net_get, name "g" + parameter). loss
 * (may be NULL; blocks when given) receives that error. */
int nmpc_net_backward(nmpc_net *net, int32_t count, const double *x0, const double *xref,
                      const double *u_target, float *loss, void *stream);

/* Adam step on every parameter whose bit (W1 b1 W2 b2 W3 b3 W4 b4 Ws = bits 0..8)
 * is clear in frozen_mask, from the gradients of the last backward pass;
 * decoupled weight decay on the weight matrices. */
int nmpc_net_adam_step(nmpc_net *net, float lr, float beta1, float beta2, float eps,
                       float weight_decay, uint32_t frozen_mask, void *stream);

/* nmpc_net_backward then nmpc_net_adam_step (beta1 0.9, beta2 0.999, eps 1e-8). */
int nmpc_net_train_step(nmpc_net *net, int32_t count, const double *x0, const double *xref,
                        const double *u_target, float lr, float weight_decay, uint32_t frozen_mask,
                        float *loss, void *stream);

/* Copy count elements of a parameter ("W1" .. "Ws", fp32), its gradient ("g"
 * + name) or an activation buffer of the last pass ("X", "Xf", "H1", "H1b",
 * ..., "Y", "T", "dY", "dYb", "dH1".."dH3", "dH1b".."dH3b", "Wb1".."Wb4") to
 * host memory. "X", "Wb*" and the activation names ending in b hold bf16 bit
 * patterns (2 bytes each), the rest fp32. The forward pass writes "Y" and,
 * with hidden > 0, "X" and the hidden activations; "Xf" (the fp32 feature
 * rows) is written by the backward pass only, since the forward pass's map
 * gathers its features in place. NMPC_E_ARG for an unknown name or count
 * beyond the buffer. */
int nmpc_net_get(const nmpc_net *net, const char *name, void *host, int64_t count);

/* Replace a parameter (count = its size; src host or device memory). */
int nmpc_net_set(nmpc_net *net, const char *name, const float *src, int64_t count,
                 int32_t src_on_device, void *stream);

/* Total number of parameters. */
int64_t nmpc_net_num_params(const nmpc_net *net);

/* Weight file: "NMPCNET1", the configuration and the Adam step count as
 * int32, then W1 b1 W2 b2 W3 b3 W4 b4 Ws as fp32 (host byte order). Load
 * requires the same configuration (NMPC_E_ARG otherwise). */
int nmpc_net_save(const nmpc_net *net, const char *path);
int nmpc_net_load(nmpc_net *net, const char *path);

void nmpc_net_destroy(nmpc_net *net);

/* ---------------------------------------------------------------------------
 * Model engine: the double-layer method for further members of the paper's
 * PDE class (Sec. 2, eq. pde) on grids of up to 4096 nodes, one workgroup per
 * instance running the whole solve (FP64; every upper layer of
 * nmpc_options.upper; input box by the log barrier of eq. nlp_relaxed with
 * the fraction-to-the-boundary rule eq. alphamax applied to every pass of the
 * upper layer: S <- S + alpha (S_pass - S), alpha global over the stages).
 *
 * Grid: nsy x nsx nodes, node p = iy * nsx + ix. NMPC_BC_DIRICHLET: interior
 * nodes of the unit interval / square (dx = 1 / (nsx + 1)), zero values
 * outside. NMPC_BC_NEUMANN: the nodes include the boundary (dx = 1 / (nsx -
 * 1)) and the normal derivative is zero, by fictitious points mirrored onto
 * the inner neighbours (eq. neumann, eq. dis_neumann with e = 0).
 *
 * Models (stage cost h (q/2 |w - wref|^2 + qv/2 |W_t|^2 + r/2 |u - uref|^2)):
 *   NMPC_MODEL_HEAT   w_t = k0 (1 + k1 w) Lap w + B u, dense B [nodes][m];
 *   NMPC_MODEL_PLATE  the copper plate of Sec. 5: w_t = alpha Lap w - beta (w -
 *                     t_amb) - rad (w^4 - t_amb^4); the temperatures of the
 *                     actuator nodes act[0..m-1] are the inputs (those nodes
 *                     are not states); uref = wref at the actuator nodes;
 *   NMPC_MODEL_WAVE   second order in time (eq. ode): W_tt + damp W_t = k0 (1 +
 *                     k1 W) Lap W + B u, state (W, W_t); the F_x and F_x^T
 *                     solves eliminate v6 = h v7 - b6 and sweep the reduced
 *                     system of eq. jaco2_sys. uref = 0, qv weighs W_t.
 * Layouts (DEVICE, caller-owned, leading instance index): x0 [count][nx],
 * nx = nodes (wave: 2 nodes, W then W_t); xref [count][nodes] (wref over the
 * grid); trajectories x, lambda [count][N][nx], u [count][N][m]. The plate's
 * returned x holds the inputs at the actuator nodes (the node temperatures),
 * its lambda zero there; those entries of a given start are ignored.
 * ------------------------------------------------------------------------ */
enum { NMPC_MODEL_HEAT = 0, NMPC_MODEL_PLATE = 1, NMPC_MODEL_WAVE = 2 };
enum { NMPC_BC_DIRICHLET = 0, NMPC_BC_NEUMANN = 1 };

typedef struct nmpc_model_problem {
    int32_t model;        /* NMPC_MODEL_* */
    int32_t boundary;     /* NMPC_BC_* */
    int32_t nsx, nsy;     /* grid nodes per axis (nsy = 1: 1D); nsx * nsy <= 4096 */
    int32_t horizon;      /* N, 1..256 */
    int32_t n_inputs;     /* m, 1..64 */
    const int32_t *act;   /* plate: [m] actuator node of each input (host, copied) */
    const double *B;      /* heat, wave: [nsx * nsy][m] row-major (host, copied) */
    double h;             /* stage length > 0 */
    double q, qv, r;      /* cost weights, r > 0 */
    double gamma;         /* regularization weight >= 0 (u~ = u^k) */
    double tau, u_lo, u_hi;   /* input box by the log barrier (tau = 0: none) */
    double u_cold;        /* inputs of the cold start (strictly inside a box) */
    double alpha, beta, rad, t_amb;   /* plate constants */
    double k0, k1, damp;  /* heat / wave constants */
} nmpc_model_problem;

typedef struct nmpc_model nmpc_model;

/* Create for up to max_batch instances on the current device (allocates the
 * device workspace). opt: tol, max_iter, n_sweep, n_schur, upper, residual
 * are used; precision must be NMPC_FP64 and omega 1 (NMPC_E_UNSUPPORTED
 * otherwise); NULL takes nmpc_default_options. Errors: NMPC_E_ARG for invalid
 * data, NMPC_E_UNSUPPORTED beyond the engine's sizes, NMPC_E_OOM/DEVICE. */
int nmpc_model_create(const nmpc_model_problem *prob, const nmpc_options *opt, int32_t max_batch,
                      nmpc_model **out);
int nmpc_model_set_options(nmpc_model *hd, const nmpc_options *opt);

/* Solve count <= max_batch instances (DEVICE buffers as above). warm_*: all
 * NULL (cold start x_i = x0, u_i = u_cold, lambda_i = 0) or all given; given
 * inputs are clipped strictly inside a box (0.5 % of its width). Work is
 * queued on `stream` (hipStream_t) and the call returns when done; info: HOST
 * [count] or NULL (err_vs_fp64 = 0: FP64 sweeps). Returns NMPC_OK if every
 * instance converged, else the first failing instance's status. */
int nmpc_model_solve_batch(nmpc_model *hd, int32_t count, const double *x0, const double *xref,
                           const double *warm_x, const double *warm_u, const double *warm_lam,
                           double *out_x, double *out_u, double *out_lam, nmpc_info *info,
                           void *stream);

/* KKT residual norms of given trajectories (DEVICE, layouts as above; the
 * trajectory is evaluated as given). r_scaled, r_paper: HOST [count]. */
int nmpc_model_residual_batch(nmpc_model *hd, int32_t count, const double *x0, const double *xref,
                              const double *x, const double *u, const double *lam,
                              double *r_scaled, double *r_paper, void *stream);

/* Kernel timing (HIP events around each solve's launch): GPU milliseconds,
 * launches, and stage visits run (each reads a stage's s_i, writes its new
 * value). */
int nmpc_model_timing_enable(nmpc_model *hd, int32_t enable);
int nmpc_model_timing_read(const nmpc_model *hd, double *kernel_ms, int64_t *launches,
                           int64_t *units);

/* Release the handle. NULL is ignored. */
void nmpc_model_destroy(nmpc_model *hd);

#ifdef __cplusplus
}
#endif

#endif /* NMPC_H */
