/*
 * spd.h -- C ABI of libspd: mixed-precision Cholesky with iterative
 * refinement for dense symmetric positive-definite systems on MI355X (gfx950).
 *
 * The problem is the paper's Eq. (1)-(2) (Klavik, Malossi, Bekas, Curioni,
 * "Changing Computing Paradigms Towards Power Efficiency", Section 3):
 *     A X = B,  A in R^{n x n} symmetric positive definite,  B, X in R^{n x m}.
 * The method is its Algorithm 1 (Section 3.1): factor A ~ R^T R once in low
 * precision, solve with the factor, then repeat { residual r = b - A x in
 * binary64; correction z from the low-precision factor; x += z } until x is
 * accurate to binary64 level.  This library stores L = R^T (lower triangular).
 *
 * Memory and ownership
 *   - Every matrix argument is binary64 (double), COLUMN-MAJOR, in DEVICE
 *     memory owned by the caller: element (i, j) of A is A[i + j*lda].
 *   - Only the lower triangle (i >= j) of A is read; A is never written.
 *   - A factor handle (spd_factor_t) owns every device buffer it allocates
 *     (the low-precision factor, the equilibration vector, workspace); the
 *     caller releases it with spd_factor_destroy.
 *   - `hip_stream` is a hipStream_t (NULL = the null stream).  Work is ordered
 *     on that stream; the library may fork internal streams of default
 *     priority and always joins them back before returning.
 *
 * Errors
 *   - Nothing throws across this ABI.  Argument errors are reported before
 *     any device work (SPD_ERR_INVALID_ARG).  HIP runtime failures map to
 *     SPD_ERR_DEVICE / SPD_ERR_OUT_OF_MEMORY.  spd_status_str() names a code.
 *   - `info` follows LAPACK: 0 on success, else the 1-based column at which
 *     the Cholesky radicand was not positive (A not SPD to the working
 *     precision).
 */
#ifndef SPD_H
#define SPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPD_OK = 0,
    SPD_ERR_INVALID_ARG = 1,
    SPD_ERR_NOT_SPD = 2,          /* a non-positive pivot; see `info` */
    SPD_ERR_NO_CONVERGENCE = 3,   /* refinement diverged or ran out of iterations */
    SPD_ERR_DEVICE = 4,
    SPD_ERR_OUT_OF_MEMORY = 5,
    SPD_ERR_UNSUPPORTED = 6
} spd_status;

/* Precision of the factorisation (the "low precision" of Algorithm 1).
 * BF16/FP16: after symmetric diagonal equilibration (and, for FP16, a
 * power-of-two scale mu), each solved panel is rounded to nearest even in that
 * format and the trailing update multiplies those operands with binary32
 * accumulation; the diagonal blocks, panel solves and the stored factor stay
 * binary32, and so do the triangular solves.  FP32: binary32 throughout.
 * FP64: plain binary64 Cholesky (the baseline and the last fallback).  AUTO:
 * chosen per system by the library (batched entry point). */
typedef enum { SPD_BF16 = 0, SPD_FP16 = 1, SPD_FP32 = 2, SPD_FP64 = 3, SPD_AUTO = 4 } spd_prec;

/* Options; passing NULL means the defaults shown. */
typedef struct {
    double tol;          /* required backward error: eta <= tol (1e-14) */
    int32_t max_iter;    /* maximum number of corrections (10); none left: no convergence */
    int32_t fallback;    /* on breakdown/divergence retry BF16/FP16 -> FP32 -> FP64 (1) */
    int32_t equilibrate; /* scale by D = diag(a_ii)^{-1/2} before rounding (1) */
    double theta;        /* FP16 headroom: mu = largest 2^k <= theta * 65504 (0.1) */
} spd_opts;

/* Outcome of a refinement (host memory).  iters_low counts low-precision
 * solves including the first one; iters_high counts binary64 residuals, both
 * for the precision finally used; eta is the final max backward error
 * max_c ||b_c - A x_c||_inf / (||A||_inf ||x_c||_inf + ||b_c||_inf). */
typedef struct {
    int32_t status;
    int32_t prec_used;
    int32_t iters_low;
    int32_t iters_high;
    int32_t fallbacks;
    int64_t info;
    double eta;
} spd_report;

typedef struct spd_factor_s *spd_factor_t;

/* Fill *o with the defaults. */
void spd_opts_default(spd_opts *o);

/* Algorithm 1's low-precision Cholesky factorisation of the lower
 * triangle of A (n x n, leading dimension lda >= max(1, n)) at precision
 * `prec` (BF16, FP16, FP32 or FP64).  If *F is NULL a new handle is created;
 * a non-NULL *F from an earlier call is reused (its buffers are kept when they
 * are large enough).  On return *info is 0 or the 1-based failing column, and
 * the status is SPD_OK or SPD_ERR_NOT_SPD (the handle stays valid either way).
 * Synchronises `hip_stream` once, to read the breakdown flag. */
spd_status spd_factor(const double *A, int64_t n, int64_t lda, spd_prec prec,
                      const spd_opts *o, void *hip_stream, spd_factor_t *F, int64_t *info);

/* A factor supplied by the caller in place of the factorisation (the perturbed-factor
 * experiment of Section 3.1, Fig. 3(b): a binary64 factor R = L^T perturbed
 * by E, then refined with Eq. (4) deciding convergence).  L: n x n,
 * column-major, leading dimension ldl >= max(1, n), device memory owned by
 * the caller; only its lower triangle is read, and only during the call.
 * prec is SPD_FP32 (L rounded once to binary32) or SPD_FP64 (used as is);
 * no equilibration or scaling (D = I, mu = 1), so spd_solve applies
 * (L L^T)^{-1} and spd_refine refines against any A given to it (with
 * fallback enabled, a binary32 import that does not converge re-factors
 * that A in binary64).  *F as in spd_factor.  On return *info is 0 or the
 * 1-based index of the first diagonal entry of L that is not positive and
 * finite, with status SPD_ERR_NOT_SPD (the handle stays valid).  Other
 * precisions, n < 0, ldl < n or a NULL L (n > 0) give SPD_ERR_INVALID_ARG
 * before any device work.  Synchronises `hip_stream` once. */
spd_status spd_factor_import(const double *L, int64_t n, int64_t ldl, spd_prec prec, void *hip_stream,
                             spd_factor_t *F, int64_t *info);

/* Algorithm 1's first solve: X = L^{-T} L^{-1} B with the handle's low-precision
 * factor (binary32 substitution), including the equilibration scaling:
 * X = s mu D L^{-T} L^{-1} round32(D B / s), s a power of two per column.
 * B (n x nrhs, ldb >= n) is read; X (n x nrhs, ldx >= n) is written; X may
 * equal B.  Asynchronous on `hip_stream`: a wait of the solve that gave up
 * cannot be reported here; the next spd_refine on the handle reports it. */
spd_status spd_solve(spd_factor_t F, const double *B, int64_t ldb, int64_t nrhs,
                     double *X, int64_t ldx, void *hip_stream);

/* Algorithm 1's refinement loop: starting from the iterate in X (counted as one
 * low-precision solve), repeat
 * { R = B - A X (binary64); eta; Z = low-precision solve of R; X += Z }
 * until every column is accurate to binary64 level (the loop's test read
 * so).  Per column, with zeta_k = ||z_k||_inf / ||x_{k+1}||_inf the size
 * of correction k, rho_k = zeta_k / zeta_{k-1} its observed contraction and
 * eta_k the backward error of the residual it was solved from, a column is
 * done when eta <= o->tol and one of: eta = 0 or zeta_k <= 2^-53;
 * rho_k < 1/2 and rho_k/(1 - rho_k) eta_k <= 2^-53 (the error left is below
 * what binary64 residuals resolve); rho_k >= 1/2 and eta_k <= 2^-51 (no
 * contraction left from a rounding-level residual).  A binary64 factor made
 * by spd_factor is backward stable: its first solve is accepted at
 * eta <= tol.  So SPD_OK means eta <= tol and x at the accuracy binary64
 * residuals allow, not eta <= tol alone.  Divergence (eta not finite, above
 * the first eta, or two steps in a row above 0.9 of the previous eta in every
 * column, while above tol) or max_iter corrections without success end it
 * with SPD_ERR_NO_CONVERGENCE.  With o->fallback set, breakdown or
 * non-convergence re-factors A at the next precision (BF16/FP16 -> FP32 ->
 * FP64; F then holds that precision) and restarts from X = solve(B).  A must
 * be the matrix F was built from.  Synchronises `hip_stream` once per
 * iteration (to read the norms); *rep (host) is filled and rep->status
 * equals the returned status.  A triangular-solve wait of this handle that
 * gave up (see spd_factor_set_wait_limit), here or in an earlier spd_solve,
 * is reported as SPD_ERR_DEVICE; the flag is cleared by the next
 * spd_factor / spd_factor_import on the handle. */
spd_status spd_refine(spd_factor_t F, const double *A, int64_t lda, const double *B, int64_t ldb,
                      int64_t nrhs, double *X, int64_t ldx, const spd_opts *o,
                      spd_report *rep, void *hip_stream);

/* The substitutions' work items wait for one another through counters in
 * device memory, each wait bounded: a wait that is not satisfied within
 * `seconds` (default 1) gives up, makes every other wait of the solve give
 * up too, and marks the handle (spd_refine then returns SPD_ERR_DEVICE; the
 * solution is not usable).  0 gives up at the first unsatisfied poll -- for
 * tests of that error path.  seconds < 0 or F NULL: SPD_ERR_INVALID_ARG. */
spd_status spd_factor_set_wait_limit(spd_factor_t F, double seconds);

/* Autotuner of the factorisation's schedule (the order of the work, never
 * its result): panels per trailing-update group, a cap on the group
 * update's workgroups (leaving compute units to the panel chain) and, for
 * binary32, the tile size (64 or 128 rows) of a group's thin trailing
 * updates, chosen by
 * timing spd_factor on a diagonally dominant test matrix of order n rounded
 * to a power of two (log scale), for precision `prec`.  The choice is kept
 * per (device architecture, HIP runtime version, precision, rounded order)
 * for the process, and in the JSON file named by the environment variable
 * SPD_TUNE_CACHE when it is set (read on first use, rewritten on each new
 * entry); every later spd_factor of that precision and size uses it unless
 * SPD_GROUP / SPD_GROUP_HALF / SPD_UPD_SLOTS / SPD_SMALL_MAIN fix the
 * schedule.  A choice
 * already held is returned without timing (from_cache 1: this process, 2:
 * read from the file).  The batched solver's grid choice per batch size is
 * kept the same way.  Allocates an n x n binary64 test matrix and a factor
 * while timing; synchronises `hip_stream`.  n outside 1..2^20, an invalid
 * precision or out NULL: SPD_ERR_INVALID_ARG. */
typedef struct {
    int32_t group;       /* 128-wide panels per trailing-update group */
    int32_t upd_slots;   /* cap on the group update's workgroups (0: one per tile) */
    double ms;           /* factorisation time of the test matrix under that schedule */
    int32_t from_cache;  /* 0 timed now, 1 held by this process, 2 read from SPD_TUNE_CACHE */
    int64_t n;           /* the rounded order the choice is kept for */
    int32_t small_tiles; /* 1: a group's thin trailing updates on 64-row tiles (binary32) */
} spd_tune_result;
spd_status spd_autotune(int64_t n, spd_prec prec, void *hip_stream, spd_tune_result *out);
/* Forget the autotuner's in-memory choices (the next use reads SPD_TUNE_CACHE again). */
void spd_autotune_clear(void);

/* The whole of Algorithm 1 in one call: spd_factor + spd_solve + spd_refine,
 * with the fallback chain applied from the factorisation on.  *F as in
 * spd_factor (reused if non-NULL).  The factorisation's breakdown check is
 * read back with the first residual rather than on its own, so the host
 * does not wait between the three steps; a breakdown still restarts at the
 * next precision (or returns SPD_ERR_NOT_SPD with rep->info) exactly as
 * spd_factor's check would.  Arguments are checked before any device work. */
spd_status spd_posv(const double *A, int64_t n, int64_t lda, const double *B, int64_t ldb,
                    int64_t nrhs, double *X, int64_t ldx, spd_prec prec, const spd_opts *o,
                    spd_report *rep, void *hip_stream, spd_factor_t *F);

/* Algorithm 1's binary64 residual on its own: R = B - A X in binary64 for the
 * symmetric A (lower triangle read; n x n, lda >= n), X and B n x nrhs.
 * R (device, ldr >= n) receives the residual unless NULL; eta (HOST array of
 * nrhs, or NULL) receives the normwise backward errors
 * ||r_c||_inf / (||A||_inf ||x_c||_inf + ||b_c||_inf).  Allocates its own
 * scratch; synchronises `hip_stream` when eta is requested. */
spd_status spd_residual(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx, const double *B,
                        int64_t ldb, int64_t nrhs, double *R, int64_t ldr, double *eta, void *hip_stream);

/* spd_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and rounding as spd_residual (R bit for bit, eta
 * to the last bit), but it calls no allocator.  Its partial sums, norms, eta
 * and (R NULL) the residual live in one static device array of
 * SPD_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; a call
 * whose parts need more is rejected with SPD_ERR_INVALID_ARG before any
 * device work (n = 16384 fits with 1 or 2 right-hand sides; with 3 or more,
 * any n up to about 60 of them).  With eta NULL the call is asynchronous on
 * `hip_stream` (capturable); with eta (host) it synchronises to read it.
 * Every call on one GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams, other threads, graph replays) race and give wrong
 * results -- the caller orders them. */
#define SPD_NOALLOC_SCRATCH_BYTES (128u << 20)
spd_status spd_residual_noalloc(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx,
                                const double *B, int64_t ldb, int64_t nrhs, double *R, int64_t ldr,
                                double *eta, void *hip_stream);

/* Limits of the batched entry point (per system). */
#define SPD_BATCH_NMAX 512
#define SPD_BATCH_MAXRHS 8

/* Many independent systems (Eq. (2) per system), each taken through all of
 * Algorithm 1 (with the fallback chain) in one persistent launch, one
 * workgroup per system, largest systems first.  Device arrays of length
 * `batch`: n[s] (0..SPD_BATCH_NMAX), nrhs[s] (0..SPD_BATCH_MAXRHS),
 * a_off[s] (offset of system s's matrix in A, in elements; column-major,
 * leading dimension n[s], lower triangle read), b_off[s] (offset of its
 * right-hand sides in B and of its solution in X; leading dimension n[s]);
 * prec[s] is the requested precision on input (AUTO: FP32) and the one used
 * on output; reps[s] (device memory) receives each system's report, with
 * SPD_ERR_INVALID_ARG for a system outside the limits.
 * The first call for a given batch size allocates the workspace (about 4.4 MB
 * per workgroup of the persistent grid), picks the launch shape by timing the
 * candidates on this very batch (the results are those of the last, chosen,
 * run) and synchronises the stream.  Later calls with the same batch size
 * allocate nothing and never synchronise the host, so they can be captured in
 * a graph; under capture without such a first call the status is
 * SPD_ERR_UNSUPPORTED.  Per-system outcomes are only in reps (the returned
 * status covers the arguments and the launch).  Each system's refinement
 * stops by the rule of spd_refine.  Every call on a device shares one
 * workspace: a call on a stream other than the previous call's first makes
 * its stream wait for that call's launch, so direct calls on different
 * streams are ordered by the library.  Graph replays are not: a captured
 * call must not run concurrently with any other batched call on the device
 * (the caller orders them). */
spd_status spd_solve_batched(int64_t batch, const int32_t *n, const int32_t *nrhs,
                             const int64_t *a_off, const double *A, const int64_t *b_off,
                             const double *B, double *X, spd_prec *prec, const spd_opts *o,
                             spd_report *reps, void *hip_stream);

/* spd_solve_batched that also writes ticks[s] (device, int64): the
 * wall-clock ticks (100 MHz) that system s took, from its first step
 * (including the picker for SPD_AUTO) to its report. */
spd_status spd_solve_batched_timed(int64_t batch, const int32_t *n, const int32_t *nrhs,
                                   const int64_t *a_off, const double *A, const int64_t *b_off,
                                   const double *B, double *X, spd_prec *prec, const spd_opts *o,
                                   spd_report *reps, int64_t *ticks, void *hip_stream);

/* ---- Learned precision picker (not in the paper: it chooses the precision
 * Algorithm 1 runs in, per system, for SPD_AUTO in the batched solver; FP64
 * stays the fallback).  A perceptron 16 -> 64 -> 64 -> 4 (ReLU, softmax over
 * BF16, FP16, FP32, FP64), binary32 parameters as one flat vector of
 * SPD_PICKER_NPARAM: W1 (64 x 16), b1 (64), W2 (64 x 64), b2 (64), W3 (4 x 64),
 * b3 (4), matrices row-major [out][in].  Features (16 per system, binary64
 * arithmetic, stored binary32), with d_i = a_ii^{-1/2} (1 where a_ii <= 0),
 * H = D A D, r_i = sum_{j != i} |h_ij| and theta the Ritz values of four
 * Lanczos steps on H from (1, ..., 1)/sqrt(n) (no reorthogonalisation; stop
 * when beta <= 1e-12 max(|alpha|, 1)):
 *   log2(n)/9, m/8, spread, mean and std of log10 a_ii (/6, /6, /3),
 *   log10(1 + max r)/3, log10(1 + mean r)/3, share of rows with r < 1,
 *   clip(1 - max r, -10, 1)/10, log10 theta_max/3, log10 max(theta_min, 1e-16)/6,
 *   log10(theta_max / max(theta_min, 1e-16))/6, max off-diagonal |h|,
 *   log10(||H||_F / sqrt(n))/3, last beta / theta_max (0 after an early stop),
 *   (theta_2 - theta_1)/(theta_max - theta_1) (0 with fewer than 3 values). */
#define SPD_PICKER_NFEAT 16
#define SPD_PICKER_NPARAM 5508

/* Parameters (device pointer, copied) used by SPD_AUTO from now on on the
 * current device; NULL switches the picker off (AUTO then means FP32). */
spd_status spd_picker_set(const float *params, void *hip_stream);

/* Features of every system of a packed batch (layout as spd_solve_batched):
 * feat (device) receives batch x 16 floats, row-major; systems outside
 * 1 <= n <= SPD_BATCH_NMAX get zeros. */
spd_status spd_picker_features(int64_t batch, const int32_t *n, const int32_t *nrhs,
                               const int64_t *a_off, const double *A, float *feat, void *hip_stream);

/* Logits (device, N x 4) of the perceptron for samples X (device, N x 16). */
spd_status spd_mlp_forward(const float *params, const float *X, int64_t N, float *logits,
                           void *hip_stream);

/* Gradient (device, SPD_PICKER_NPARAM) of the mean softmax cross-entropy
 * over the N samples with labels y (device, int32 in 0..3), and the loss
 * (device scalar, or NULL).  Sums over samples in a fixed order.  Allocates
 * (and synchronises) when N grows past the largest N seen. */
spd_status spd_mlp_grad(const float *params, const float *X, const int32_t *y, int64_t N,
                        float *grad, float *loss, void *hip_stream);

/* One Adam step (step >= 1; bias-corrected moments m, v, updated in place). */
spd_status spd_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                        int32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* Launch shape the batched solver chose for this batch size on the current
 * device (workgroups of the persistent grid, timed among 256, 512, 768 and
 * 1024 on the first call; waves per workgroup, always 4: the kernels are
 * built for that size); SPD_ERR_INVALID_ARG if no call with that batch size
 * has been made yet. */
spd_status spd_batched_config(int64_t batch, int32_t *grid, int32_t *waves);

/* Release every device buffer the handle owns.  NULL is ignored. */
void spd_factor_destroy(spd_factor_t F);

/* Introspection of a handle: n, the precision held, the panel width. */
spd_status spd_factor_query(spd_factor_t F, int64_t *n, int32_t *prec, int32_t *nb);

/* Copy the handle's factor out for inspection: Lout (device, binary64, n x n,
 * ldl >= n) receives L of H = mu D A D ~ L L^T (zeros above the diagonal),
 * dout (device, n) receives D's diagonal, *mu (host) the scale.  Any output
 * pointer may be NULL.  Stream-ordered on `hip_stream`. */
spd_status spd_factor_export(spd_factor_t F, double *Lout, int64_t ldl, double *dout,
                             double *mu, void *hip_stream);

/* ---- Algorithm 2 (Section 3.2): conjugate gradients with iterative
 * refinement, on a dense or banded binary32 copy A~ of A (the banded
 * approximation of Section 4: entries with |i - j| > half_band dropped).
 *
 * One outer step forms r = b - A x and each column's backward error eta in
 * binary64 (as in Algorithm 1); a column is finished by spd_refine's
 * stopping rule, with the change of x over its last inner phase as the
 * correction (the entry x_0 counts as a first solve, so even an accurate
 * x_0 takes one confirming phase).  The others run CG on A~ from the current x: z = A~ p in binary32 (p rounded to
 * binary32, binary32 products and sums), and alpha = r^T r / p^T z,
 * x += alpha p, r -= alpha z, beta = r'^T r' / r^T r, p = r + beta p all in
 * binary64 (beta in the standard conjugate-direction form), until
 * ||r||_2 <= inner_tol * ||r_0||_2 or max_inner products.  Columns advance in
 * lockstep (a column that has stopped waits unchanged).  The outer steps
 * repeat until every column is finished (SPD_OK) or eta is not finite, rises
 * above its first value, or fails to fall below 0.9 of its previous value at
 * two residuals in a row (Eq. (4) does not hold for A~), or after max_outer
 * inner phases (SPD_ERR_NO_CONVERGENCE).  The report's iters_low counts
 * products with A~ (the sum over phases of the longest column's count),
 * iters_high the binary64 residuals, prec_used is SPD_FP32, eta the largest
 * final backward error. */
typedef struct {
    double tol;        /* required backward error: eta <= tol (1e-14) */
    double inner_tol;  /* inner stop: ||r||_2 <= inner_tol ||r_0||_2 (1e-6) */
    int32_t max_outer; /* inner phases at most (30) */
    int32_t max_inner; /* products per phase at most (2000) */
} spd_cg_opts;

typedef struct spd_cg_s *spd_cg_t;

void spd_cg_opts_default(spd_cg_opts *o);

/* Builds A~ from the lower triangle of A (n x n, leading dimension
 * lda >= max(1, n), device memory; A is not kept).  half_band < 0 or
 * >= n - 1: dense A~ (about 4 n^2 bytes of device memory); otherwise band
 * storage of (2 half_band + 1) n binary32 values (half_band <= 4096, else
 * SPD_ERR_UNSUPPORTED).  *H NULL creates a handle; a handle from an earlier
 * call is rebuilt.  Asynchronous on hip_stream.  The handle owns its device
 * memory; release it with spd_cg_destroy. */
spd_status spd_cg_prepare(const double *A, int64_t n, int64_t lda, int64_t half_band, void *hip_stream,
                          spd_cg_t *H);

/* Refines X (n x nrhs, ldx, nrhs <= 65535; device memory; its entry value
 * is x_0, e.g. zero) for A X = B with the handle's A~; A must be the matrix the handle
 * was built from (binary64 residuals).  o NULL: defaults.  Synchronises
 * hip_stream once per outer step and once per few inner iterations (the
 * stopping tests).  Returns rep->status. */
spd_status spd_cg_refine(spd_cg_t H, const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrhs,
                         double *X, int64_t ldx, const spd_cg_opts *o, spd_report *rep, void *hip_stream);

/* Releases the handle (waits for the device first).  NULL is ignored. */
void spd_cg_destroy(spd_cg_t H);

/* Kernel timing for measurement tools.  While enabled, the library brackets
 * every launch of the kernel classes below with HIP events recorded on the
 * stream that launch uses, and tallies the algorithmic work of each launch:
 *   SPD_K_UPDATE   trailing update H_ij -= L_ik L_jk^T (flops of the lower
 *                  triangle, bytes = tiles of H read and written once plus
 *                  their two panel operands)
 *   SPD_K_RESIDUAL binary64 residual (2 n^2 m flops; bytes = the lower
 *                  triangle of A plus X, B and R)
 *   SPD_K_CG_MV    CG product z = A~ p (2 n^2 m flops dense, 2 (2k + 1) n m
 *                  banded; bytes = A~ once (4 n^2, or 4 (2k + 1) n) plus
 *                  the binary32 and binary64 directions read and z written,
 *                  20 n m)
 *   SPD_K_UPDATE is a group's trailing update (the factorisation's bulk);
 *   SPD_K_CHAIN_UPDATE the panel chain's update of one panel's columns by the
 *                  group's earlier panels (same flop/byte accounting)
 *   SPD_K_TRSV     one pair of triangular solves L L^T (both directions;
 *                  flops 2 n^2 m, bytes = the factor's lower triangle read
 *                  once per direction plus the vectors)
 *   SPD_K_CONVERT  equilibrate/convert A -> H (bytes = A's lower triangle read
 *                  in binary64 and H's written in the factor type)
 * spd_profile_query synchronises on the recorded events, folds them into the
 * totals and returns launches, summed milliseconds, flops and bytes.  Not
 * thread-safe against concurrent factorisations; meant for benchmarks. */
enum { SPD_K_UPDATE = 0, SPD_K_RESIDUAL = 1, SPD_K_CG_MV = 2, SPD_K_CHAIN_UPDATE = 3, SPD_K_TRSV = 4,
       SPD_K_CONVERT = 5, SPD_K_COUNT = 6 };
void spd_profile_enable(int on);
void spd_profile_reset(void);
spd_status spd_profile_query(int kernel, int64_t *launches, double *total_ms, double *total_flops,
                             double *total_bytes);

/* Human-readable name of a status code (static string). */
const char *spd_status_str(spd_status s);

/* Library version string (static). */
const char *spd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPD_H */
