/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct CPU
 * reference for the SPD solve of the paper (Klavik, Malossi, Bekas, Curioni,
 * "Changing Computing Paradigms Towards Power Efficiency", Section 3.1).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or constant with the GPU
 * library; both are fed from the seeded generators in spdgen/.
 *
 * Conventions: every matrix is column-major (element (i,j) at p[i + j*ld]),
 * indices are 0-based inside the code, `info` is 1-based like LAPACK.  A is
 * symmetric and only its lower triangle (i >= j) is ever read.
 *
 * Contents
 *   oracle_potrf     Cholesky A = L L^T (Section 3.1: A = R^T R with R = L^T)
 *   oracle_fsub      forward substitution  L Y = B   (first half of Eq. (3))
 *   oracle_bsub      back substitution   L^T X = Y   (second half of Eq. (3))
 *   oracle_residual  R = B - A X in binary64 (Algorithm 1, residual step);
 *                    _rows / _given_rows: of listed rows only
 *   oracle_norm1_sym / oracle_backward_error  norms and eta
 *   oracle_rne_f16 / oracle_rne_bf16  binary32 -> binary16 / bfloat16 rounding
 *                    to nearest even, from the formats' definitions
 *   oracle_lowprec_factor  Algorithm 1's low-precision factorisation with its
 *                    scaling (d, mu) on its own, for pins
 *   oracle_ir        Algorithm 1 emulated step by step with a low-precision
 *                    factor (binary32, or binary16/bfloat16 operands with
 *                    binary32 accumulation) and binary64 residual/update.
 *   oracle_ir_factor Algorithm 1 after its factorisation, with a given factor
 *                    (the perturbed-factor experiment, Fig. 3(b)).
 *   oracle_cg_ir     Algorithm 2 (conjugate gradients with the matrix-vector
 *                    product in binary32 on a dense or banded copy of A,
 *                    everything else in binary64), restarted from a binary64
 *                    residual until the backward error reaches the tolerance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------ */
/* Cholesky factorisation A = L L^T, L lower with positive diagonal.
 * Definition (Section 3.1; Golub & Van Loan's outer-product form):
 *   for j = 0..n-1:
 *     L_jj = sqrt(a_jj - sum_{k<j} L_jk^2)       (fail if radicand <= 0)
 *     L_ij = (a_ij - sum_{k<j} L_ik L_jk) / L_jj  for i > j
 * Written right-looking: after column j is final, its outer product is
 * subtracted from the trailing lower triangle.  Returns 0, or the 1-based
 * column whose radicand is not positive (L is then partially written).
 * L may alias A only if ldl == lda and L == A. */
int64_t oracle_potrf(int64_t n, const double *A, int64_t lda, double *L, int64_t ldl)
{
    if (L != A)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                L[IDX(i, j, ldl)] = (i >= j) ? A[IDX(i, j, lda)] : 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double piv = L[IDX(j, j, ldl)];
        if (!(piv > 0.0)) /* also catches NaN */
            return j + 1;
        double ljj = sqrt(piv);
        L[IDX(j, j, ldl)] = ljj;
        for (int64_t i = j + 1; i < n; ++i)
            L[IDX(i, j, ldl)] /= ljj;
        /* trailing update  a_ik -= L_ij L_kj  for j < k <= i */
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = j + 1; k < n; ++k) {
            double lkj = L[IDX(k, j, ldl)];
            for (int64_t i = k; i < n; ++i)
                L[IDX(i, k, ldl)] -= L[IDX(i, j, ldl)] * lkj;
        }
    }
    return 0;
}

/* Forward substitution, in place: Y <- L^{-1} Y for m columns (Eq. (3)). */
void oracle_fsub(int64_t n, int64_t m, const double *L, int64_t ldl, double *Y, int64_t ldy)
{
    for (int64_t c = 0; c < m; ++c) {
        double *y = Y + (size_t)c * (size_t)ldy;
        for (int64_t j = 0; j < n; ++j) {
            y[j] /= L[IDX(j, j, ldl)];
            double yj = y[j];
            for (int64_t i = j + 1; i < n; ++i)
                y[i] -= L[IDX(i, j, ldl)] * yj;
        }
    }
}

/* Back substitution, in place: Y <- L^{-T} Y for m columns (Eq. (3)). */
void oracle_bsub(int64_t n, int64_t m, const double *L, int64_t ldl, double *Y, int64_t ldy)
{
    for (int64_t c = 0; c < m; ++c) {
        double *y = Y + (size_t)c * (size_t)ldy;
        for (int64_t j = n - 1; j >= 0; --j) {
            double s = y[j];
            for (int64_t i = j + 1; i < n; ++i)
                s -= L[IDX(i, j, ldl)] * y[i];
            y[j] = s / L[IDX(j, j, ldl)];
        }
    }
}

/* Full solve X = L^{-T} L^{-1} B (Eq. (3)); X may alias B. */
void oracle_potrs(int64_t n, int64_t m, const double *L, int64_t ldl,
                  const double *B, int64_t ldb, double *X, int64_t ldx)
{
    if (X != B)
        for (int64_t c = 0; c < m; ++c)
            memcpy(X + (size_t)c * ldx, B + (size_t)c * ldb, (size_t)n * sizeof(double));
    oracle_fsub(n, m, L, ldl, X, ldx);
    oracle_bsub(n, m, L, ldl, X, ldx);
}

/* Symmetric element a_ij read from the lower triangle. */
static inline double sym(const double *A, int64_t lda, int64_t i, int64_t j)
{
    return (i >= j) ? A[IDX(i, j, lda)] : A[IDX(j, i, lda)];
}

/* R = B - A X in binary64, A symmetric (lower triangle read).  Each residual
 * entry is the plain sum b_i - sum_j a_ij x_j taken in index order. */
void oracle_residual(int64_t n, int64_t m, const double *A, int64_t lda,
                     const double *X, int64_t ldx, const double *B, int64_t ldb,
                     double *R, int64_t ldr)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < n; ++i) {
            const double *x = X + (size_t)c * ldx;
            double s = B[IDX(i, c, ldb)];
            for (int64_t j = 0; j < n; ++j)
                s -= sym(A, lda, i, j) * x[j];
            R[IDX(i, c, ldr)] = s;
        }
}

/* Residual of a subset of rows (used on large systems, where a full residual
 * is too slow for a spot check): R[k, c] for the rows listed in `rows`. */
void oracle_residual_rows(int64_t n, int64_t m, const double *A, int64_t lda,
                          const double *X, int64_t ldx, const double *B, int64_t ldb,
                          int64_t nrows, const int64_t *rows, double *R /* nrows x m */)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t c = 0; c < m; ++c)
        for (int64_t k = 0; k < nrows; ++k) {
            int64_t i = rows[k];
            const double *x = X + (size_t)c * ldx;
            double s = B[IDX(i, c, ldb)];
            for (int64_t j = 0; j < n; ++j)
                s -= sym(A, lda, i, j) * x[j];
            R[IDX(k, c, nrows)] = s;
        }
}

/* The same residual of listed rows when only those rows of the symmetric A
 * are at hand (systems too large to copy whole to the host): Arows is
 * nrows x n, row k holding a_{rows[k], j} for j = 0..n-1, leading dimension
 * ldr (column-major: element (k, j) at Arows[k + j*ldr]). */
void oracle_residual_given_rows(int64_t n, int64_t m, const double *Arows, int64_t ldr,
                                const double *X, int64_t ldx, const double *B, int64_t ldb,
                                int64_t nrows, const int64_t *rows, double *R /* nrows x m */)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t c = 0; c < m; ++c)
        for (int64_t k = 0; k < nrows; ++k) {
            const double *x = X + (size_t)c * ldx;
            double s = B[IDX(rows[k], c, ldb)];
            for (int64_t j = 0; j < n; ++j)
                s -= Arows[IDX(k, j, ldr)] * x[j];
            R[IDX(k, c, nrows)] = s;
        }
}

/* ||A||_inf = max_i sum_j |a_ij| (= ||A||_1 for symmetric A). */
double oracle_norminf_sym(int64_t n, const double *A, int64_t lda)
{
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s += fabs(sym(A, lda, i, j));
        if (!(s <= best)) /* propagate NaN */
            best = s;
    }
    return best;
}

static double vec_maxabs(int64_t n, const double *v)
{
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (!(a <= best))
            best = a;
    }
    return best;
}

/* Normwise relative backward error per column, infinity norm:
 *   eta_c = ||r_c||_inf / (||A||_inf ||x_c||_inf + ||b_c||_inf)
 * with r_c = b_c - A x_c in binary64.  (The paper's loop test uses ||r||_2
 * against an absolute tolerance; this scale-free form is the reading used to
 * define "FP64-accurate".) */
void oracle_backward_error(int64_t n, int64_t m, const double *A, int64_t lda,
                           const double *X, int64_t ldx, const double *B, int64_t ldb,
                           double *eta)
{
    double *R = (double *)malloc((size_t)n * (size_t)m * sizeof(double));
    oracle_residual(n, m, A, lda, X, ldx, B, ldb, R, n);
    double an = oracle_norminf_sym(n, A, lda);
    for (int64_t c = 0; c < m; ++c) {
        double rn = vec_maxabs(n, R + (size_t)c * n);
        double xn = vec_maxabs(n, X + (size_t)c * ldx);
        double bn = vec_maxabs(n, B + (size_t)c * ldb);
        double den = an * xn + bn;
        eta[c] = (den > 0.0) ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
        if (rn != rn)
            eta[c] = NAN;
    }
    free(R);
}

/* ------------------------------------------------------------------------ */
/* Rounding binary32 -> binary16 / bfloat16, round to nearest, ties to even,
 * written from the formats' definitions (IEEE 754-2008 binary16: 1 sign,
 * 5 exponent bits with bias 15, 10 fraction bits; bfloat16: the top 16 bits of
 * binary32).  The result is returned widened back to binary32, which is exact. */
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

float oracle_rne_f16(float x)
{
    if (x != x)
        return x;
    float a = fabsf(x);
    float sgn = signbit(x) ? -1.0f : 1.0f;
    /* largest finite binary16 is 65504; values at or above 65520 round to inf */
    if (a >= 65520.0f)
        return sgn * INFINITY;
    /* quantum (spacing) of binary16 at |x|: 2^(e-10) for normal e >= -14,
     * 2^-24 for the subnormal range */
    int e;
    frexpf(a, &e);           /* a = f * 2^e, f in [0.5, 1) -> unbiased exponent e-1 */
    int ue = e - 1;
    if (ue < -14)
        ue = -14;
    double q = ldexp(1.0, ue - 10);
    double t = (double)a / q;        /* exact: a has 24 bits, q a power of two */
    double r = nearbyint(t);         /* default rounding mode: ties to even */
    return sgn * (float)(r * q);
}

float oracle_rne_bf16(float x)
{
    uint32_t u = f2u(x);
    if ((u & 0x7fffffffu) > 0x7f800000u)    /* NaN: keep it a quiet NaN */
        return u2f((u | 0x00400000u) & 0xffff0000u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;                     /* round half to even on bit 16 */
    return u2f(u & 0xffff0000u);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Cholesky with iterative refinement), emulated.
 *
 * Precision codes: 0 = bfloat16 operands, 1 = binary16 operands,
 * 2 = binary32, 3 = binary64.  Status codes: 0 ok, 2 not SPD, 3 no convergence.
 *
 * Steps, in the paper's order, with the readings this project takes where the
 * paper is silent:
 *   scaling  D = diag(a_ii)^(-1/2) (for binary16/bfloat16/binary32 when
 *            `equil` is set), mu = largest power of two <= theta * 65504 for
 *            binary16 and 1 otherwise; H = round32(mu * D A D).
 *   factor   low-precision factor H ~ L L^T: right-looking Cholesky in binary32
 *            arithmetic; for binary16/bfloat16 every update product uses the
 *            operands rounded to that format (binary32 accumulation).
 *            binary64 factors A itself in binary64.
 *   solve    x = s mu D L^{-T} L^{-1} round32(D b / s), s a power of two
 *            normalising max |D b| (per column); binary32 substitution.
 *   residual r = b - A x in binary64; eta per column as above.
 *   test     the loop ends when every column is done: eta <= tol and the
 *            corrections show x accurate to binary64 level (the rule is
 *            stated above ir_loop).  Divergence (only while eta > tol): eta
 *            not finite, eta above the first eta, or two consecutive steps
 *            with eta_k > 0.9 eta_{k-1}.  At most `max_iter` corrections;
 *            without success by then, no convergence.
 *   correct  z from the same low-precision solve of r; x += z (binary64);
 *            new residual.
 *   fallback on breakdown or divergence: binary16/bfloat16 -> binary32 ->
 *            binary64 (if `fallback` is set).
 * Iteration counts: low = number of low-precision solves (incl. the first),
 * high = number of binary64 residuals, both for the final precision.
 */
typedef struct {
    int32_t status, prec_used, iters_low, iters_high, fallbacks;
    int64_t info;
    double eta;
} oracle_report;

static float round_op(float v, int prec)
{
    if (prec == 0) return oracle_rne_bf16(v);
    if (prec == 1) return oracle_rne_f16(v);
    return v;
}

/* binary32 Cholesky of the n x n lower triangle of H (column-major, ld n),
 * operands of every update rounded to `prec`; accumulation in binary32. */
static int64_t potrf_lowprec(int64_t n, float *H, int prec)
{
    for (int64_t j = 0; j < n; ++j) {
        float piv = H[IDX(j, j, n)];
        if (!(piv > 0.0f))
            return j + 1;
        float ljj = sqrtf(piv);
        H[IDX(j, j, n)] = ljj;
        for (int64_t i = j + 1; i < n; ++i)
            H[IDX(i, j, n)] /= ljj;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = j + 1; k < n; ++k) {
            float lkj = round_op(H[IDX(k, j, n)], prec);
            for (int64_t i = k; i < n; ++i)
                H[IDX(i, k, n)] -= round_op(H[IDX(i, j, n)], prec) * lkj;
        }
    }
    return 0;
}

static void solve_f32(int64_t n, const float *L, float *y)
{
    for (int64_t j = 0; j < n; ++j) {
        y[j] /= L[IDX(j, j, n)];
        float yj = y[j];
        for (int64_t i = j + 1; i < n; ++i)
            y[i] -= L[IDX(i, j, n)] * yj;
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        float s = y[j];
        for (int64_t i = j + 1; i < n; ++i)
            s -= L[IDX(i, j, n)] * y[i];
        y[j] = s / L[IDX(j, j, n)];
    }
}

/* When the refinement is done (Algorithm 1's while-test read as "until x is
 * accurate to binary64 level"; Eq. (4) decides whether it converges at all).
 * The backward error alone does not tell: eta <= tol, even eta at the
 * binary64 floor, is reached while x still carries error along the
 * eigenvectors of the smallest eigenvalues, which the residual hardly sees.
 * The corrections do see it.  Per column, after correction k (z_k solved
 * from the residual of x_k, whose backward error is eta_k; x_{k+1} = x_k + z_k):
 *   zeta_k = ||z_k||_inf / ||x_{k+1}||_inf   (about the relative error of x_k)
 *   rho_k  = zeta_k / zeta_{k-1}              (the observed contraction)
 * With geometric contraction the error left in x_{k+1} is about
 * rho_k/(1 - rho_k) zeta_k; the solve turned a backward error eta_k into
 * zeta_k, so residuals rounded at binary64 level (eta ~ u) limit x to about
 * (zeta_k/eta_k) u.  A column is done once eta_{k+1} <= tol and
 *   (a) eta_{k+1} = 0 or zeta_k <= u (x no longer moves), or
 *   (b) rho_k < 1/2 and rho_k/(1 - rho_k) eta_k <= u (the error left is below
 *       what binary64 residuals resolve), or
 *   (c) rho_k >= 1/2 and eta_k <= 4u (the correction came from a residual
 *       at rounding level and no longer contracts: x is as accurate as the
 *       binary64 residual allows).
 * A binary64 factor of A itself is backward stable, so its first solve is
 * accepted at eta <= tol.  The refinement succeeds when every column is done;
 * divergence (eta not finite, above its first value, or two consecutive steps
 * with eta_k > 0.9 eta_{k-1} in every column) is judged only while eta > tol;
 * after max_iter corrections without success it has not converged. */
#define U64 (0x1p-53)
#define ETA_FLOOR (0x1p-51)

/* power of two s with s/2 < v <= s (1 for v == 0 or non-finite) */
static double pow2_ceil(double v)
{
    if (!(v > 0.0) || isinf(v))
        return 1.0;
    int e;
    double f = frexp(v, &e); /* v = f 2^e, f in [0.5,1) */
    return (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

static int ir_loop(int64_t n, int64_t m, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *X, int64_t ldx, int prec, const double *d, double mu, const double *L64,
                   const float *L32, int stable, double tol, int max_iter, oracle_report *rep);

/* The low-precision factorisation with its scaling: d (equilibration, 1 for binary64 or when `equil`
 * is off), mu, and the low-precision factor -- L64 (binary64, from A itself)
 * or L32 (binary32 factor of H = round32(mu D A D), update operands rounded
 * to binary16/bfloat16 for prec 1/0).  The caller frees *L64 / *L32.
 * Returns the 1-based breakdown column, or 0. */
static int64_t lowprec_factor(int64_t n, const double *A, int64_t lda, int prec, int equil, double theta,
                              double *d, double *mu, double **L64, float **L32)
{
    size_t nn = (size_t)n * (size_t)n;
    *mu = 1.0;
    *L64 = NULL;
    *L32 = NULL;
    /* scaling (not in the paper; needed so binary16 neither overflows nor underflows) */
    for (int64_t i = 0; i < n; ++i) {
        double a = A[IDX(i, i, lda)];
        d[i] = (prec != 3 && equil && a > 0.0) ? 1.0 / sqrt(a) : 1.0;
    }
    if (prec == 1) {
        /* largest power of two <= theta * 65504 */
        int e;
        frexp(theta * 65504.0, &e);
        *mu = ldexp(1.0, e - 1);
    }
    if (prec == 3) {
        *L64 = (double *)malloc(nn * sizeof(double));
        return oracle_potrf(n, A, lda, *L64, n);
    }
    float *H = (float *)malloc(nn * sizeof(float));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            H[IDX(i, j, n)] = (i >= j) ? (float)(*mu * d[i] * A[IDX(i, j, lda)] * d[j]) : 0.0f;
    *L32 = H;
    return potrf_lowprec(n, H, prec);
}

/* The factorisation on its own, for pins: the scaling and the low-precision factor as
 * ir_attempt forms them.  L (n x n, leading dimension ldl) receives the
 * factor widened to binary64 (lower triangle; zeros above), d the
 * equilibration, *mu the scale.  Returns the 1-based breakdown column, or 0
 * (L then holds the partial factor). */
int64_t oracle_lowprec_factor(int64_t n, const double *A, int64_t lda, int32_t prec, int32_t equil,
                              double theta, double *L, int64_t ldl, double *d, double *mu)
{
    double *L64;
    float *L32;
    int64_t info = lowprec_factor(n, A, lda, prec, equil, theta, d, mu, &L64, &L32);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            L[IDX(i, j, ldl)] = (i < j) ? 0.0 : (L64 ? L64[IDX(i, j, n)] : (double)L32[IDX(i, j, n)]);
    free(L64);
    free(L32);
    return info;
}

/* One attempt of Algorithm 1 at precision `prec`.  Returns status. */
static int ir_attempt(int64_t n, int64_t m, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double *X, int64_t ldx, int prec,
                      int equil, double theta, double tol, int max_iter,
                      oracle_report *rep)
{
    double *d = (double *)malloc((size_t)n * sizeof(double));
    double *L64 = NULL;
    float *L32 = NULL;
    double mu = 1.0;
    int status = 0;
    rep->iters_low = rep->iters_high = 0;
    rep->eta = NAN;

    /* the low-precision factorisation */
    rep->info = lowprec_factor(n, A, lda, prec, equil, theta, d, &mu, &L64, &L32);
    if (rep->info) {
        status = 2;
        goto done;
    }

    status = ir_loop(n, m, A, lda, B, ldb, X, ldx, prec, d, mu, L64, L32, prec == 3, tol, max_iter, rep);
done:
    free(d); free(L64); free(L32);
    return status;
}

/* Algorithm 1 after its factorisation, with a given factor: L64 (binary64
 * solves) or L32 (binary32 solves of the scaled right-hand side),
 * D = diag(d), mu.  The first solve (from r = b) and the corrections share
 * one routine: z = s mu D L^{-T} L^{-1} round(D r / s).  `stable`: the
 * factor is the method's own binary64 factor (first solve accepted at
 * eta <= tol).
 * Returns the status. */
static int ir_loop(int64_t n, int64_t m, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *X, int64_t ldx, int prec, const double *d, double mu, const double *L64,
                   const float *L32, int stable, double tol, int max_iter, oracle_report *rep)
{
    double *R = (double *)malloc((size_t)n * (size_t)m * sizeof(double));
    double *eta = (double *)malloc((size_t)m * 4 * sizeof(double));
    double *eprev = eta + m, *zeta = eta + 2 * m, *zprev = eta + 3 * m;
    int *done = (int *)calloc((size_t)m, sizeof(int));
    float *y = (float *)malloc((size_t)n * sizeof(float));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    int status = 0;
    rep->iters_low = rep->iters_high = 0;
    rep->eta = NAN;
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < n; ++i)
            X[IDX(i, c, ldx)] = 0.0;
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < n; ++i)
            R[IDX(i, c, n)] = B[IDX(i, c, ldb)];
    int stalls = 0;
    double eta0 = 0.0;
    for (;;) {
        /* low-precision solve of the current residual, then x += z */
        for (int64_t c = 0; c < m; ++c) {
            double *r = R + (size_t)c * n;
            if (prec == 3) {
                oracle_fsub(n, 1, L64, n, r, n);
                oracle_bsub(n, 1, L64, n, r, n);
                for (int64_t i = 0; i < n; ++i)
                    z[i] = r[i];
            } else {
                double mx = 0.0;
                for (int64_t i = 0; i < n; ++i)
                    if (fabs(d[i] * r[i]) > mx) mx = fabs(d[i] * r[i]);
                double s = pow2_ceil(mx);
                for (int64_t i = 0; i < n; ++i)
                    y[i] = (float)(d[i] * r[i] / s);
                solve_f32(n, L32, y);
                for (int64_t i = 0; i < n; ++i)
                    z[i] = s * mu * d[i] * (double)y[i];
            }
            for (int64_t i = 0; i < n; ++i)
                X[IDX(i, c, ldx)] += z[i];
            double zn = vec_maxabs(n, z), xn = vec_maxabs(n, X + (size_t)c * ldx);
            zeta[c] = (zn == 0.0) ? 0.0 : zn / xn; /* xn = 0 < zn: +inf */
        }
        rep->iters_low++;
        /* binary64 residual and backward error */
        oracle_residual(n, m, A, lda, X, ldx, B, ldb, R, n);
        rep->iters_high++;
        double an = oracle_norminf_sym(n, A, lda);
        double worst = 0.0;
        int finite = 1;
        for (int64_t c = 0; c < m; ++c) {
            double rn = vec_maxabs(n, R + (size_t)c * n);
            double den = an * vec_maxabs(n, X + (size_t)c * ldx) + vec_maxabs(n, B + (size_t)c * ldb);
            eta[c] = (den > 0.0) ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
            if (!isfinite(eta[c]) || rn != rn)
                finite = 0;
            if (eta[c] > worst) worst = eta[c];
        }
        rep->eta = finite ? worst : NAN;
        if (!finite) { status = 3; break; }
        /* which columns are done (k = corrections so far) */
        const int k = rep->iters_high - 1;
        int all = 1;
        for (int64_t c = 0; c < m; ++c) {
            if (!done[c] && eta[c] <= tol) {
                if (eta[c] == 0.0 || zeta[c] <= U64)
                    done[c] = 1;
                else if (k == 0)
                    done[c] = stable;
                else {
                    double rho = zeta[c] / zprev[c];
                    done[c] = (rho < 0.5) ? (rho / (1.0 - rho)) * eprev[c] <= U64 : eprev[c] <= ETA_FLOOR;
                }
            }
            all = all && done[c];
        }
        if (all && worst <= tol) { status = 0; break; }
        if (k == 0) {
            eta0 = worst;
        } else {
            int stall = 1;
            for (int64_t c = 0; c < m; ++c)
                if (!(eta[c] > 0.9 * eprev[c])) stall = 0;
            stalls = stall ? stalls + 1 : 0;
            if (worst > tol && (worst > eta0 || stalls >= 2)) { status = 3; break; }
        }
        if (rep->iters_low > max_iter) { status = 3; break; }
        memcpy(eprev, eta, (size_t)m * sizeof(double));
        memcpy(zprev, zeta, (size_t)m * sizeof(double));
    }
    free(R); free(eta); free(done); free(y); free(z);
    return status;
}

int32_t oracle_ir(int64_t n, int64_t m, const double *A, int64_t lda,
                  const double *B, int64_t ldb, double *X, int64_t ldx,
                  int32_t prec, int32_t equil, double theta, double tol, int32_t max_iter,
                  int32_t fallback, oracle_report *rep)
{
    rep->fallbacks = 0;
    for (;;) {
        rep->prec_used = prec;
        int st = ir_attempt(n, m, A, lda, B, ldb, X, ldx, prec, equil, theta, tol, max_iter, rep);
        rep->status = st;
        if (st == 0 || !fallback || prec == 3)
            return st;
        prec = (prec < 2) ? 2 : 3;
        rep->fallbacks++;
    }
}

/* Algorithm 1 after its factorisation, with the factor it would have
 * produced replaced by a given lower-triangular L (n x n, leading dimension ldl): the
 * perturbed-factor experiment of Section 3.1 (Fig. 3(b)), where R = L^T
 * comes from a binary64 factorisation and is perturbed before use.  prec 3:
 * binary64 substitutions with L; prec 2: L rounded once to binary32 and the
 * binary32 solve of the scaled right-hand side.  No equilibration (D = I),
 * mu = 1.  rep->info = first diagonal entry of L that is not positive and
 * finite (1-based; status 2), else the refinement's status (0 converged,
 * 3 no convergence). */
int32_t oracle_ir_factor(int64_t n, int64_t m, const double *A, int64_t lda, const double *L, int64_t ldl,
                         const double *B, int64_t ldb, double *X, int64_t ldx, int32_t prec, double tol,
                         int32_t max_iter, oracle_report *rep)
{
    size_t nn = (size_t)n * (size_t)n;
    double *d = (double *)malloc((size_t)n * sizeof(double));
    double *L64 = NULL;
    float *L32 = NULL;
    int status;
    rep->fallbacks = 0;
    rep->prec_used = prec;
    rep->info = 0;
    rep->iters_low = rep->iters_high = 0;
    rep->eta = NAN;
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 1.0;
        double a = L[IDX(i, i, ldl)];
        if (!(a > 0.0) || !isfinite(a)) {
            if (!rep->info) rep->info = i + 1;
        }
    }
    if (rep->info) {
        free(d);
        rep->status = 2;
        return 2;
    }
    if (prec == 3) {
        L64 = (double *)malloc(nn * sizeof(double));
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                L64[IDX(i, j, n)] = (i >= j) ? L[IDX(i, j, ldl)] : 0.0;
    } else {
        L32 = (float *)malloc(nn * sizeof(float));
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                L32[IDX(i, j, n)] = (i >= j) ? (float)L[IDX(i, j, ldl)] : 0.0f;
    }
    status = ir_loop(n, m, A, lda, B, ldb, X, ldx, prec, d, 1.0, L64, L32, 0, tol, max_iter, rep);
    free(d); free(L64); free(L32);
    rep->status = status;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (Section 3.2): conjugate gradients with iterative refinement.
 *
 * The low-precision operator: A~ = fl32(A) on the band |i - j| <= k
 * (k = half_band; k < 0 keeps every entry: the dense variant), zero outside
 * it (Section 4's banded approximation).  One product z = A~ p rounds p to
 * binary32 and forms each z_i as a binary32 dot product taken in the order
 * j = 0, 1, ..., n-1 (binary32 products and sums), widened to binary64.
 * Every other quantity (x, r, p, rho, alpha, beta) is binary64.
 *
 * One outer step (counted in iters_high): r = b - A x in binary64 and the
 * backward error eta of each column.  A column is done by Algorithm 1's
 * stopping rule (above ir_loop): eta <= tol and the change of x over its
 * last inner phase (the correction) shows x accurate to binary64 level;
 * a start x0 counts as a first solve.
 * Otherwise CG runs on the current residual -- Algorithm 2's loop body with
 * x updated in place --
 *     p = r, rho = r^T r, stop when r^T r <= inner_tol^2 rho_0 or after
 *     max_inner products:
 *       z = A~ p;  alpha = rho / (p^T z);  x += alpha p;  r -= alpha z;
 *       rho' = r^T r;  beta = rho' / rho;  p = r + beta p;  rho = rho'
 * (beta in the standard Fletcher-Reeves form: the printed beta = r^T z / rho
 * is read as a misprint, since it does not give conjugate directions.)
 * The columns run in lockstep: one inner phase lasts as long as its longest
 * column, and iters_low counts the products of that schedule (the sum over
 * outer steps of the longest inner run).  A column's own arithmetic does not
 * depend on the others.
 *
 * After max_outer inner phases the residual is formed once more.  Status 0
 * when every column is done; 3 when eta is not finite, rises above
 * its value at the first residual, or fails to fall below 0.9 of its
 * previous value at two residuals in a row (no contraction: Eq. (4) does not
 * hold for A~), or when max_outer phases end above tol.  X holds x0 on
 * entry and the result on exit. */
static void lowmv(int64_t n, const float *At, int64_t k, const double *p, float *pf, double *z)
{
    for (int64_t j = 0; j < n; ++j)
        pf[j] = (float)p[j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t j0 = 0, j1 = n;
        if (k >= 0) {
            j0 = i - k < 0 ? 0 : i - k;
            j1 = i + k + 1 > n ? n : i + k + 1;
        }
        float s = 0.0f;
        /* At holds column i of A~ (= row i, A~ being symmetric) */
        for (int64_t j = j0; j < j1; ++j)
            s += At[IDX(j, i, n)] * pf[j];
        z[i] = (double)s;
    }
}

static double dot64(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

int32_t oracle_cg_ir(int64_t n, int64_t m, const double *A, int64_t lda, int64_t half_band,
                     const double *B, int64_t ldb, double *X, int64_t ldx, double tol, double inner_tol,
                     int32_t max_outer, int32_t max_inner, oracle_report *rep)
{
    size_t nn = (size_t)n * (size_t)n;
    float *At = (float *)malloc(nn * sizeof(float));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            int inb = half_band < 0 || (i - j <= half_band && j - i <= half_band);
            At[IDX(i, j, n)] = inb ? (float)sym(A, lda, i, j) : 0.0f;
        }
    double *R = (double *)malloc((size_t)n * (size_t)m * sizeof(double));
    double *P = (double *)malloc((size_t)n * sizeof(double));
    double *Z = (double *)malloc((size_t)n * sizeof(double));
    double *X0 = (double *)malloc((size_t)n * sizeof(double));
    float *pf = (float *)malloc((size_t)n * sizeof(float));
    double *eta = (double *)malloc((size_t)m * 5 * sizeof(double));
    double *eta1 = eta + m, *prev = eta + 2 * m, *zeta = eta + 3 * m, *zprev = eta + 4 * m;
    int *done = (int *)calloc((size_t)m, sizeof(int));
    int *stalls = (int *)calloc((size_t)m, sizeof(int));
    double an = oracle_norminf_sym(n, A, lda);
    int status = 3;
    rep->status = 0;
    rep->prec_used = 2;
    rep->fallbacks = 0;
    rep->info = 0;
    rep->iters_low = rep->iters_high = 0;
    rep->eta = NAN;
    for (int64_t c = 0; c < m; ++c)
        zeta[c] = 1.0; /* no phase before the first: x0 counts as a first solve */
    for (int outer = 0;; ++outer) {
        oracle_residual(n, m, A, lda, X, ldx, B, ldb, R, n);
        rep->iters_high++;
        double worst = 0.0;
        int bad = 0, all_done = 1;
        for (int64_t c = 0; c < m; ++c) {
            double rn = vec_maxabs(n, R + (size_t)c * n);
            double den = an * vec_maxabs(n, X + (size_t)c * ldx) + vec_maxabs(n, B + (size_t)c * ldb);
            double e = (den > 0.0) ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
            if (rn != rn) e = NAN;
            if (!done[c]) {
                eta[c] = e;
                if (!isfinite(e)) {
                    bad = 1;
                } else if (e <= tol) {
                    /* the stopping rule of Algorithm 1 (see ir_loop), with the
                     * correction = the change of x over the last inner phase */
                    if (e == 0.0 || zeta[c] <= U64) {
                        done[c] = 1;
                    } else if (outer > 0) {
                        double rho = zeta[c] / zprev[c];
                        done[c] = (rho < 0.5) ? (rho / (1.0 - rho)) * prev[c] <= U64 : prev[c] <= ETA_FLOOR;
                    }
                } else if (outer > 0) {
                    stalls[c] = (e > 0.9 * prev[c]) ? stalls[c] + 1 : 0;
                    if (e > eta1[c] || stalls[c] >= 2) bad = 1;
                }
                if (outer == 0) eta1[c] = e;
                prev[c] = e;
            }
            if (!done[c]) all_done = 0;
            if (!(eta[c] <= worst)) worst = eta[c];
        }
        rep->eta = worst;
        if (bad) { status = 3; break; }
        if (all_done) { status = 0; break; }
        if (outer >= max_outer) { status = 3; break; }
        /* inner phase: CG on A~ for every column not done */
        int longest = 0;
        for (int64_t c = 0; c < m; ++c) {
            if (done[c]) continue;
            double *x = X + (size_t)c * ldx, *r = R + (size_t)c * n;
            memcpy(X0, x, (size_t)n * sizeof(double));
            memcpy(P, r, (size_t)n * sizeof(double));
            double rho = dot64(n, r, r);
            double thr = inner_tol * inner_tol * rho;
            int k = 0;
            while (k < max_inner && rho > thr) {
                lowmv(n, At, half_band, P, pf, Z);
                ++k;
                double alpha = rho / dot64(n, P, Z);
                for (int64_t i = 0; i < n; ++i) x[i] += alpha * P[i];
                for (int64_t i = 0; i < n; ++i) r[i] -= alpha * Z[i];
                double rho1 = dot64(n, r, r);
                double beta = rho1 / rho;
                for (int64_t i = 0; i < n; ++i) P[i] = r[i] + beta * P[i];
                rho = rho1;
            }
            if (k > longest) longest = k;
            /* the phase's correction, relative to the new iterate */
            double dn = 0.0;
            for (int64_t i = 0; i < n; ++i)
                if (fabs(x[i] - X0[i]) > dn) dn = fabs(x[i] - X0[i]);
            zprev[c] = zeta[c];
            zeta[c] = (dn == 0.0) ? 0.0 : dn / vec_maxabs(n, x);
        }
        rep->iters_low += longest;
    }
    free(At); free(R); free(P); free(Z); free(X0); free(pf); free(eta); free(done); free(stalls);
    rep->status = status;
    return status;
}

/* Threads the OpenMP runtime would use (reported beside CPU timings). */
#ifdef _OPENMP
#include <omp.h>
int32_t oracle_threads(void) { return omp_get_max_threads(); }
/* threads of the parallel loops from now on (timing with one core) */
void oracle_set_threads(int32_t k) { omp_set_num_threads(k > 0 ? k : 1); }
#else
int32_t oracle_threads(void) { return 1; }
void oracle_set_threads(int32_t k) { (void)k; }
#endif
