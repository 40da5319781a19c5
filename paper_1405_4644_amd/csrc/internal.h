// Host-side declarations shared by the libspd translation units.
#pragma once
#include <string>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <spd.h>

// Operand rounding of the trailing update: none (binary32 / binary64
// operands), binary16 or bfloat16 (binary32 accumulation).
enum spd_half_kind { HALF_NONE = 0, HALF_F16 = 1, HALF_BF16 = 2 };

namespace spd {

// Panel width of the blocked factorisation per factor type.  128 for both:
// the diagonal-block factor is a chain of NB dependent column steps per
// panel, and at NB = 128 the panel chain (diagonal factor + panel solve)
// stays short enough for the lookahead to hide it behind the trailing
// update, which is still MFMA-bound at K = 128 in binary32 (about 81 TFLOP/s
// measured) and in binary64.
template <typename T> struct Panel;
template <> struct Panel<float> { static constexpr int NB = 128; };
template <> struct Panel<double> { static constexpr int NB = 128; };

// --- factorisation (k_factor.hip) ---
void launch_equil(const double *A, int64_t lda, int64_t n, double *d, int equil, hipStream_t st);
template <typename T>
void launch_convert(const double *A, int64_t lda, int64_t n, int64_t npad, const double *d, double mu, T *H,
                    int64_t ldh, hipStream_t st);
template <typename T>
void launch_potrf_diag(T *Hkk, int64_t ld, int64_t col0, T *Winv, unsigned long long *info, hipStream_t st);
// With half != HALF_NONE (binary32 only) the solved rows are also written,
// rounded to nearest even, to Lh (nrows x NB halves, fragment layout of
// launch_syrk_update_half).
template <typename T>
void launch_trsm_panel(T *H, int64_t ld, int64_t k0, int64_t row0, int64_t nrows, const T *Winv,
                       const unsigned long long *info, hipStream_t st, void *Lh = nullptr, int half = HALF_NONE);
// small_tiles: a binary32 launch with fewer than 512 128-tiles may run on
// 64-tiles (more workgroups for a thin region)
template <typename T>
void launch_syrk_update(T *H, int64_t ld, int64_t k0, int nbk, int64_t r0, int t, int tj_lo, int tj_hi,
                        const unsigned long long *info, hipStream_t st, int prio = 0, int max_grid = 0,
                        bool small_tiles = true);
// Trailing update with binary16 / bfloat16 operands from np panel copies
// (K = 128 each) on 128 x 128 tiles, binary32 accumulation into H: panel p's
// copy in ring slot (slot0 + p) % 16 of Lh (slot stride sstride fragments of
// 8 halves), with skip0 - 4 p 32-row blocks before row r0.
void launch_syrk_update_half(float *H, int64_t ld, const void *Lh, int slot0, int64_t sstride, int skip0, int np,
                             int half, int64_t r0, int t, int tj_lo, int tj_hi, const unsigned long long *info,
                             hipStream_t st, int prio = 0, int max_grid = 0);
// The same for a whole group of np <= 16 panels on 256 x 256 tiles (t per
// side of the region at r0, tile columns [tj_lo, tj_hi)): panel p's copy in
// ring slot (slot0 + p) % 16 of Lh (slot stride sstride fragments of 8
// halves), with skip0 - 4 p 32-row blocks before row r0.
void launch_syrk_update_h256(float *H, int64_t ld, const void *Lh, int slot0, int64_t sstride, int skip0, int np,
                             int half, int64_t r0, int t, int tj_lo, int tj_hi, const unsigned long long *info,
                             hipStream_t st, int prio = 0, int max_grid = 0);
// max_grid > 0 caps the workgroups (multiple of 8); they then loop over tiles
template <typename T>
void launch_trtri_blocks(const T *H, int64_t ld, int64_t nt, const T *Winv, T *W, hipStream_t st);
// Inverses of the 32 x 32 diagonal sub-blocks of a given factor (Winv layout
// as left by the factorisation); a non-positive diagonal entry raises info.
template <typename T>
void launch_inv32_blocks(const T *H, int64_t ld, int64_t npad, T *Winv, unsigned long long *info, hipStream_t st);

// --- triangular solves and scaling (k_solve.hip) ---
// smax[c] = max_i |d_i r_ic| over the n rows (zeroed by the caller first)
void launch_rhs_max(const double *R, int64_t ldr, int64_t n, int m, const double *d, double *smax,
                    hipStream_t st);
// Y[i][c] = round_T(d_i r_ic / s_c) for i < n, 0 for n <= i < npad; s_c = pow2_ceil(smax[c]);
// the same launch clears zd[0, nzd) and zi[0, nzi) when given (neither may
// overlap smax)
template <typename T>
void launch_rhs_scale(const double *R, int64_t ldr, int64_t n, int64_t npad, int m, const double *d,
                      const double *smax, T *Y, int64_t ldy, double *zd, int64_t nzd, int *zi, int64_t nzi,
                      hipStream_t st);
// Triangular solves (k_trsv.hip), blocked by big diagonal blocks of
// solve_nbs(npad) rows whose inverses WB (solve_winv_elems(npad) elements)
// are built once per factorisation from L and the 128-wide block inverses
// W128, with solve_tmp_elems(npad) elements of scratch Tb.
int solve_nbs(int64_t npad);
int solve_nblocks(int64_t npad);
int64_t solve_winv_elems(int64_t npad);
int64_t solve_tmp_elems(int64_t npad);
template <typename T>
void launch_build_winv(const T *L, int64_t ld, int64_t npad, const T *W128, T *WB, T *Tb, hipStream_t st);
// Forward Y -> Z then backward Z -> Y for m right-hand sides (TRSV_MC per
// launch).  P: trsv_scratch_elems(npad) elements; ctl: 2 trsv_ctl_ints(npad)
// ints (the first half for the forward direction, the second for the
// backward), zeroed by the launches themselves unless ctl_zeroed says the
// caller cleared both halves; err: sticky int raised on a timed-out wait.
#define TRSV_MC 8
int64_t trsv_scratch_elems(int64_t npad);
int trsv_ctl_ints(int64_t npad);
template <typename T>
void launch_trsv(const T *L, int64_t ld, const T *WB, int64_t npad, int m, T *Y, T *Z, int64_t ldy, T *P, int *ctl,
                 bool ctl_zeroed, int *err, unsigned long long wait_ticks, hipStream_t st);
// X[i][c] (+)= s_c mu d_i Y[i][c]; zmax (optional, m entries, non-negative on
// entry): raised to max_i |s_c mu d_i Y[i][c]| per column
template <typename T>
void launch_update_x(double *X, int64_t ldx, int64_t n, int m, const T *Y, int64_t ldy, const double *d,
                     double mu, const double *smax, int accumulate, double *zmax, hipStream_t st);
// out[c] = max(out[c], max_i |X[i][c] - S[i][c]|), then S = X (n x m)
void launch_col_maxdiff(const double *X, int64_t ldx, double *S, int64_t lds, int64_t n, int m, double *out,
                        hipStream_t st);
// fill a double array with zeros (a kernel, not a memset node)
void launch_zero(double *p, int64_t count, hipStream_t st);
// dst[0, count) = src[0, count), *dflag = *flag and, when dinfo is given,
// *dinfo = *info, by one workgroup (dst, dflag, dinfo: host-visible memory)
void launch_publish(const double *src, int64_t count, const int *flag, const unsigned long long *info, double *dst,
                    int *dflag, unsigned long long *dinfo, hipStream_t st);
// Lout (binary64, n x n, column-major) <- lower triangle of the factor, zeros above
template <typename T>
void launch_export(const T *L, int64_t ld, int64_t n, double *Lout, int64_t ldo, hipStream_t st);

// --- binary64 residual (k_resid.hip) ---
// R = B - A X for the symmetric A (lower triangle read) and, per column c,
// norms[1 + k m + c] for k = 0..3: max|r|, max|x|, max|b|, max|d r| (atomic
// max; zero them first);
// with want_anorm, norms[0] = ||A||_inf.  P is scratch of resid_scratch(n, m) doubles.
int64_t resid_scratch(int64_t n, int m);
// eta (device, m) from the norms launch_residual wrote (with want_anorm)
void launch_eta_from_norms(const double *norms, int m, double *eta, hipStream_t st);
void launch_residual(const double *A, int64_t lda, int64_t n, const double *X, int64_t ldx, const double *B,
                     int64_t ldb, int m, double *R, int64_t ldr, const double *d, double *norms, int want_anorm,
                     double *P, hipStream_t st);

// --- batched solver (k_batch.hip) ---
struct BatchLaunch {
    int64_t batch;
    const int32_t *n, *nrhs;
    const int64_t *a_off, *b_off;
    const double *A, *B;
    double *X;
    int32_t *prec;
    spd_report *reps;
    double tol, mu16;
    int max_iter, fallback, equilibrate;
    int32_t *order;  // batch entries of scratch
    int *queue;      // one int of scratch
    void *ws;        // grid * batch_ws_stride() bytes
    int grid, waves;
    const float *picker = nullptr;  // perceptron parameters for SPD_AUTO, or NULL
    int64_t *ticks = nullptr;       // per-system wall-clock ticks, or NULL
};
int64_t batch_ws_stride();
// autotuner cache (tune.cpp): values a, b, c of a setting and its time
struct TuneVal {
    int a = 0, b = 0, c = 0;
    double ms = 0.0;
};
int64_t tune_bucket(int64_t n);                               // n rounded to a power of two (log scale)
std::string tune_key(const char *kind, int64_t size);         // "<arch>|hip<ver>|<kind>|<size>"
int tune_lookup(const std::string &key, TuneVal *v);          // 0 absent, 1 in memory, 2 read from the file
void tune_store(const std::string &key, const TuneVal &v);    // memory, and the file when SPD_TUNE_CACHE is set
void tune_clear();                                            // forget memory; the next lookup rereads the file
// a diagonally dominant symmetric n x n test matrix (tuning input): a_ii = 2,
// a_ij = hash(i, j) / n in (-1/n, 1/n) off the diagonal (both triangles)
void launch_tune_matrix(double *A, int64_t n, hipStream_t st);
hipError_t launch_batch(const BatchLaunch &l, hipStream_t st);
// picker features of every system (16 floats each)
void launch_features(int64_t batch, const int32_t *n, const int32_t *nrhs, const int64_t *a_off, const double *A,
                     float *feat, hipStream_t st);
// perceptron training kernels (k_picker.hip); parameters as in spd.h
#define PICK_NPARAM 5508
void launch_mlp_forward(const float *P, const float *X, int64_t N, float *logits, hipStream_t st);
int64_t mlp_grad_scratch(int64_t N);
void launch_mlp_grad(const float *P, const float *X, const int32_t *y, int64_t N, float *grad, float *loss,
                     float *scratch, hipStream_t st);
void launch_adam(float *P, const float *g, float *m, float *v, int64_t count, int step, float lr, float b1, float b2,
                 float eps, hipStream_t st);

// --- conjugate gradients with refinement (k_cg.hip) ---
// Binary32 operator A~ (dense ldt x ldt, or band rows d = -k..k of length
// ldt) and the steps of one CG iteration (product, x/r, p); partial sums per
// workgroup are reduced per column by their consumers.  sc = rho[2][m],
// thr[m]; act = act[2][m] (slots by iteration parity).
int64_t cg_ldt(int64_t n);
int cg_band_ok(int64_t k);
void launch_cg_dense(const double *A, int64_t lda, int64_t n, float *At, int64_t ldt, hipStream_t st);
void launch_cg_band(const double *A, int64_t lda, int64_t n, int64_t k, float *Bd, int64_t ldt, hipStream_t st);
int cg_pf_width(int m);
int64_t cg_pf_elems(int64_t ldt, int m);  // binary32 direction storage (elements)
int64_t cg_mv_parts(int64_t n, int64_t ldt, int64_t k, int m);
int64_t cg_vec_parts(int64_t n);
// Zp: binary32 k-slice partials of the 5..32-column dense product, cg_zp_elems(n, m) elements
int64_t cg_zp_elems(int64_t n, int m);
void launch_cg_mv(const float *At, int64_t ldt, int64_t n, int64_t k, int m, const float *Pf, const double *P,
                  double *Z, double *part, int64_t npart, const int *act, float *Zp, hipStream_t st);
void launch_cg_start(int64_t n, int m, const double *R, double *P, float *Pf, int64_t ldt, double *part,
                     int64_t npart, const int *go, hipStream_t st);
void launch_cg_xr(int64_t n, int m, const double *pzp, int64_t npz, const double *sc, int par, const double *P,
                  const double *Z, double *X, int64_t ldx, double *R, double *part, int64_t npart, const int *act,
                  hipStream_t st);
void launch_cg_p(int64_t n, int m, const double *rrp, int64_t nrr, double *sc, int par, const double *R, double *P,
                 float *Pf, int64_t ldt, int *act, int *cnt, int max_inner, hipStream_t st);
void launch_cg_begin(const double *part, int64_t npart, double *sc, int *act, const int *go, int *cnt,
                     double inner_tol2, int max_inner, int m, hipStream_t st);

}  // namespace spd
