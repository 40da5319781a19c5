// Factorisation kernels: the low-precision Cholesky factorisation of Algorithm 1.
//
// Blocked right-looking Cholesky of H = mu D A D (binary32) or of A itself
// (binary64), panel width NB, stored lower-triangular column-major in an
// npad x npad buffer (npad a multiple of NB; the padding is the identity).
// Per panel k:
//   k_potrf_diag  factor the NB x NB diagonal block in one workgroup, in 32-wide
//                 strips; also store the inverse of every 32 x 32 diagonal
//                 sub-block (used by the panel solve).
//   k_trsm_panel  L_ik = H_ik L_kk^{-T} for the rows below, strip by strip
//                 (MFMA products with the solved strips, then the 32 x 32 inverse).
//   (the trailing update H_ij -= L_ik L_jk^T is in k_update.hip)
// After the last panel, k_trtri_blocks forms W_k = L_kk^{-1} for every
// diagonal block (consumed by the triangular solves).
#include "common.h"
#include "internal.h"
#include "half_ops.h"
#include <type_traits>

// ---------------------------------------------------------------------------
// K1a: equilibration vector d_i = a_ii^{-1/2} (1 where a_ii <= 0 or not
// equilibrating; a non-positive diagonal then surfaces as a breakdown).
__global__ void k_equil(const double *__restrict__ A, int64_t lda, int64_t n, double *__restrict__ d, int equil)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        double a = A[i + i * lda];
        d[i] = (equil && a > 0.0) ? 1.0 / sqrt(a) : 1.0;
    }
}

// K1b: H = round(mu * D A D) on the lower triangle; identity padding.
// Grid: x = row tiles of 256 rows, y = groups of 64 columns (eight at a
// time: eight loads in flight per thread before the stores).
template <typename T>
__global__ __launch_bounds__(256) void k_convert(const double *__restrict__ A, int64_t lda, int64_t n, int64_t npad,
                                                 const double *__restrict__ d, double mu, T *__restrict__ H,
                                                 int64_t ldh)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t jb = (int64_t)blockIdx.y * 64;
    if ((int64_t)blockIdx.x * 256 + 255 < jb || i >= npad)
        return;
    const double mdi = (i < n) ? mu * d[i] : 0.0;
    for (int64_t j0 = jb; j0 < jb + 64 && j0 <= i && j0 < npad; j0 += 8) {
        double a[8], dj[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t j = j0 + c;
            const bool in = (j <= i && i < n && j < n);
            a[c] = in ? A[i + j * lda] : 0.0;
            dj[c] = in ? d[j] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t j = j0 + c;
            if (j > i || j >= npad)
                continue;
            H[i + j * ldh] = (i < n && j < n) ? (T)((mdi * a[c]) * dj[c]) : ((i == j) ? (T)1 : (T)0);
        }
    }
}

// ---------------------------------------------------------------------------
// Value of `v` held by lane `src` of the wavefront (src uniform).
template <typename T> SPD_DEV T bcast(T v, int src);
template <> SPD_DEV float bcast<float>(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
template <> SPD_DEV double bcast<double>(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Square root and reciprocal for the diagonal factor: the hardware
// approximations (about 1 ulp) for binary32, IEEE-correct for binary64.
SPD_DEV float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
SPD_DEV float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
SPD_DEV double fast_sqrt(double x) { return sqrt(x); }
SPD_DEV double fast_rcp(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// K2: Cholesky of one NB x NB diagonal block by one workgroup of 4 waves.
// The lower triangle is held in registers as 32 x 32 MFMA accumulator tiles
// (tile t of the row-major lower triangle belongs to wave t % 4).  For each
// 32-wide strip s (rows 32 s .. NB-1):
//   1. the owners of tile column s spill it to LDS;
//   2. the strip is factored column by column inside each wave, without
//      block barriers: every wave holds its own copy of the 32 x 32 top
//      block in lanes 0..31 and 32 of the rows below in lanes 32..63 (a
//      second pass covers rows beyond 128), broadcasting column values
//      between lanes with readlane;
//   3. the strip is stored and every wave subtracts its outer product from
//      its remaining tiles with MFMA.
// Finally each 32 x 32 diagonal sub-block is inverted (for the panel solve).
// `info` receives min(1-based global column) of a non-positive pivot.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_potrf_diag(T *__restrict__ Hkk, int64_t ld, int64_t col0,
                                                    T *__restrict__ Winv, unsigned long long *info)
{
    constexpr int IB = SPD_IB, NT = NB / IB, NTILES = NT * (NT + 1) / 2, NW = 4;
    constexpr int SLOTS = (NTILES + NW - 1) / NW;
    constexpr int SLD = NB + 1, CLD = IB + 4;
    __shared__ T S[IB * SLD];                     // strip: S[k * SLD + r], r = row offset from 32 s
    __shared__ __align__(16) T Lc[NT][IB * CLD];  // factored 32 x 32 blocks, column-major: Lc[t*CLD + c] = L[c][t]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    __builtin_amdgcn_s_setprio(3);  // on the critical path of the factorisation

    Acc32<T> acc[SLOTS];
    int tI[SLOTS], tJ[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int t = wave + NW * q;
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        tI[q] = (t < NTILES) ? ti : -1;
        tJ[q] = (t < NTILES) ? t - ti * (ti + 1) / 2 : -1;
        // accumulator orientation: register j holds C[ti*32 + col(j)][tj*32 + row(j)]
        if (t < NTILES) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                acc[q].set(j, Hkk[(tI[q] * IB + Acc32<T>::col(j, lane)) + (int64_t)(tJ[q] * IB + Acc32<T>::row(j, lane)) * ld]);
        }
    }

    for (int s = 0; s < NT; ++s) {
        const int rows = NB - s * IB;
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
            if (tJ[q] == s) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    S[Acc32<T>::row(j, lane) * SLD + (tI[q] - s) * IB + Acc32<T>::col(j, lane)] = acc[q].get(j);
            }
        __syncthreads();
        // Strip factorisation without block barriers: lanes 0..31 of EVERY
        // wave hold the 32 x 32 top block (row = lane) and factor it
        // redundantly; lanes 32..63 of wave w carry rows below the top block
        // through the same column operations (pass p: below-rows
        // 128 p + 32 w .. +31; the second pass reuses the final top block).
        // Column j: pivot from lane j, scale, L[k][j] broadcast from lane k
        // (readlane), rank-1 update.  Entries above the diagonal in the top
        // lanes are updated too but never read.
        {
            const int nbelow = rows - IB;
            const int npass = nbelow > 128 ? 2 : 1;
            T *lc = Lc[s];
            for (int pass = 0; pass < npass; ++pass) {
                int row;
                if (lane < IB)
                    row = lane;
                else {
                    const int bidx = pass * 128 + wave * 32 + (lane - IB);
                    row = (bidx < nbelow) ? IB + bidx : -1;
                }
                T v[IB];
#pragma unroll
                for (int k = 0; k < IB; ++k)
                    v[k] = (row >= 0) ? S[k * SLD + row] : (T)0;
#pragma unroll
                for (int j = 0; j < IB; ++j) {
                    const T piv = bcast(v[j], j);
                    if (pass == 0 && !(piv > (T)0) && wave == 0 && lane == 0)
                        atomicMin(info, (unsigned long long)(col0 + s * IB + j + 1));
                    // pass 0 factors; later passes find the final L_jj in lane j
                    const T ljj = (pass == 0) ? fast_sqrt(piv) : piv;
                    const T rinv = fast_rcp(ljj);
                    const T sc = v[j] * rinv;
                    const bool top = lane < IB;
                    v[j] = (pass == 0) ? ((lane == j) ? ljj : sc) : (top ? v[j] : sc);
                    // broadcast L[k][j] from lane k and apply the rank-1 update
                    const T vj = v[j];
                    const bool upd = (pass == 0) || lane >= IB;
#pragma unroll
                    for (int k = j + 1; k < IB; ++k) {
                        const T lkj = bcast(vj, k);
                        if (upd)
                            v[k] -= vj * lkj;
                    }
                }
                if (row >= 0 && (lane >= IB || (pass == 0 && wave == 0))) {
#pragma unroll
                    for (int k = 0; k < IB; ++k) {
                        const T x = (row >= k) ? v[k] : (T)0;
                        S[k * SLD + row] = x;
                        if (row < IB)
                            lc[k * CLD + row] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (int idx = tid; idx < IB * rows; idx += 256) {
            const int j = idx / rows, rr = idx - j * rows;
            Hkk[(s * IB + rr) + (int64_t)(s * IB + j) * ld] = S[j * SLD + rr];
        }
        // trailing update of the owned tiles: D(ti,tj) -= L_tj L_ti^T
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
            if (tJ[q] > s) {
                const T *pa = &S[(tJ[q] - s) * IB];
                const T *pb = &S[(tI[q] - s) * IB];
#pragma unroll
                for (int k = 0; k < IB; k += Frag<T>::K) {
                    Frag<T> fa, fb;
                    fa.load(pa + k * SLD, SLD, lane);
                    fb.load(pb + k * SLD, SLD, lane);
                    fa.negate();
                    mma(acc[q], fa, fb);
                }
            }
        __syncthreads();
    }
    // inverses of the 32 x 32 diagonal sub-blocks: lane r forms row r of
    // W = L^{-1} from W L = I:  W[r][c] = (delta_rc - sum_{k>c} W[r][k] L[k][c]) / L[c][c]
    for (int b = wave; b < NT; b += NW) {
        const int rr = lane & 31;
        const T *lc = Lc[b];
        T w[IB];
#pragma unroll
        for (int c = IB - 1; c >= 0; --c) {
            T a = (c == rr) ? (T)1 : (T)0;
#pragma unroll
            for (int k = c + 1; k < IB; ++k)
                a -= w[k] * lc[c * CLD + k];
            w[c] = (c <= rr) ? a / lc[c * CLD + c] : (T)0;
        }
        if (lane < IB) {
#pragma unroll
            for (int c = 0; c < IB; ++c)
                Winv[(size_t)b * IB * IB + rr + c * IB] = w[c];
        }
    }
}

// ---------------------------------------------------------------------------
// K3: panel solve L_ik = H_ik L_kk^{-T}, in place, rows [row0, row0 + nrows).
// A workgroup of 2 waves owns 64 rows (32 per wave, kept in LDS).  Strip s:
// the workgroup stages L_kk[32 s .. 32 s + 31][0 .. 32 s) and the 32 x 32
// inverse W_s in LDS; each wave computes X_s -= X_{<s} L_{s,<s}^T (MFMA) and
// then X_s <- X_s W_s^T (MFMA) and stores the strip.
template <typename T, int NB, int HK>
__global__ __launch_bounds__(128) void k_trsm_panel(T *__restrict__ H, int64_t ld, int64_t k0, int64_t row0,
                                                    int64_t nrows, const T *__restrict__ Winv,
                                                    const unsigned long long *info, void *__restrict__ Lh)
{
    constexpr int IB = SPD_IB;
    __shared__ T Xs[2][NB * 32];
    __shared__ T Ls[NB * 32];     // Ls[k * 32 + m] = L_kk[32 s + m][k]
    __shared__ T Ws[IB * IB];     // W_s column-major
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    __builtin_amdgcn_s_setprio(3);  // on the critical path of the factorisation
    const int64_t rbase = row0 + (int64_t)blockIdx.x * 64 + wave * 32;
    const bool active = rbase < row0 + nrows;
    T *X = Xs[wave];
    if (active)
        copy_g2s<T, 32, 64, 16>(X, 32, H + rbase + k0 * ld, ld, NB, lane);
    const T *Lkk = H + k0 + k0 * ld;
    for (int s = 0; s < NB / IB; ++s) {
        __syncthreads();
        copy_g2s<T, 32, 128, 8>(Ls, 32, Lkk + 32 * s, ld, IB * s, tid);
        copy_g2s<T, 32, 128, 8>(Ws, IB, Winv + (size_t)s * IB * IB, IB, IB, tid);
        __syncthreads();
        if (active) {
            Acc32<T> acc;
            acc.zero();
            // D[m][n] = sum_{k < 32 s} L_kk[32 s + m][k] X[n][k]
            if (s > 0)
                mma_tile<T>(acc, Ls, 32, X, 32, 32 * s, lane);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = Acc32<T>::row(j, lane), nn = Acc32<T>::col(j, lane);
                X[(32 * s + m) * 32 + nn] -= acc.get(j);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
            // D2[m][n] = sum_t W_s[m][t] Y[n][t] = (Y W_s^T)[n][m]
            Acc32<T> acc2;
            acc2.zero();
            mma_tile<T>(acc2, Ws, IB, X + 32 * s * 32, 32, IB, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = Acc32<T>::row(j, lane), nn = Acc32<T>::col(j, lane);
                const T v = acc2.get(j);
                X[(32 * s + m) * 32 + nn] = v;
                H[(rbase + nn) + (k0 + 32 * s + m) * ld] = v;
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if constexpr (HK != HALF_NONE) {
        // the same 32 rows rounded to binary16 / bfloat16 (round to nearest
        // even), in the fragment layout of the half-precision update
        if (active) {
            using V8 = typename HalfT<HK>::V8;
            V8 *dst = (V8 *)Lh + (size_t)((rbase - row0) / 32) * (NB / 16) * 64;
            const int rr = lane & 31, kh = lane >> 5;
#pragma unroll
            for (int ks = 0; ks < NB / 16; ++ks) {
                V8 v;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v[i] = (typename HalfT<HK>::E)X[(16 * ks + 8 * kh + i) * 32 + rr];
                dst[ks * 64 + lane] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K2, binary32: the same factor with every column step as an MFMA rank-1
// update held in registers.  The 32 x 32 accumulator layout of
// v_mfma_f32_32x32x2f32 (register jj of lane l: row 8(jj/4) + 4(l/32) + jj%4,
// column l%32) puts row j of a tile in register 4(j/8) + j%4 of the 32 lanes
// of half h = (j/4)%2, which is exactly where the MFMA takes a column vector
// for k-slot h.  Tiles are held transposed (T[m][n] = C[n][m]), so column j
// of a tile needs no data movement: one readlane for the pivot, one
// reciprocal square root, then
//     top    -= x x^T        (diagonal tile, every wave keeps a copy)
//     below  -= x x_b^T      (one tile below the diagonal per wave)
//     Binv   -= x w^T        (the wave without a below tile: forward
//                             substitution L W = I for W = L^{-1}, w = row j of W)
// with x = column j of L.  Columns are saved in the same layout, so L and W
// come out ready to store.  One barrier pair per 32-wide strip; the trailing
// tiles are updated from LDS as in the generic kernel.
__global__ __launch_bounds__(256, 2) void k_potrf_f32(float *__restrict__ Hkk, int64_t ld, int64_t col0,
                                                  float *__restrict__ Winv, unsigned long long *info)
{
    constexpr int NB = 128, IB = SPD_IB, NT = NB / IB, NTILES = NT * (NT + 1) / 2, NW = 4;
    constexpr int SLOTS = (NTILES + NW - 1) / NW;
    constexpr int SLD = NB + 1;
    using A = Acc32<float>;
    // S: the strip, S[k * SLD + r] = C[32 s + r][32 s + k], overwritten by
    // the factored strip; SW: W_s = L_ss^{-1}, SW[j * SLD + c] = W[j][c];
    // SD: scratch target of lanes with nothing to keep
    __shared__ float S[IB * SLD];
    __shared__ float SW[IB * SLD];
    __shared__ float SD[IB * SLD];
    __shared__ float SP[IB];  // the strip's pivots
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    __builtin_amdgcn_s_setprio(3);  // on the critical path of the factorisation

    A acc[SLOTS];
    int tI[SLOTS], tJ[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int t = wave + NW * q;
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        tI[q] = (t < NTILES) ? ti : -1;
        tJ[q] = (t < NTILES) ? t - ti * (ti + 1) / 2 : -1;
        if (t < NTILES) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                acc[q].set(j, Hkk[(tI[q] * IB + A::col(j, lane)) + (int64_t)(tJ[q] * IB + A::row(j, lane)) * ld]);
        }
    }
    // per-lane selectors of the two k-slots (lane halves)
    const float hs[2] = {(lane < 32) ? 1.0f : 0.0f, (lane < 32) ? 0.0f : 1.0f};
    const float nhs[2] = {-hs[0], -hs[1]};
    const int r = lane & 31;
    for (int s = 0; s < NT; ++s) {
        const int nbelow = NT - 1 - s;
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
            if (tJ[q] == s) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    S[A::row(j, lane) * SLD + (tI[q] - s) * IB + A::col(j, lane)] = acc[q].get(j);
            }
        lds_barrier();
        // top: the diagonal tile, symmetrised from its lower triangle;
        // sec: below tile s+1+wave, or the identity (wave NW-1), or nothing
        const bool has_below = wave < nbelow, has_inv = wave == NW - 1;
        floatx16 top, sec;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int m = A::row(j, lane), n = A::col(j, lane);
            top[j] = (n >= m) ? S[m * SLD + n] : S[n * SLD + m];
            sec[j] = has_below ? S[m * SLD + (1 + wave) * IB + n] : ((has_inv && m == n) ? 1.0f : 0.0f);
        }
        lds_barrier();  // the strip is overwritten below
        // Column j.  The k-slot selector zeroes the other half exactly; in
        // rows above j of the tile, x picks up rounding residue of entries
        // already eliminated -- it only touches columns (and rows of W) that
        // are final, and those rows are not stored.  (Above the diagonal W
        // stays exactly zero.)  Each column of L and row of W goes to shared
        // memory as it is formed; lanes of the other half, and waves with
        // nothing to keep, write to SD instead, so the addresses are one
        // base per half plus a constant offset per column.
        float *xb[2], *yb[2];
        {
            float *ycol = has_inv ? SW : (has_below ? &S[(1 + wave) * IB] : SD);
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const bool mine = (lane >> 5) == hh;
                xb[hh] = (mine && wave == 0) ? &S[r] : &SD[r];
                yb[hh] = mine ? ycol + r : &SD[r];
            }
        }
        // The update of sec by column j is issued one step late, after the
        // next pivot has been read: a read of an MFMA result waits for every
        // MFMA in flight, so issuing it right behind the diagonal tile's
        // update would put it on the pivot chain.
        float xn_prev = 0.0f, rih_prev = 0.0f;
#pragma unroll
        for (int j = 0; j <= IB; ++j) {
            const int h = (j >> 2) & 1, jj = 4 * (j >> 3) + (j & 3);
            const float t = (j < IB) ? top[jj] : 0.0f;
            if (j > 0) {
                const int hp = ((j - 1) >> 2) & 1, jp = 4 * ((j - 1) >> 3) + ((j - 1) & 3);
                const float y = sec[jp] * rih_prev;
                __builtin_amdgcn_sched_barrier(0);
                sec = __builtin_amdgcn_mfma_f32_32x32x2f32(xn_prev, y, sec, 0, 0, 0);
                yb[hp][(j - 1) * SLD] = y;
            }
            if (j == IB)
                break;
            __builtin_amdgcn_sched_barrier(0);
            const float p = bcast(t, 32 * h + j);
            SP[j] = p;  // the same value from every lane; checked after the strip
            const float ri = __builtin_amdgcn_rsqf(p);
            const float rih = ri * hs[h], nrih = ri * nhs[h];
            const float x = t * rih, xn = t * nrih;
            top = __builtin_amdgcn_mfma_f32_32x32x2f32(xn, x, top, 0, 0, 0);
            xb[h][j * SLD] = x;  // rows above j: masked when stored
            xn_prev = xn;
            rih_prev = rih;
        }
        lds_barrier();
        // the factored strip (rows 32 s .. NB-1) and W_s to global memory
        if (wave == 0) {
            const unsigned long long badm = __ballot(lane < IB && !(SP[lane & 31] > 0.0f));
            if (badm && lane == 0)
                atomicMin(info, (unsigned long long)(col0 + s * IB + __builtin_ctzll(badm) + 1));
        }
        {
            // wave w stores columns w, w+4, ... of the strip (rows 32 s .. NB-1) and of W_s
            const int rows = NB - s * IB;
            float v[8][2], w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = wave + NW * i;
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int rr = lane + 64 * h2;
                    v[i][h2] = (rr < rows) ? ((rr < c) ? 0.0f : S[c * SLD + rr]) : 0.0f;
                }
                w[i] = SW[(lane & 31) * SLD + c];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = wave + NW * i;
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int rr = lane + 64 * h2;
                    if (rr < rows)
                        Hkk[(s * IB + rr) + (int64_t)(s * IB + c) * ld] = v[i][h2];
                }
                if (lane < IB)  // Winv column-major: W[lane][c]
                    Winv[(size_t)s * IB * IB + lane + c * IB] = w[i];
            }
        }
        // trailing update of the owned tiles: D(ti,tj) -= L_tj L_ti^T
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
            if (tJ[q] > s) {
                const float *pa = &S[(tJ[q] - s) * IB];
                const float *pb = &S[(tI[q] - s) * IB];
#pragma unroll
                for (int k = 0; k < IB; k += Frag<float>::K) {
                    Frag<float> fa, fb;
                    fa.load(pa + k * SLD, SLD, lane);
                    fb.load(pb + k * SLD, SLD, lane);
                    fa.negate();
                    mma(acc[q], fa, fb);
                }
            }
        lds_barrier();  // S is refilled by the next strip
    }
}
// ---------------------------------------------------------------------------
// K3, binary32: panel solve Y = X L_kk^{-T} with the rows in registers.
// Each wave owns 16 rows as the transposed block Y^T (128 x 16) in eight
// v_mfma_f32_16x16x4f32 accumulators: register q of lane l of block b holds
// Y[l%16][16 b + 4 (l/16) + q].  The MFMA's k-slots are a free summation
// order, so k-step q of a 16-column block pairs slot u = l/16 with column
// 16 b + 4 u + q -- which is register q of block b in that lane: a solved
// block is its own MFMA operand, no transposition or LDS round trip.
// Strip s (columns 32 s .. 32 s + 31, blocks 2s and 2s+1):
//     Z   = X_s - sum_{t<s} Y_t L_st^T
//     Y_s = Z W_s^T                 (W_s = L_ss^{-1}, from the diagonal factor)
// L_st and W_s are staged once per workgroup in LDS, row-major, so that
// each operand fetch is one 16-byte read of four consecutive k.
template <int HK>
__global__ __launch_bounds__(256) void k_trsm_f32(float *__restrict__ H, int64_t ld, int64_t k0, int64_t row0,
                                                 int64_t nrows, const float *__restrict__ Winv,
                                                 const unsigned long long *info, void *__restrict__ Lh)
{
    constexpr int NB = 128, IB = SPD_IB, PL = IB + 4;
    constexpr int NLB = 6, NBLK = NLB + 4;  // L_st for t < s (s(s-1)/2 + t), then W_0..W_3
    __shared__ __align__(16) float Bs[NBLK][IB * PL];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    __builtin_amdgcn_s_setprio(3);  // on the critical path of the factorisation
    const int64_t rw = row0 + (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
    const bool valid = rw < row0 + nrows;
    const int u = lane >> 4, c4 = 4 * u;
    // the rows, transposed into the accumulators
    floatx4 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc[b][q] = valid ? H[rw + (k0 + 16 * b + c4 + q) * ld] : 0.0f;
    // stage the operands: element (r, c) of block blk at Bs[blk][r * PL + c]
    const float *Lkk = H + k0 + k0 * ld;
    for (int base = 0; base < NBLK * IB * IB; base += 256 * 8) {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int idx = base + i * 256 + tid;
            const int blk = idx >> 10, e = idx & 1023, c = e >> 5, rr = e & 31;
            if (blk < NLB) {
                const int sb = blk < 1 ? 1 : (blk < 3 ? 2 : 3);
                const int tb = blk - sb * (sb - 1) / 2;
                v[i] = Lkk[(IB * sb + rr) + (int64_t)(IB * tb + c) * ld];
            } else {
                v[i] = Winv[(size_t)(blk - NLB) * IB * IB + rr + c * IB];
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int idx = base + i * 256 + tid;
            const int blk = idx >> 10, e = idx & 1023, c = e >> 5, rr = e & 31;
            Bs[blk][rr * PL + c] = v[i];
        }
    }
    __syncthreads();
    const int rl = lane & 15;
#pragma unroll
    for (int s = 0; s < NB / IB; ++s) {
        // Z: blocks 2s, 2s+1 minus the solved blocks 2t, 2t+1 (t < s) times L_st^T
#pragma unroll
        for (int t = 0; t < s; ++t) {
            const float *Lb = Bs[s * (s - 1) / 2 + t];
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const floatx4 a = *(const floatx4 *)&Lb[(16 * o + rl) * PL + 16 * bb + c4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[2 * s + o] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[q], acc[2 * t + bb][q],
                                                                              acc[2 * s + o], 0, 0, 0);
                }
        }
        // Y_s = Z W_s^T (W_s lower triangular: block o needs k-blocks kb <= o)
        const float *Wb = Bs[NLB + s];
        floatx4 y[2];
        y[0] = floatx4{0.f, 0.f, 0.f, 0.f};
        y[1] = y[0];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int o = kb; o < 2; ++o) {
                const floatx4 a = *(const floatx4 *)&Wb[(16 * o + rl) * PL + 16 * kb + c4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    y[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], acc[2 * s + kb][q], y[o], 0, 0, 0);
            }
        acc[2 * s] = y[0];
        acc[2 * s + 1] = y[1];
        if (valid) {
#pragma unroll
            for (int o = 0; o < 2; ++o)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    H[rw + (k0 + IB * s + 16 * o + c4 + q) * ld] = y[o][q];
        }
    }
    if constexpr (HK != HALF_NONE) {
        // the rows rounded to binary16 / bfloat16 (nearest even) in the
        // fragment layout of the half-precision update: element (r, k) at
        // ((r/32)(NB/16) + k/16) 512 + (32 ((k%16)/8) + r%32) 8 + k%8; the
        // four columns of a lane are consecutive there
        if (valid) {
            using E = typename HalfT<HK>::E;
            typedef E E4 __attribute__((ext_vector_type(4)));
            const int64_t rr = rw - row0;
            E *dst = (E *)Lh + (size_t)((rr >> 5) * (NB / 16)) * 512 + (32 * (u >> 1) + (rr & 31)) * 8 + 4 * (u & 1);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                E4 v;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    v[q] = (E)acc[b][q];
                *(E4 *)(dst + (size_t)b * 512) = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K5 (post-factorisation): W_k = L_kk^{-1} for every diagonal block, one
// workgroup per block.  A wave owns block columns j (32 wide): W_jj is the
// stored 32 x 32 inverse and, going down,
//   W_ij = -W_ii * sum_{q=j}^{i-1} L_iq W_qj.
// The block column lives in LDS row-major so it can be an MFMA B operand.
template <typename T, int NB, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_trtri_blocks(const T *__restrict__ H, int64_t ld,
                                                             const T *__restrict__ Winv, T *__restrict__ W)
{
    constexpr int IB = SPD_IB, WS = IB + 1;
    __shared__ T Col[WAVES][NB * WS];
    __shared__ T Pb[WAVES][IB * WS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t k = blockIdx.x, k0 = k * NB;
    const T *Lkk = H + k0 + k0 * ld;
    const T *Wi = Winv + (size_t)k * (NB / IB) * IB * IB;
    T *Wk = W + (size_t)k * NB * NB;
    T *col = Col[wave];
    T *pb = Pb[wave];
    for (int j = wave; j < NB / IB; j += WAVES) {
        // diagonal block
        for (int idx = lane; idx < IB * IB; idx += 64) {
            const int r = idx % IB, c = idx / IB;
            const T v = Wi[(size_t)j * IB * IB + r + c * IB];
            col[(IB * j + r) * WS + c] = v;
            Wk[(IB * j + r) + (size_t)(IB * j + c) * NB] = v;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int i = j + 1; i < NB / IB; ++i) {
            // P = sum_q L_iq W_qj   (D = P: A = L rows of block i, B(k, n) = col[k][n])
            Acc32<T> acc;
            acc.zero();
            const int r = lane & 31;
            if constexpr (sizeof(T) == 4) {
                for (int q = IB * j; q < IB * i; q += 2) {
                    const int kk = q + (lane >> 5);
                    const float a = Lkk[(IB * i + r) + (int64_t)kk * ld];
                    const float b = col[kk * WS + r];
                    acc.mma(a, b);
                }
            } else {
                const int r16 = lane & 15, k4 = lane >> 4;
                for (int q = IB * j; q < IB * i; q += 4) {
                    const int kk = q + k4;
                    double a[2] = {Lkk[(IB * i + r16) + (int64_t)kk * ld], Lkk[(IB * i + 16 + r16) + (int64_t)kk * ld]};
                    double b[2] = {col[kk * WS + r16], col[kk * WS + 16 + r16]};
                    acc.mma(a, b);
                }
            }
            // P to LDS row-major, then W_ij = -W_ii P
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const int m = Acc32<T>::row(jj, lane), nn = Acc32<T>::col(jj, lane);
                pb[m * WS + nn] = acc.get(jj);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
            Acc32<T> acc2;
            acc2.zero();
            const T *wii = Wi + (size_t)i * IB * IB;
            if constexpr (sizeof(T) == 4) {
                for (int q = 0; q < IB; q += 2) {
                    const int kk = q + (lane >> 5);
                    acc2.mma(wii[r + kk * IB], pb[kk * WS + r]);
                }
            } else {
                const int r16 = lane & 15, k4 = lane >> 4;
                for (int q = 0; q < IB; q += 4) {
                    const int kk = q + k4;
                    double a[2] = {wii[r16 + kk * IB], wii[16 + r16 + kk * IB]};
                    double b[2] = {pb[kk * WS + r16], pb[kk * WS + 16 + r16]};
                    acc2.mma(a, b);
                }
            }
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const int m = Acc32<T>::row(jj, lane), nn = Acc32<T>::col(jj, lane);
                const T v = -acc2.get(jj);
                col[(IB * i + m) * WS + nn] = v;
                Wk[(IB * i + m) + (size_t)(IB * j + nn) * NB] = v;
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_export(const T *__restrict__ L, int64_t ld, int64_t n,
                                                double *__restrict__ Lout, int64_t ldo)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i < n)
        Lout[i + j * ldo] = (i >= j) ? (double)L[i + j * ld] : 0.0;
}

// ---------------------------------------------------------------------------
// Launchers
namespace spd {

template <typename T>
void launch_export(const T *L, int64_t ld, int64_t n, double *Lout, int64_t ldo, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_export<T>, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, st, L, ld, n, Lout,
                       ldo);
}
template void launch_export<float>(const float *, int64_t, int64_t, double *, int64_t, hipStream_t);
template void launch_export<double>(const double *, int64_t, int64_t, double *, int64_t, hipStream_t);

void launch_equil(const double *A, int64_t lda, int64_t n, double *d, int equil, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_equil, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, lda, n, d, equil);
}

template <typename T>
void launch_convert(const double *A, int64_t lda, int64_t n, int64_t npad, const double *d, double mu, T *H,
                    int64_t ldh, hipStream_t st)
{
    dim3 grid((unsigned)(npad / 256 + (npad % 256 != 0)), (unsigned)((npad + 63) / 64));
    hipLaunchKernelGGL(k_convert<T>, grid, dim3(256), 0, st, A, lda, n, npad, d, mu, H, ldh);
}
template void launch_convert<float>(const double *, int64_t, int64_t, int64_t, const double *, double, float *,
                                    int64_t, hipStream_t);
template void launch_convert<double>(const double *, int64_t, int64_t, int64_t, const double *, double, double *,
                                     int64_t, hipStream_t);

template <typename T>
void launch_potrf_diag(T *Hkk, int64_t ld, int64_t col0, T *Winv, unsigned long long *info, hipStream_t st)
{
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL(k_potrf_f32, dim3(1), dim3(256), 0, st, Hkk, ld, col0, Winv, info);
    else
        hipLaunchKernelGGL((k_potrf_diag<T, Panel<T>::NB>), dim3(1), dim3(256), 0, st, Hkk, ld, col0, Winv, info);
}
template void launch_potrf_diag<float>(float *, int64_t, int64_t, float *, unsigned long long *, hipStream_t);
template void launch_potrf_diag<double>(double *, int64_t, int64_t, double *, unsigned long long *, hipStream_t);

template <typename T>
void launch_trsm_panel(T *H, int64_t ld, int64_t k0, int64_t row0, int64_t nrows, const T *Winv,
                       const unsigned long long *info, hipStream_t st, void *Lh, int half)
{
    if (nrows <= 0) return;
    const unsigned blocks = (unsigned)((nrows + 63) / 64);
    constexpr int NB = Panel<T>::NB;
    if constexpr (sizeof(T) == 4) {
        static_assert(NB == 128, "binary32 panel solve is written for 128 columns");
        if (half == HALF_F16)
            hipLaunchKernelGGL(k_trsm_f32<HALF_F16>, dim3(blocks), dim3(256), 0, st, H, ld, k0, row0, nrows, Winv,
                               info, Lh);
        else if (half == HALF_BF16)
            hipLaunchKernelGGL(k_trsm_f32<HALF_BF16>, dim3(blocks), dim3(256), 0, st, H, ld, k0, row0, nrows, Winv,
                               info, Lh);
        else
            hipLaunchKernelGGL(k_trsm_f32<HALF_NONE>, dim3(blocks), dim3(256), 0, st, H, ld, k0, row0, nrows, Winv,
                               info, nullptr);
    } else {
        hipLaunchKernelGGL((k_trsm_panel<T, NB, HALF_NONE>), dim3(blocks), dim3(128), 0, st, H, ld, k0, row0, nrows,
                           Winv, info, nullptr);
    }
}
template void launch_trsm_panel<float>(float *, int64_t, int64_t, int64_t, int64_t, const float *,
                                       const unsigned long long *, hipStream_t, void *, int);
template void launch_trsm_panel<double>(double *, int64_t, int64_t, int64_t, int64_t, const double *,
                                        const unsigned long long *, hipStream_t, void *, int);

template <typename T>
void launch_trtri_blocks(const T *H, int64_t ld, int64_t nt, const T *Winv, T *W, hipStream_t st)
{
    constexpr int WV = sizeof(T) == 4 ? 4 : 2;
    hipLaunchKernelGGL((k_trtri_blocks<T, Panel<T>::NB, WV>), dim3((unsigned)nt), dim3(64 * WV), 0, st, H, ld, Winv,
                       W);
}
template void launch_trtri_blocks<float>(const float *, int64_t, int64_t, const float *, float *, hipStream_t);
template void launch_trtri_blocks<double>(const double *, int64_t, int64_t, const double *, double *, hipStream_t);

}  // namespace spd

// ---------------------------------------------------------------------------
// For a factor supplied by the caller (no factorisation ran): the inverse of
// every 32 x 32 diagonal sub-block, in the layout the factorisation leaves
// (block g at Winv + 1024 g, column-major).  One workgroup of 32 threads per
// block; thread c forms column c of W = L_gg^{-1} by forward substitution.
// A diagonal entry that is not positive and finite raises info (1-based
// column, smallest wins), as a breakdown of the factorisation would.
template <typename T>
__global__ __launch_bounds__(32) void k_inv32_blocks(const T *__restrict__ H, int64_t ld, T *__restrict__ Winv,
                                                     unsigned long long *info)
{
    __shared__ T Ls[32][33];
    const int c = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * 32;
    for (int j = 0; j < 32; ++j) Ls[c][j] = (c >= j) ? H[(g0 + c) + (g0 + j) * ld] : (T)0;
    __syncthreads();
    const T dc = Ls[c][c];
    if (!(dc > (T)0) || !(dc < (T)INFINITY))
        atomicMin(info, (unsigned long long)(g0 + c + 1));
    T w[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        T s = (r == c) ? (T)1 : (T)0;
#pragma unroll
        for (int k = 0; k < r; ++k)
            if (k >= c)
                s -= Ls[r][k] * w[k];
        w[r] = (r >= c) ? s / Ls[r][r] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < 32; ++r) Winv[blockIdx.x * 1024 + r + c * 32] = w[r];
}

namespace spd {

template <typename T>
void launch_inv32_blocks(const T *H, int64_t ld, int64_t npad, T *Winv, unsigned long long *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_inv32_blocks<T>, dim3((unsigned)(npad / 32)), dim3(32), 0, st, H, ld, Winv, info);
}
template void launch_inv32_blocks<float>(const float *, int64_t, int64_t, float *, unsigned long long *,
                                         hipStream_t);
template void launch_inv32_blocks<double>(const double *, int64_t, int64_t, double *, unsigned long long *,
                                          hipStream_t);

}  // namespace spd
