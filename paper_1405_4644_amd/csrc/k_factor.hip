// Factorisation kernels: Algorithm 1, line 1 (low-precision Cholesky).
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
//   k_syrk_update H_ij -= L_ik L_jk^T for the lower trailing tiles (MFMA).
// After the last panel, k_trtri_blocks forms W_k = L_kk^{-1} for every
// diagonal block (consumed by the triangular solves).
#include "common.h"
#include "internal.h"
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
// Grid: x = row tiles of 256 rows, y = groups of 8 columns.
template <typename T>
__global__ __launch_bounds__(256) void k_convert(const double *__restrict__ A, int64_t lda, int64_t n, int64_t npad,
                                                 const double *__restrict__ d, double mu, T *__restrict__ H,
                                                 int64_t ldh)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * 8;
    if ((int64_t)blockIdx.x * 256 + 255 < j0 || i >= npad)
        return;
    const double mdi = (i < n) ? mu * d[i] : 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t j = j0 + c;
        if (j > i || j >= npad)
            continue;
        T v;
        if (i < n && j < n)
            v = (T)((mdi * A[i + j * lda]) * d[j]);
        else
            v = (i == j) ? (T)1 : (T)0;
        H[i + j * ldh] = v;
    }
}

// ---------------------------------------------------------------------------
// K2: Cholesky of one NB x NB diagonal block (one workgroup, 256 threads).
// Strip s (columns c0 = 32 s .. c0+31, rows c0 .. NB-1) is loaded to LDS;
// wave 0 factors its top 32 x 32 block in registers and inverts it; every
// thread then solves one row below against that block; the strip is written
// back and its outer product is subtracted from the rest of the block (MFMA).
// `info` receives min(1-based global column) of a non-positive pivot.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_potrf_diag(T *__restrict__ Hkk, int64_t ld, int64_t col0,
                                                    T *__restrict__ Winv, unsigned long long *info)
{
    constexpr int IB = SPD_IB;
    constexpr int SLD = NB + 1;
    __shared__ T S[IB * SLD];
    __shared__ T Wt[IB * (IB + 1)];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;

    for (int s = 0; s < NB / IB; ++s) {
        const int c0 = s * IB, rows = NB - c0;
        for (int idx = tid; idx < rows * IB; idx += 256) {
            const int r = idx % rows, j = idx / rows;
            S[j * SLD + r] = Hkk[(c0 + r) + (int64_t)(c0 + j) * ld];
        }
        __syncthreads();
        if (wave == 0) {
            T v[IB];
#pragma unroll
            for (int j = 0; j < IB; ++j)
                v[j] = (lane < IB && j <= lane) ? S[j * SLD + lane] : (T)0;
            bool failed = false;
#pragma unroll
            for (int j = 0; j < IB; ++j) {
                const T piv = __shfl(v[j], j);
                if (!(piv > (T)0) && !failed) {
                    failed = true;
                    if (lane == 0)
                        atomicMin(info, (unsigned long long)(col0 + c0 + j + 1));
                }
                const T ljj = sqrt(piv);
                if (lane == j)
                    v[j] = ljj;
                else if (lane > j)
                    v[j] = v[j] / ljj;
#pragma unroll
                for (int k = j + 1; k < IB; ++k) {
                    const T lkj = __shfl(v[j], k);
                    if (lane >= k)
                        v[k] -= v[j] * lkj;
                }
            }
            if (lane < IB) {
#pragma unroll
                for (int j = 0; j < IB; ++j)
                    S[j * SLD + lane] = (j <= lane) ? v[j] : (T)0;
            }
            // inverse of the 32 x 32 factor, row `lane`: W L = I gives
            // W[r][c] = (delta_rc - sum_{k=c+1..r} W[r][k] L[k][c]) / L[c][c]
            T w[IB];
#pragma unroll
            for (int c = IB - 1; c >= 0; --c) {
                const T lcc = S[c * SLD + c];
                T acc = (c == lane) ? (T)1 : (T)0;
#pragma unroll
                for (int k = c + 1; k < IB; ++k)
                    if (k <= lane)
                        acc -= w[k] * S[c * SLD + k];
                w[c] = (c <= lane) ? acc / lcc : (T)0;
            }
            if (lane < IB) {
#pragma unroll
                for (int c = 0; c < IB; ++c) {
                    Wt[lane + c * (IB + 1)] = w[c];
                    Winv[(size_t)s * IB * IB + lane + c * IB] = w[c];
                }
            }
        }
        __syncthreads();
        // rows below the top block: x = s_row * W_top^T
        for (int r = IB + tid; r < rows; r += 256) {
            T srow[IB];
#pragma unroll
            for (int t = 0; t < IB; ++t)
                srow[t] = S[t * SLD + r];
#pragma unroll
            for (int c = 0; c < IB; ++c) {
                T acc = (T)0;
#pragma unroll
                for (int t = 0; t <= c; ++t)
                    acc += srow[t] * Wt[c + t * (IB + 1)];
                S[c * SLD + r] = acc;
            }
        }
        __syncthreads();
        for (int idx = tid; idx < rows * IB; idx += 256) {
            const int r = idx % rows, j = idx / rows;
            Hkk[(c0 + r) + (int64_t)(c0 + j) * ld] = S[j * SLD + r];
        }
        // trailing update of the block: rows/cols [c0+IB, NB), 32 x 32 tiles
        const int nt = (rows - IB) / 32;
        const int ntiles = nt * (nt + 1) / 2;
        for (int tIdx = wave; tIdx < ntiles; tIdx += 4) {
            int ti = (int)((sqrtf(8.f * tIdx + 1.f) - 1.f) * 0.5f);
            while (ti * (ti + 1) / 2 > tIdx) --ti;
            while ((ti + 1) * (ti + 2) / 2 <= tIdx) ++ti;
            const int tj = tIdx - ti * (ti + 1) / 2;
            Acc32<T> acc;
            acc.zero();
            // transposed product: D[m][n] = sum_k S[tj-row m][k] S[ti-row n][k] = C[ti n][tj m]
            mma_tile<T>(acc, &S[IB + tj * 32], SLD, &S[IB + ti * 32], SLD, IB, lane);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = Acc32<T>::row(j, lane), nn = Acc32<T>::col(j, lane);
                const int64_t gi = c0 + IB + ti * 32 + nn, gj = c0 + IB + tj * 32 + m;
                Hkk[gi + gj * ld] -= acc.get(j);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K3: panel solve L_ik = H_ik L_kk^{-T}, in place, rows [row0, row0 + nrows).
// Each wave owns 32 rows, kept in LDS; strip s: X_s -= X_{<s} L_{s,<s}^T
// (MFMA), then X_s <- X_s W_s^T with W_s the inverse of the 32 x 32 diagonal
// sub-block.  Waves are independent (no block barrier after the load).
template <typename T, int NB, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_trsm_panel(T *__restrict__ H, int64_t ld, int64_t k0, int64_t row0,
                                                           int64_t nrows, const T *__restrict__ Winv,
                                                           const unsigned long long *info)
{
    constexpr int IB = SPD_IB;
    __shared__ T Xs[WAVES][NB * 32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    const int64_t rbase = row0 + ((int64_t)blockIdx.x * WAVES + wave) * 32;
    if (rbase >= row0 + nrows)
        return;  // whole wave idle; no block barriers follow
    T *X = Xs[wave];
    for (int idx = lane; idx < 32 * NB; idx += 64) {
        const int m = idx & 31, k = idx >> 5;
        X[k * 32 + m] = H[(rbase + m) + (k0 + k) * ld];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const T *Lkk = H + k0 + k0 * ld;
    for (int s = 0; s < NB / IB; ++s) {
        Acc32<T> acc;
        acc.zero();
        // D[m][n] = sum_{k < 32 s} L_kk[32 s + m][k] X[n][k]  (= (X L_s^T)^T)
        if (s > 0)
            mma_tile<T>(acc, Lkk + 32 * s, (int)ld, X, 32, 32 * s, lane);
        __builtin_amdgcn_wave_barrier();
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
        mma_tile<T>(acc2, Winv + (size_t)s * IB * IB, IB, X + 32 * s * 32, 32, IB, lane);
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

// ---------------------------------------------------------------------------
// K4: trailing update H_ij -= L_ik L_jk^T on 128 x 128 lower tiles (MFMA).
// Tiles are numbered over the lower triangle of the trailing region (t tiles
// per side) restricted to tile columns [tj_lo, tj_hi); block indices are
// remapped so that consecutive tiles land on the same XCD (blocks are
// dispatched round-robin over the 8 XCDs).
SPD_DEV void decode_tile(int b, int t, int tj_lo, int tj_hi, int &ti, int &tj)
{
    if (tj_hi - tj_lo <= 4) {
        for (int c = tj_lo; c < tj_hi; ++c) {
            const int cnt = t - c;
            if (b < cnt) {
                ti = c + b;
                tj = c;
                return;
            }
            b -= cnt;
        }
        ti = tj = -1;
        return;
    }
    // lower triangle of the sub-block starting at tile (tj_lo, tj_lo), row-major
    int r = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > b) --r;
    while ((r + 1) * (r + 2) / 2 <= b) ++r;
    ti = tj_lo + r;
    tj = tj_lo + (b - r * (r + 1) / 2);
}

template <typename T> struct SyrkCfg;
template <> struct SyrkCfg<float> { static constexpr int KC = 32; };
template <> struct SyrkCfg<double> { static constexpr int KC = 16; };

template <typename T>
__global__ __launch_bounds__(256) void k_syrk_update(T *__restrict__ H, int64_t ld, int64_t k0, int nbk, int64_t r0,
                                                     int t, int tj_lo, int tj_hi, int ntiles,
                                                     const unsigned long long *info)
{
    constexpr int KC = SyrkCfg<T>::KC;
    constexpr int LDT = SPD_TILE + 4;  // LDS column stride
    __shared__ T As[2][KC * LDT];
    __shared__ T Bs[2][KC * LDT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    const int per = gridDim.x / 8;
    const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (logical >= ntiles)
        return;
    int ti, tj;
    decode_tile(logical, t, tj_lo, tj_hi, ti, tj);
    if (ti < 0)
        return;
    const int64_t crow = r0 + (int64_t)ti * SPD_TILE, ccol = r0 + (int64_t)tj * SPD_TILE;
    const T *pa = H + ccol + k0 * ld;  // rows of tile tj (D rows = C columns)
    const T *pb = H + crow + k0 * ld;  // rows of tile ti (D columns = C rows)
    const int wm = wave >> 1, wn = wave & 1;

    Acc32<T> acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b].zero();

    // 128 rows x KC columns of each operand per chunk, 16-byte vector loads,
    // staged through registers so the next chunk's loads overlap the MFMAs.
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int PER_COL = SPD_TILE / VEC;
    constexpr int NV = PER_COL * KC / 256;  // vectors per thread per operand
    V ra[NV], rb[NV];
    auto gload = [&](int kb) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int idx = tid + 256 * v;
            const int col = idx / PER_COL, r = (idx % PER_COL) * VEC;
            const size_t go = (size_t)(kb + col) * ld + r;
            ra[v] = *(const V *)&pa[go];
            rb[v] = *(const V *)&pb[go];
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int idx = tid + 256 * v;
            const int col = idx / PER_COL, r = (idx % PER_COL) * VEC;
            *(V *)&As[buf][col * LDT + r] = ra[v];
            *(V *)&Bs[buf][col * LDT + r] = rb[v];
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (int kb = 0; kb < nbk; kb += KC) {
        const bool more = kb + KC < nbk;
        if (more)
            gload(kb + KC);
        const T *a0 = &As[buf][64 * wm];
        const T *b0 = &Bs[buf][64 * wn];
#pragma unroll
        for (int k = 0; k < KC; k += Frag<T>::K) {
            Frag<T> fa[2], fb[2];
            fa[0].load(a0 + k * LDT, LDT, lane);
            fa[1].load(a0 + 32 + k * LDT, LDT, lane);
            fb[0].load(b0 + k * LDT, LDT, lane);
            fb[1].load(b0 + 32 + k * LDT, LDT, lane);
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    mma(acc[mi][ni], fa[mi], fb[ni]);
        }
        if (more)
            sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // epilogue: C[crow + 64 wn + 32 ni + n][ccol + 64 wm + 32 mi + m] -= D
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = Acc32<T>::row(j, lane), nn = Acc32<T>::col(j, lane);
                T *p = H + (crow + 64 * wn + 32 * ni + nn) + (ccol + 64 * wm + 32 * mi + m) * ld;
                *p -= acc[mi][ni].get(j);
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
    dim3 grid((unsigned)(npad / 256 + (npad % 256 != 0)), (unsigned)((npad + 7) / 8));
    hipLaunchKernelGGL(k_convert<T>, grid, dim3(256), 0, st, A, lda, n, npad, d, mu, H, ldh);
}
template void launch_convert<float>(const double *, int64_t, int64_t, int64_t, const double *, double, float *,
                                    int64_t, hipStream_t);
template void launch_convert<double>(const double *, int64_t, int64_t, int64_t, const double *, double, double *,
                                     int64_t, hipStream_t);

template <typename T>
void launch_potrf_diag(T *Hkk, int64_t ld, int64_t col0, T *Winv, unsigned long long *info, hipStream_t st)
{
    hipLaunchKernelGGL((k_potrf_diag<T, SPD_NB>), dim3(1), dim3(256), 0, st, Hkk, ld, col0, Winv, info);
}
template void launch_potrf_diag<float>(float *, int64_t, int64_t, float *, unsigned long long *, hipStream_t);
template void launch_potrf_diag<double>(double *, int64_t, int64_t, double *, unsigned long long *, hipStream_t);

template <typename T> constexpr int trsm_waves() { return sizeof(T) == 4 ? 4 : 2; }

template <typename T>
void launch_trsm_panel(T *H, int64_t ld, int64_t k0, int64_t row0, int64_t nrows, const T *Winv,
                       const unsigned long long *info, hipStream_t st)
{
    if (nrows <= 0) return;
    constexpr int W = trsm_waves<T>();
    const unsigned blocks = (unsigned)((nrows + 32 * W - 1) / (32 * W));
    hipLaunchKernelGGL((k_trsm_panel<T, SPD_NB, W>), dim3(blocks), dim3(64 * W), 0, st, H, ld, k0, row0, nrows,
                       Winv, info);
}
template void launch_trsm_panel<float>(float *, int64_t, int64_t, int64_t, int64_t, const float *,
                                       const unsigned long long *, hipStream_t);
template void launch_trsm_panel<double>(double *, int64_t, int64_t, int64_t, int64_t, const double *,
                                        const unsigned long long *, hipStream_t);

template <typename T>
void launch_syrk_update(T *H, int64_t ld, int64_t k0, int nbk, int64_t r0, int t, int tj_lo, int tj_hi,
                        const unsigned long long *info, hipStream_t st)
{
    if (t <= 0 || tj_lo >= tj_hi) return;
    int64_t ntiles = 0;
    for (int c = tj_lo; c < tj_hi; ++c) ntiles += t - c;
    const int64_t grid = ((ntiles + 7) / 8) * 8;
    hipLaunchKernelGGL(k_syrk_update<T>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, k0, nbk, r0, t, tj_lo,
                       tj_hi, (int)ntiles, info);
}
template void launch_syrk_update<float>(float *, int64_t, int64_t, int, int64_t, int, int, int,
                                        const unsigned long long *, hipStream_t);
template void launch_syrk_update<double>(double *, int64_t, int64_t, int, int64_t, int, int, int,
                                         const unsigned long long *, hipStream_t);

template <typename T>
void launch_trtri_blocks(const T *H, int64_t ld, int64_t nt, const T *Winv, T *W, hipStream_t st)
{
    constexpr int WV = sizeof(T) == 4 ? 4 : 2;
    hipLaunchKernelGGL((k_trtri_blocks<T, SPD_NB, WV>), dim3((unsigned)nt), dim3(64 * WV), 0, st, H, ld, Winv, W);
}
template void launch_trtri_blocks<float>(const float *, int64_t, int64_t, const float *, float *, hipStream_t);
template void launch_trtri_blocks<double>(const double *, int64_t, int64_t, const double *, double *, hipStream_t);

}  // namespace spd
