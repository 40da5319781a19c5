// Batched solver: many independent SPD systems A_s X_s = B_s (Eq. (2) per
// system) in one persistent launch, each system taken through all of
// Algorithm 1 by one workgroup:
//   equilibrate and round (mu D A D), blocked Cholesky in the factor's
//   precision (32-wide panels; trailing update on MFMA, with binary16 /
//   bfloat16 rounded operands for the half formats), triangular solves with
//   the 32 x 32 diagonal-block inverses, binary64 residual and backward error,
//   correction loop with the same stopping, divergence and fallback rules as
//   the single-system path (BF16/FP16 -> FP32 -> FP64).
// Systems are handed out by an atomic counter in decreasing order of n
// (counting sort on the device), so the largest start first.  Each workgroup
// owns a fixed slice of workspace (factor, inverses, d, residual): a call
// allocates nothing once the workspace exists, and never synchronises the
// host, so it can be captured in a graph.  Only the lower triangle of each
// A_s is read.
#include <spd.h>

#include <type_traits>

#include "common.h"
#include "internal.h"

#define BNB 32  // panel and tile width
// precision picker: 16 features -> 64 -> 64 -> 4 classes (BF16, FP16, FP32, FP64)
#define PICK_NFEAT 16
#define PICK_NH 64
#define PICK_NCLS 4
#define PICK_LANCZOS 4

struct BatchArgs {
    int64_t batch;
    const int32_t *n, *nrhs;
    const int64_t *a_off, *b_off;
    const double *A, *B;
    double *X;
    int32_t *prec;
    spd_report *reps;
    double tol, mu16;
    int max_iter, fallback, equilibrate;
    const int32_t *order;
    int *queue;
    char *ws;
    int64_t ws_stride;
    const float *picker;  // perceptron parameters for SPD_AUTO (NULL: binary32)
    int64_t *ticks;       // optional: wall-clock ticks of each system's solve
};

// workspace slice of one workgroup
struct BatchWs {
    void *L;      // np x np factor (binary32 or binary64), column-major
    void *Winv;   // np/32 blocks of 32 x 32 inverses of the diagonal blocks
    double *d;    // equilibration
    double *R;    // n x m residual
    double *Am;   // np x np: A's strict lower triangle mirrored into the strict upper (Am[i + j np] = a_ji, i < j)
};

SPD_DEV BatchWs batch_ws(const BatchArgs &a)
{
    char *p = a.ws + (int64_t)blockIdx.x * a.ws_stride;
    BatchWs w;
    w.L = p;
    p += (int64_t)SPD_BATCH_NMAX * SPD_BATCH_NMAX * 8;
    w.Winv = p;
    p += (int64_t)SPD_BATCH_NMAX * BNB * 8;
    w.d = (double *)p;
    p += (int64_t)SPD_BATCH_NMAX * 8;
    w.R = (double *)p;
    p += (int64_t)SPD_BATCH_NMAX * SPD_BATCH_MAXRHS * 8;
    w.Am = (double *)p;
    return w;
}

SPD_DEV double b_nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// shared state of the workgroup
struct SolveSmem {
    double ys[SPD_BATCH_MAXRHS * SPD_BATCH_NMAX];  // solve vectors (factor type)
    double Lk[BNB * (BNB + 1)];                    // inverse of the diagonal block
    double ts[SPD_BATCH_MAXRHS * BNB];
    double red[16][4 * SPD_BATCH_MAXRHS + 1];
    double norms[1 + 4 * SPD_BATCH_MAXRHS];
    double smax[SPD_BATCH_MAXRHS];
    unsigned long long zmax[SPD_BATCH_MAXRHS];  // max |z| per column of the last solve (binary64 bits)
    double arow[SPD_BATCH_NMAX];  // row sums of |A|
    double part[4][SPD_BATCH_MAXRHS + 1][64];  // the residual's per-wave partial row sums (+ |A|)
    int info;
};
// the picker's features and perceptron (about 30 KB: several workgroups per CU)
struct PickSmem {
    double d[SPD_BATCH_NMAX];   // d_i = a_ii^{-1/2}
    double v[SPD_BATCH_NMAX];   // Lanczos vectors v_j, v_{j-1}, w
    double vp[SPD_BATCH_NMAX];
    double w[SPD_BATCH_NMAX];
    double rs[SPD_BATCH_NMAX];  // Gershgorin radii of H
    double ycol[SPD_BATCH_NMAX];
    double rcol[SPD_BATCH_NMAX];
    double red[16][8];
    double ab[2][PICK_LANCZOS];  // Lanczos alpha, beta
    double th[PICK_LANCZOS];     // Ritz values
    float feat[PICK_NFEAT];
    float hid[2][PICK_NH];
    float logit[PICK_NCLS];
};

template <typename T>
SPD_DEV T round_half(T v, int half)
{
    if constexpr (sizeof(T) == 4) {
        if (half == HALF_F16)
            return (float)(_Float16)v;
        if (half == HALF_BF16)
            return (float)(__bf16)v;
    }
    return v;
}

// value of v in lane src (src uniform); binary64 as two 32-bit halves
SPD_DEV float rl(float v, int src) { return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src)); }
SPD_DEV double rl(double v, int src)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// H = round(mu D A D) (lower), identity padding up to np; d (binary64); and
// Am, A's strict lower triangle mirrored into the strict upper triangle of an
// np x np array, so that the residual can stream whole rows of A with
// coalesced loads while A itself is read only in its lower triangle.  32 x 32
// tiles of the lower triangle, one per wave at a time: the tile is loaded
// once (lane = row, 16 columns per lane), converted into L, and transposed
// through the wave's buffer in shared memory (element (c, r) at
// c * 32 + (r ^ c)) for the mirror's coalesced stores.
template <typename T, int WAVES>
__device__ __attribute__((noinline)) void b_convert(const double *A, int n, int np, double *d, double mu, int equil,
                                                    T *L, double *Am, SolveSmem &sm)
{
    // global memory (see gmem): the parameters re-derived as global pointers
    A = (const double *)gmem(A);
    d = (double *)gmem(d);
    L = (T *)gmem(L);
    Am = (double *)gmem(Am);
    constexpr int NT = WAVES * 64;
    static_assert(WAVES * BNB * BNB * 8 <= (int)sizeof(sm.ys), "tile buffers");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *dsh = sm.arow;
    for (int i = tid; i < n; i += NT) {
        const double a = A[i + (int64_t)i * n];
        const double di = (equil && a > 0.0) ? 1.0 / sqrt(a) : 1.0;
        d[i] = di;
        dsh[i] = di;
    }
    __syncthreads();
    const int r = lane & 31, h = lane >> 5;
    const int nb = np / BNB, ntiles = nb * (nb + 1) / 2;
    double *tb = sm.ys + wave * BNB * BNB;
    for (int q = wave; q < ntiles; q += WAVES) {
        int I = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);  // q = I (I + 1) / 2 + J, J <= I
        while (I * (I + 1) / 2 > q) --I;
        while ((I + 1) * (I + 2) / 2 <= q) ++I;
        const int J = q - I * (I + 1) / 2;
        const int i = I * BNB + r;
        double a[BNB / 2];
#pragma unroll
        for (int u = 0; u < BNB / 2; ++u) {
            const int j = J * BNB + 2 * u + h;
            a[u] = (i < n && j < n && j <= i) ? A[i + (int64_t)j * n] : 0.0;
        }
        const double di = (i < n) ? dsh[i] : 0.0;
#pragma unroll
        for (int u = 0; u < BNB / 2; ++u) {
            const int c = 2 * u + h, j = J * BNB + c;
            if (j <= i) {
                T v;
                if (i < n && j < n)
                    v = (T)(((mu * di) * a[u]) * dsh[j]);
                else
                    v = (i == j) ? (T)1 : (T)0;
                L[i + (int64_t)j * np] = v;
            }
            tb[c * BNB + (r ^ c)] = a[u];
        }
        __builtin_amdgcn_wave_barrier();
        // Am (row J*32 + c, column I*32 + rr) = a (I*32 + rr, J*32 + c), c = lane % 32, strictly above the diagonal
        double *dst = Am + (int64_t)J * BNB + (int64_t)I * BNB * np;
#pragma unroll
        for (int u = 0; u < BNB / 2; ++u) {
            const int rr = 2 * u + h;
            if (I > J || r < rr)
                dst[r + (int64_t)rr * np] = tb[r * BNB + (rr ^ r)];
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
}

// Factor the 32 x 32 diagonal block at (k0, k0) in one wavefront and form
// its inverse W, left-looking: lane r holds row r; at column j every lane
// forms a_rj - sum_{q<j} L[r][q] L[j][q] with row j of L read from shared
// memory (Lr, row-major, every lane the same address: a broadcast, four
// values per read), lane j's value is the pivot (one readlane), and each lane
// publishes its new L[r][j] to Lr.  W follows by forward substitution
// L W = I, lane c building column c (W[r][c] = (delta_rc -
// sum_{q<r} L[r][q] W[q][c]) / L[r][r]) from the same rows.  Lanes 32..63
// mirror lanes 0..31 and store nothing.  Outputs: the block in L, W in Ws
// (Ws[c * 33 + r]) and Wg (column-major).  Returns the 1-based failing
// column of the block, 0 on success.
template <typename T>
__device__ __attribute__((noinline)) int b_diag(T *L, int np, int k0, T *Ws, T *Wg, T *Lr)
{
    L = (T *)gmem(L);  // global memory (see gmem)
    Wg = (T *)gmem(Wg);
    constexpr int S = 36;  // Lr row stride (16-byte aligned rows)
    const int lane = threadIdx.x & 63, r = lane & 31;
    const bool store = lane < BNB;
    T row[BNB];
#pragma unroll
    for (int c = 0; c < BNB; ++c)
        row[c] = (c <= r) ? L[(k0 + r) + (int64_t)(k0 + c) * np] : (T)0;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < BNB; ++j) {
        T p[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int q = 0; q < j; ++q) p[q & 3] = fma(row[q], Lr[j * S + q], p[q & 3]);
        const T sv = row[j] - ((p[0] + p[1]) + (p[2] + p[3]));
        const T piv = rl(sv, j);
        if (!(piv > (T)0)) {
            bad = j + 1;
            break;
        }
        const T ljj = sqrt(piv);
        row[j] = (r == j) ? ljj : ((r > j) ? sv / ljj : (T)0);
        if (store)
            Lr[r * S + j] = row[j];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_sched_barrier(0);
    }
    if (bad)
        return bad;
    // W: each new row of W goes to Ws as it is formed
    T w[BNB];
#pragma unroll
    for (int i = 0; i < BNB; ++i) {
        T p[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int q = 0; q < i; ++q) p[q & 3] = fma(Lr[i * S + q], w[q], p[q & 3]);
        const T rhs = ((r == i) ? (T)1 : (T)0) - ((p[0] + p[1]) + (p[2] + p[3]));
        w[i] = (i < r) ? (T)0 : rhs / Lr[i * S + i];
        if (store)
            Ws[r * (BNB + 1) + i] = w[i];  // lane r = column r of W
        __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_wave_barrier();
    // the block of L and W (column-major) to global memory, column by column
    for (int e = lane; e < BNB * BNB; e += 64) {
        const int rr = e % BNB, cc = e / BNB;
        if (cc <= rr)
            L[(k0 + rr) + (int64_t)(k0 + cc) * np] = Lr[rr * S + cc];
        Wg[e] = Ws[cc * (BNB + 1) + rr];
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Blocked right-looking Cholesky of the np x np lower matrix in L.  Returns
// the 1-based failing column (0 on success); Winv receives the inverses of
// the 32 x 32 diagonal blocks.  With half != HALF_NONE the trailing-update
// operands are rounded to that format (binary32 accumulation).
template <typename T, int WAVES>
__device__ __attribute__((noinline)) int b_factor(T *L, int np, T *Winv, int half, SolveSmem &sm)
{
    L = (T *)gmem(L);  // global memory (see gmem)
    Winv = (T *)gmem(Winv);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = np / BNB;
    T *Ws = (T *)sm.Lk;  // inverse of the diagonal block: Ws[c * 33 + r] = W[r][c]
    for (int kb = 0; kb < nb; ++kb) {
        const int k0 = kb * BNB;
        if (wave == 0) {
            const int bad = b_diag<T>(L, np, k0, Ws, Winv + (int64_t)kb * BNB * BNB, (T *)sm.ys);
            if (lane == 0)
                sm.info = bad ? k0 + bad : 0;
        }
        __syncthreads();
        if (sm.info)
            return sm.info;
        // panel: L_ik = H_ik W^T for the row blocks below, one 32 x 32 block per
        // wave.  A binary32 factor's blocks also go, transposed, to U = L^T in
        // the strict upper triangle of the same array (for its backward
        // substitutions), through the wave's 32 x 32 buffer in shared memory
        // (element (c, r) at c * 32 + (r ^ c): both sides conflict-free) so
        // that both global stores are coalesced.  The buffers overlap b_diag's
        // rows, which are no longer needed.
        T *tb = (T *)sm.ys + wave * BNB * BNB;
        for (int I = kb + 1 + wave; I < nb; I += WAVES) {
            Acc32<T> acc;
            acc.zero();
            // D[c][r] = sum_q W[c][q] H[r][q]
            mma_tile<T>(acc, Ws, BNB + 1, L + (int64_t)I * BNB + (int64_t)k0 * np, np, BNB, lane);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int c = Acc32<T>::row(j, lane), r = Acc32<T>::col(j, lane);
                L[((int64_t)I * BNB + r) + (int64_t)(k0 + c) * np] = acc.get(j);
                if constexpr (sizeof(T) == 4)
                    tb[c * BNB + (r ^ c)] = acc.get(j);
            }
            if constexpr (sizeof(T) == 4) {
                __builtin_amdgcn_wave_barrier();
                // U (row k0 + c, column I*32 + rr) = L (I*32 + rr, k0 + c), c = lane % 32
                const int cc = lane & 31, h = lane >> 5;
                T *dst = L + k0 + (int64_t)I * BNB * np;
#pragma unroll
                for (int u = 0; u < BNB / 2; ++u) {
                    const int rr = 2 * u + h;
                    dst[cc + (int64_t)rr * np] = tb[cc * BNB + (rr ^ cc)];
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        // trailing update of the lower tiles (I, J), kb < J <= I; a wave's
        // next tile's C values and this tile's operands are loaded before
        // this tile's MFMAs
        const int t = nb - kb - 1, ntile = t * (t + 1) / 2;
        auto tile_of = [&](int q, int &gI, int &gJ) {
            int I = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
            while (I * (I + 1) / 2 > q) --I;
            while ((I + 1) * (I + 2) / 2 <= q) ++I;
            gI = kb + 1 + I;
            gJ = kb + 1 + q - I * (I + 1) / 2;
        };
        auto load_c = [&](Acc32<T> &acc, const T *C) {
            // register j: column Acc32::row(j) of the tile, row Acc32::col(j)
#pragma unroll
            for (int j = 0; j < 16; ++j)
                acc.set(j, C[Acc32<T>::col(j, lane) + (int64_t)Acc32<T>::row(j, lane) * np]);
        };
        int gI = 0, gJ = 0;
        Acc32<T> nxt;
        if (wave < ntile) {
            tile_of(wave, gI, gJ);
            load_c(nxt, L + (int64_t)gI * BNB + (int64_t)gJ * BNB * np);
        }
        for (int q = wave; q < ntile; q += WAVES) {
            T *C = L + (int64_t)gI * BNB + (int64_t)gJ * BNB * np;
            const T *pJ = L + (int64_t)gJ * BNB + (int64_t)k0 * np;
            const T *pI = L + (int64_t)gI * BNB + (int64_t)k0 * np;
            Acc32<T> acc = nxt;
            Frag<T> fa[BNB / Frag<T>::K], fb[BNB / Frag<T>::K];
#pragma unroll
            for (int s2 = 0; s2 < BNB / Frag<T>::K; ++s2) {
                fa[s2].load(pJ + (int64_t)s2 * Frag<T>::K * np, np, lane);
                fb[s2].load(pI + (int64_t)s2 * Frag<T>::K * np, np, lane);
            }
            if (q + WAVES < ntile) {
                tile_of(q + WAVES, gI, gJ);
                load_c(nxt, L + (int64_t)gI * BNB + (int64_t)gJ * BNB * np);
            }
#pragma unroll
            for (int s2 = 0; s2 < BNB / Frag<T>::K; ++s2) {
                if constexpr (sizeof(T) == 4) {
                    if (half) {
                        fa[s2].v = round_half(fa[s2].v, half);
                        fb[s2].v = round_half(fb[s2].v, half);
                    }
                }
                fa[s2].negate();
                mma(acc, fa[s2], fb[s2]);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                C[Acc32<T>::col(j, lane) + (int64_t)Acc32<T>::row(j, lane) * np] = acc.get(j);
        }
        __syncthreads();
    }
    return 0;
}

// ---------------------------------------------------------------------------
// X (+)= s mu D L^{-T} L^{-1} round(D R / s) for m right-hand sides; the
// scales s_c = pow2_ceil(smax[c]) (smax in shared memory).  Every global
// read is coalesced across lanes and issued in batches (no loop carries a
// load-to-use dependency).
template <typename T, int WAVES>
__device__ __attribute__((noinline)) void b_solve(const T *L, const T *Winv, int n, int np, int m, const double *R, const double *d, double mu,
                     double *X, int accumulate, SolveSmem &sm)
{
    constexpr int NT = WAVES * 64, MR = SPD_BATCH_MAXRHS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = np / BNB;
    const auto gL = gmem(L), gW = gmem(Winv);
    const auto gR = gmem(R), gd = gmem(d);
    const auto gX = gmem(X);
    T *ys = (T *)sm.ys;  // ys[c * NMAX + i]
    constexpr int NM = SPD_BATCH_NMAX;
    for (int idx = tid; idx < m * np; idx += NT) {
        const int c = idx / np, i = idx % np;
        const double s = pow2_ceil(sm.smax[c]);
        ys[c * NM + i] = (i < n) ? (T)(gd[i] * gR[i + (int64_t)c * n] / s) : (T)0;
    }
    __syncthreads();
    // Each step first issues the loads it needs -- the W block (staged in
    // shared memory, Wl[q * 33 + r] = W[r][q]) and the matrix values of the
    // step -- so that their latencies overlap; sums keep the same order.
    constexpr int WPT = BNB * BNB / NT;  // W values staged per thread
    static_assert(WPT * NT == BNB * BNB, "W staging");
    T *Wl = (T *)sm.Lk;
    T *zs = (T *)sm.ts;  // the block just solved, zs[c * BNB + r]
    // forward: z_k = W_k y_k, then y_below -= L_below,k z_k
    for (int kb = 0; kb < nb; ++kb) {
        const int k0 = kb * BNB;
        const auto W = gW + (int64_t)kb * BNB * BNB;
        T wt[WPT];
#pragma unroll
        for (int u = 0; u < WPT; ++u) wt[u] = W[tid + u * NT];
        const int i1 = k0 + BNB + tid;
        T lv[BNB];
        if (i1 < np) {
#pragma unroll
            for (int q = 0; q < BNB; ++q) lv[q] = gL[i1 + (int64_t)(k0 + q) * np];
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int e = tid + u * NT;
            Wl[(e / BNB) * (BNB + 1) + e % BNB] = wt[u];
        }
        __syncthreads();
        if (tid < BNB * m) {
            const int r = tid % BNB, c = tid / BNB;
            T z = (T)0;
#pragma unroll
            for (int q = 0; q < BNB; ++q) z += Wl[q * (BNB + 1) + r] * ys[c * NM + k0 + q];  // W is zero above its diagonal
            zs[tid] = z;
        }
        __syncthreads();
        if (tid < BNB * m)
            ys[(tid / BNB) * NM + k0 + tid % BNB] = zs[tid];
        if (i1 < np) {
#pragma unroll
            for (int c = 0; c < MR; ++c) {
                if (c < m) {
                    T sacc = (T)0;
#pragma unroll
                    for (int q = 0; q < BNB; ++q) sacc += lv[q] * zs[c * BNB + q];
                    ys[c * NM + i1] -= sacc;
                }
            }
        }
        for (int i = i1 + NT; i < np; i += NT) {
            T lw[BNB];
#pragma unroll
            for (int q = 0; q < BNB; ++q) lw[q] = gL[i + (int64_t)(k0 + q) * np];
#pragma unroll
            for (int c = 0; c < MR; ++c) {
                if (c < m) {
                    T sacc = (T)0;
#pragma unroll
                    for (int q = 0; q < BNB; ++q) sacc += lw[q] * zs[c * BNB + q];
                    ys[c * NM + i] -= sacc;
                }
            }
        }
        __syncthreads();
    }
    // backward.  A binary32 factor serves three or more solves on average and
    // carries U = L^T (written by its panel steps): a sweep that mirrors the
    // forward one.  A binary64 factor serves one solve, where the copy did not
    // pay (measured): column sums by wave over L itself.
    if constexpr (sizeof(T) == 4) {
        // backward, right-looking on U = L^T (held in the strict upper triangle
        // of the same array, written by the factorisation's panel steps):
        // x_k = W_k^T y_k, then
        // y_above -= U_above,k x_k -- the forward sweep's mirror, each row's
        // values of a step one coalesced load per column of the block
        for (int kb = nb - 1; kb >= 0; --kb) {
            const int k0 = kb * BNB;
            const auto W = gW + (int64_t)kb * BNB * BNB;
            T wt[WPT];
#pragma unroll
            for (int u = 0; u < WPT; ++u) wt[u] = W[tid + u * NT];
            const int i1 = tid;  // rows above the block: 0 .. k0 - 1
            T lv[BNB];
            if (i1 < k0) {
#pragma unroll
                for (int q = 0; q < BNB; ++q) lv[q] = gL[i1 + (int64_t)(k0 + q) * np];
            }
#pragma unroll
            for (int u = 0; u < WPT; ++u) {
                const int e = tid + u * NT;
                Wl[(e / BNB) * (BNB + 1) + e % BNB] = wt[u];
            }
            __syncthreads();
            if (tid < BNB * m) {
                const int r = tid % BNB, c = tid / BNB;
                T x = (T)0;
#pragma unroll
                for (int q = 0; q < BNB; ++q) x += Wl[r * (BNB + 1) + q] * ys[c * NM + k0 + q];  // W^T: zero below
                zs[tid] = x;
            }
            __syncthreads();
            if (tid < BNB * m)
                ys[(tid / BNB) * NM + k0 + tid % BNB] = zs[tid];
            if (i1 < k0) {
#pragma unroll
                for (int c = 0; c < MR; ++c) {
                    if (c < m) {
                        T sacc = (T)0;
#pragma unroll
                        for (int q = 0; q < BNB; ++q) sacc += lv[q] * zs[c * BNB + q];
                        ys[c * NM + i1] -= sacc;
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            for (int i = i1 + NT; i < k0; i += NT) {
                T lw[BNB];
#pragma unroll
                for (int q = 0; q < BNB; ++q) lw[q] = gL[i + (int64_t)(k0 + q) * np];
#pragma unroll
                for (int c = 0; c < MR; ++c) {
                    if (c < m) {
                        T sacc = (T)0;
#pragma unroll
                        for (int q = 0; q < BNB; ++q) sacc += lw[q] * zs[c * BNB + q];
                        ys[c * NM + i] -= sacc;
                    }
                }
            }
            __syncthreads();
        }
    } else {
        // backward: x_k = W_k^T (y_k - L_below,k^T x_below); the column sums by
        // wave (lanes over rows), column q + WAVES's values loaded while column
        // q's are used
        constexpr int RCH = NM / 64;
        T *ts = (T *)sm.ts;
        for (int kb = nb - 1; kb >= 0; --kb) {
            const int k0 = kb * BNB, r0 = k0 + BNB;
            const auto W = gW + (int64_t)kb * BNB * BNB;
            T wt[WPT];
#pragma unroll
            for (int u = 0; u < WPT; ++u) wt[u] = W[tid + u * NT];
            const int nch = (np - r0 + 63) / 64;
            T cur[RCH], nxt[RCH];
            auto load_col = [&](T *dst, int q) {
                const auto col = gL + (int64_t)(k0 + q) * np;
#pragma unroll
                for (int u = 0; u < RCH; ++u) {
                    const int i = r0 + 64 * u + lane;
                    dst[u] = (u < nch && i < np) ? col[i] : (T)0;
                }
            };
            load_col(cur, wave);
#pragma unroll 1
            for (int q = wave; q < BNB; q += WAVES) {
                if (q + WAVES < BNB)
                    load_col(nxt, q + WAVES);
                T acc[MR];
#pragma unroll
                for (int c = 0; c < MR; ++c) acc[c] = (T)0;
#pragma unroll
                for (int u = 0; u < RCH; ++u) {
                    const int i = r0 + 64 * u + lane;
                    if (u < nch && i < np) {
#pragma unroll
                        for (int c = 0; c < MR; ++c)
                            if (c < m)
                                acc[c] += cur[u] * ys[c * NM + i];
                    }
                }
#pragma unroll
                for (int c = 0; c < MR; ++c) {
                    if (c < m) {
                        T v = acc[c];
#pragma unroll
                        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                        if (lane == 0)
                            ts[c * BNB + q] = v;
                    }
                }
#pragma unroll
                for (int u = 0; u < RCH; ++u) cur[u] = nxt[u];
            }
#pragma unroll
            for (int u = 0; u < WPT; ++u) {
                const int e = tid + u * NT;
                Wl[(e / BNB) * (BNB + 1) + e % BNB] = wt[u];
            }
            __syncthreads();
            T x = (T)0;
            if (tid < BNB * m) {
                const int r = tid % BNB, c = tid / BNB;
#pragma unroll
                for (int q = 0; q < BNB; ++q) x += Wl[r * (BNB + 1) + q] * (ys[c * NM + k0 + q] - ts[c * BNB + q]);
            }
            __syncthreads();
            if (tid < BNB * m)
                ys[(tid / BNB) * NM + k0 + tid % BNB] = x;
            __syncthreads();
        }
    }
    if (tid < m)
        sm.zmax[tid] = 0ull;
    __syncthreads();
    for (int idx = tid; idx < m * n; idx += NT) {
        const int c = idx / n, i = idx % n;
        const double s = pow2_ceil(sm.smax[c]);
        const double z = ((s * mu) * gd[i]) * (double)ys[c * NM + i];
        const auto px = gX + i + (int64_t)c * n;
        *px = accumulate ? *px + z : z;
        atomicMax(&sm.zmax[c], (unsigned long long)__double_as_longlong(fabs(z)));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// R = B - A X (binary64) and the norms: norms[1 + k m + c], k = 0..3:
// max|r|, max|x|, max|b|, max|d r|; with want_anorm also norms[0] =
// ||A||_inf.  X is staged in shared memory.  Rows in passes of 64 (lane =
// row), the columns split among the waves in whole batches of CH: a_ij from
// A for j <= i and from the mirror Am (written by b_convert) for j > i, so
// each load is coalesced (reading the lower triangle alone would need a
// second, column-wise pass whose loads touch a cache line per lane), with the
// next batch in flight.  Each row's four wave partials are added in a fixed
// order, so the result does not depend on timing.  Splitting the columns
// rather than the rows keeps the waves level for every n (rows per wave
// left one wave a second full pass whenever n was just above 256).
template <int WAVES>
__device__ __attribute__((noinline)) void b_residual(const double *A, const double *Am, int n, int np, int m,
                                                     const double *X, const double *B, const double *d, double *R,
                                                     int want_anorm, SolveSmem &sm)
{
    constexpr int NT = WAVES * 64, NM = SPD_BATCH_NMAX;
    static_assert(WAVES == 4, "partial sums are laid out for four waves");
    const auto gA = gmem(A), gAm = gmem(Am), gX = gmem(X), gB = gmem(B);
    const auto gR = gmem(R);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int MR = SPD_BATCH_MAXRHS;
    double *xs = sm.ys;  // xs[c * NMAX + j]
    double *abs_rows = sm.arow;
    for (int idx = tid; idx < m * n; idx += NT) {
        const int c = idx / n, j = idx % n;
        xs[c * NM + j] = gX[j + (int64_t)c * n];
    }
    __syncthreads();
    constexpr int CH = 16;
    const int nch = (n + CH - 1) / CH, cpw = (nch + WAVES - 1) / WAVES;
    const int jlo = wave * cpw * CH, jhi = min(n, (wave + 1) * cpw * CH);
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        double acc[MR], aa = 0.0;
#pragma unroll
        for (int c = 0; c < MR; ++c) acc[c] = 0.0;
        double a[CH], an[CH];
        auto load = [&](double *dst, int j0) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int j = j0 + u;
                dst[u] = (i < n && j < jhi) ? ((j <= i) ? gA[i + (int64_t)j * n] : gAm[i + (int64_t)j * np]) : 0.0;
            }
        };
        if (jlo < jhi)
            load(a, jlo);
        for (int j0 = jlo; j0 < jhi; j0 += CH) {
            if (j0 + CH < jhi)
                load(an, j0 + CH);
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int j = min(j0 + u, n - 1);
#pragma unroll
                for (int c = 0; c < MR; ++c)
                    if (c < m)
                        acc[c] = fma(a[u], xs[c * NM + j], acc[c]);
                if (want_anorm)
                    aa += fabs(a[u]);
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) a[u] = an[u];
        }
#pragma unroll
        for (int c = 0; c < MR; ++c)
            if (c < m)
                sm.part[wave][c][lane] = acc[c];
        sm.part[wave][MR][lane] = aa;
        __syncthreads();
        for (int idx = tid; idx < (m + 1) * 64; idx += NT) {
            const int c = idx / 64, l = idx % 64, r = i0 + l;
            const int slot = (c < m) ? c : MR;
            if (r < n && (c < m || want_anorm)) {
                const double s = ((sm.part[0][slot][l] + sm.part[1][slot][l]) + sm.part[2][slot][l]) + sm.part[3][slot][l];
                if (c < m)
                    gR[r + (int64_t)c * n] = gB[r + (int64_t)c * n] - s;
                else
                    abs_rows[r] = s;
            }
        }
        __syncthreads();
    }
    // maxima (NaN propagates), per column, one kind at a time (kind 0..3:
    // |r|, |x|, |b|, |d r|), then ||A||_inf
#pragma unroll 1
    for (int kind = 0; kind < 4; ++kind) {
        double v[MR];
#pragma unroll
        for (int c = 0; c < MR; ++c) v[c] = 0.0;
        for (int i = tid; i < n; i += NT) {
#pragma unroll
            for (int c = 0; c < MR; ++c)
                if (c < m) {
                    const double x = (kind == 0) ? gR[i + (int64_t)c * n]
                                     : (kind == 1) ? xs[c * NM + i]
                                     : (kind == 2) ? gB[i + (int64_t)c * n]
                                                   : gmem(d)[i] * gR[i + (int64_t)c * n];
                    v[c] = b_nanmax(v[c], fabs(x));
                }
        }
#pragma unroll
        for (int c = 0; c < MR; ++c) {
            if (c >= m)
                break;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[c] = b_nanmax(v[c], __shfl_xor(v[c], off));
            if (lane == 0)
                sm.red[wave][c] = v[c];
        }
        __syncthreads();
        if (tid < m) {
            double x = 0.0;
            for (int w = 0; w < WAVES; ++w) x = b_nanmax(x, sm.red[w][tid]);
            sm.norms[1 + kind * m + tid] = x;
        }
        __syncthreads();
    }
    if (want_anorm) {
        double x = 0.0;
        for (int i = tid; i < n; i += NT) x = b_nanmax(x, abs_rows[i]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x = b_nanmax(x, __shfl_xor(x, off));
        if (lane == 0)
            sm.red[wave][0] = x;
        __syncthreads();
        if (tid == 0) {
            double y = 0.0;
            for (int w = 0; w < WAVES; ++w) y = b_nanmax(y, sm.red[w][0]);
            sm.norms[0] = y;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Precision picker (a project addition around Algorithm 1: which precision to
// run it in).  Features of one system, in binary64, by the workgroup:
// d_i = a_ii^{-1/2} (1 where a_ii <= 0), H = D A D, r_i = sum_{j != i} |h_ij|;
// four Lanczos steps on H from (1, ..., 1)/sqrt(n) without
// reorthogonalisation (stopping early when beta <= 1e-12 max(|alpha|, 1));
// theta = eigenvalues of the tridiagonal (bisection on Sturm counts).
//   f0 log2(n)/9, f1 m/8, f2..f4 spread/mean/std of log10 a_ii (/6, /6, /3),
//   f5 log10(1 + max r)/3, f6 log10(1 + mean r)/3, f7 share of rows r < 1,
//   f8 clip(1 - max r, -10, 1)/10, f9 log10 theta_max/3,
//   f10 log10 max(theta_min, 1e-16)/6, f11 log10(theta_max/max(theta_min, 1e-16))/6,
//   f12 max off-diagonal |h_ij|, f13 log10(||H||_F/sqrt(n))/3,
//   f14 last beta/theta_max (0 after an early stop),
//   f15 (theta_2 - theta_1)/(theta_max - theta_1) (0 with fewer than 3 values).

// block reduction of NV values per thread, fixed order (wave butterflies,
// then waves in order); op 0 = sum, 1 = max, 2 = min.  Result in every thread.
template <int WAVES, int NV>
SPD_DEV void b_reduce(double v[NV], const int op[NV], PickSmem &sm)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v[k], off);
            v[k] = op[k] == 0 ? v[k] + o : op[k] == 1 ? fmax(v[k], o) : fmin(v[k], o);
        }
        if (lane == 0)
            sm.red[wave][k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = sm.red[0][k];
        for (int w = 1; w < WAVES; ++w) {
            const double o = sm.red[w][k];
            x = op[k] == 0 ? x + o : op[k] == 1 ? fmax(x, o) : fmin(x, o);
        }
        v[k] = x;
    }
    __syncthreads();
}

// y = H v (v, y in shared memory), H = D A D from the lower triangle of A.
// With first: rs[i] = r_i, and per thread the partial max off-diagonal |h|
// and sum of h^2 (each stored element once, off-diagonal ones counted twice).
template <int WAVES>
SPD_DEV void b_hv(const double *A, int n, const double *v, double *y, bool first, double &hmax, double &fro,
                  PickSmem &sm)
{
    constexpr int NT = WAVES * 64, CH = 8;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *d = sm.d;
    // rows: sum_{j <= i} h_ij v_j; 8 columns per batch of loads, the next
    // batch in flight while the current one is used
    for (int i0 = wave * 64; i0 < n; i0 += NT) {
        const int i = i0 + lane;
        const int jmax = min(i0 + 63, n - 1);
        const double di = (i < n) ? d[i] : 0.0;
        double acc = 0.0, ra = 0.0;
        double a[CH], an[CH];
        auto load = [&](double *dst, int j0) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int j = j0 + u;
                dst[u] = (i < n && j <= i) ? A[i + (int64_t)j * n] : 0.0;
            }
        };
        load(a, 0);
        for (int j0 = 0; j0 <= jmax; j0 += CH) {
            if (j0 + CH <= jmax)
                load(an, j0 + CH);
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int j = min(j0 + u, n - 1);
                const double h = (di * a[u]) * d[j];
                acc = fma(h, v[j], acc);
                if (first && i < n && j0 + u < i) {
                    ra += fabs(h);
                    hmax = fmax(hmax, fabs(h));
                    fro += 2.0 * h * h;
                } else if (first && i < n && j0 + u == i) {
                    fro += h * h;
                }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) a[u] = an[u];
        }
        if (i < n) {
            y[i] = acc;
            if (first)
                sm.rs[i] = ra;
        }
    }
    // columns: lane = column, sum_{i > j} h_ij v_i, the same double buffering
    for (int j0 = wave * 64; j0 < n; j0 += NT) {
        const int j = j0 + lane;
        const double dj = (j < n) ? d[j] : 0.0;
        double acc = 0.0, ca = 0.0;
        double a[CH], an[CH];
        auto load = [&](double *dst, int i0) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int i = i0 + u;
                dst[u] = (j < n && i > j && i < n) ? A[i + (int64_t)j * n] : 0.0;
            }
        };
        load(a, j0 + 1);
        for (int i0 = j0 + 1; i0 < n; i0 += CH) {
            if (i0 + CH < n)
                load(an, i0 + CH);
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int i = min(i0 + u, n - 1);
                const double h = (d[i] * a[u]) * dj;
                acc = fma(h, v[i], acc);
                if (first)
                    ca += fabs(h);
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) a[u] = an[u];
        }
        if (j < n) {
            sm.ycol[j] = acc;
            if (first)
                sm.rcol[j] = ca;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) {
        y[i] += sm.ycol[i];
        if (first)
            sm.rs[i] += sm.rcol[i];
    }
    __syncthreads();
}

// eigenvalues (ascending) of the k x k symmetric tridiagonal (al, be), k <= 4
SPD_DEV int sturm_below(const double *al, const double *be, int k, double x)
{
    int c = 0;
    double q = al[0] - x;
    if (q < 0)
        ++c;
    for (int i = 1; i < k; ++i) {
        if (q == 0.0)
            q = 1e-300;
        q = (al[i] - x) - be[i - 1] * be[i - 1] / q;
        if (q < 0)
            ++c;
    }
    return c;
}

// Ritz value q (0-based, ascending) of the k x k tridiagonal (al, be) by
// multisection in one wavefront: each step evaluates the Sturm count at 64
// interior points of [lo, hi] and keeps the subinterval where the count
// passes q, until no representable point lies strictly inside.  Every lane
// returns the same value.
SPD_DEV double ritz_multisect(const double *al, const double *be, int k, int q, double lo, double hi)
{
    const int lane = threadIdx.x & 63;
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
        const bool above = (x > lo && x < hi) ? sturm_below(al, be, k, x) > q : false;
        const unsigned long long mk = __ballot(above);
        // x_l is increasing in l; the count is non-decreasing in x
        const int first = mk ? __builtin_ctzll(mk) : 64;
        const double xlo = __shfl(x, first > 0 ? first - 1 : 0), xhi = __shfl(x, first < 64 ? first : 63);
        const double nlo = (first > 0) ? fmax(lo, xlo) : lo;
        const double nhi = (first < 64) ? fmin(hi, xhi) : hi;
        if (nlo == lo && nhi == hi)
            break;  // the grid collapsed onto the ends: no interior point left
        lo = nlo;
        hi = nhi;
    }
    return 0.5 * (lo + hi);
}

template <int WAVES>
SPD_DEV void b_features(const double *A, int n, int m, PickSmem &sm)
{
    constexpr int NT = WAVES * 64, K = PICK_LANCZOS;
    const int tid = threadIdx.x;
    double *d = sm.d, *v = sm.v, *vp = sm.vp, *w = sm.w;
    // diagonal statistics
    double st[3] = {0.0, -1e300, 1e300};  // sum, max, min of log10|a_ii|
    const int ops3[3] = {0, 1, 2};
    for (int i = tid; i < n; i += NT) {
        const double a = A[i + (int64_t)i * n];
        d[i] = (a > 0.0) ? 1.0 / sqrt(a) : 1.0;
        const double la = log10(fmax(fabs(a), 1e-300));
        st[0] += la;
        st[1] = fmax(st[1], la);
        st[2] = fmin(st[2], la);
        v[i] = 1.0 / sqrt((double)n);
        vp[i] = 0.0;
    }
    b_reduce<WAVES, 3>(st, ops3, sm);
    const double mean_la = st[0] / n;
    double sq[1] = {0.0};
    const int ops1[1] = {0};
    for (int i = tid; i < n; i += NT) {
        const double la = log10(fmax(fabs(A[i + (int64_t)i * n]), 1e-300)) - mean_la;
        sq[0] += la * la;
    }
    b_reduce<WAVES, 1>(sq, ops1, sm);
    // Lanczos; the first product also yields the Gershgorin radii and |H| stats
    double al[K], be[K];
    int k = 0;
    bool early = false;
    double hmax = 0.0, fro = 0.0;
    double bprev = 0.0;
    for (int j = 0; j < K; ++j) {
        b_hv<WAVES>(A, n, v, w, j == 0, hmax, fro, sm);
        double a1[1] = {0.0};
        for (int i = tid; i < n; i += NT) a1[0] += w[i] * v[i];
        b_reduce<WAVES, 1>(a1, ops1, sm);
        const double alpha = a1[0];
        double b2[1] = {0.0};
        for (int i = tid; i < n; i += NT) {
            const double x = (w[i] - alpha * v[i]) - bprev * vp[i];
            w[i] = x;
            b2[0] += x * x;
        }
        b_reduce<WAVES, 1>(b2, ops1, sm);
        const double beta = sqrt(b2[0]);
        al[j] = alpha;
        k = j + 1;
        if (j == K - 1) {
            be[j] = beta;
            break;
        }
        if (beta <= 1e-12 * fmax(fabs(alpha), 1.0)) {
            be[j] = 0.0;
            early = true;
            break;
        }
        be[j] = beta;
        for (int i = tid; i < n; i += NT) {
            vp[i] = v[i];
            v[i] = w[i] / beta;
        }
        bprev = beta;
        __syncthreads();
    }
    // Gershgorin statistics of H and the |H| statistics (first product)
    double gs[5] = {-1e300, 0.0, 0.0, hmax, fro};  // max r, sum r, count r < 1, max |h|, ||H||_F^2
    const int ops5[5] = {1, 0, 0, 1, 0};
    for (int i = tid; i < n; i += NT) {
        gs[0] = fmax(gs[0], sm.rs[i]);
        gs[1] += sm.rs[i];
        gs[2] += (sm.rs[i] < 1.0) ? 1.0 : 0.0;
    }
    b_reduce<WAVES, 5>(gs, ops5, sm);
    // Ritz values: wave q finds the q-th (al, be and k are the same in every thread)
    const int wave = tid >> 6;
    double lo = al[0], hi = al[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < k ? fabs(be[i]) : 0.0);
        lo = fmin(lo, al[i] - r);
        hi = fmax(hi, al[i] + r);
    }
    for (int q = wave; q < k; q += WAVES) {
        const double t = ritz_multisect(al, be, k, q, lo, hi);
        if ((tid & 63) == 0)
            sm.th[q] = t;
    }
    __syncthreads();
    if (tid == 0) {
        double th[K];
        for (int q = 0; q < k; ++q) th[q] = sm.th[q];
        const double tmin = th[0], tmax = th[k - 1];
        double f[PICK_NFEAT];
        f[0] = log2((double)n) / 9.0;
        f[1] = m / 8.0;
        f[2] = (st[1] - st[2]) / 6.0;
        f[3] = mean_la / 6.0;
        f[4] = sqrt(sq[0] / n) / 3.0;
        f[5] = log10(1.0 + gs[0]) / 3.0;
        f[6] = log10(1.0 + gs[1] / n) / 3.0;
        f[7] = gs[2] / n;
        f[8] = fmin(fmax(1.0 - gs[0], -10.0), 1.0) / 10.0;
        f[9] = log10(tmax) / 3.0;
        f[10] = log10(fmax(tmin, 1e-16)) / 6.0;
        f[11] = log10(tmax / fmax(tmin, 1e-16)) / 6.0;
        f[12] = (n > 1) ? gs[3] : 0.0;
        f[13] = log10(sqrt(gs[4]) / sqrt((double)n)) / 3.0;
        f[14] = early ? 0.0 : be[k - 1] / tmax;
        f[15] = (k >= 3 && tmax > th[0]) ? (th[1] - th[0]) / (tmax - th[0]) : 0.0;
        for (int q = 0; q < PICK_NFEAT; ++q) sm.feat[q] = (float)f[q];
    }
    __syncthreads();
}

// the perceptron on sm.feat: class with the largest logit (the first on ties)
SPD_DEV int b_pick(const float *P, PickSmem &sm)
{
    const float *W1 = P, *b1 = W1 + PICK_NH * PICK_NFEAT, *W2 = b1 + PICK_NH, *b2 = W2 + PICK_NH * PICK_NH,
                *W3 = b2 + PICK_NH, *b3 = W3 + PICK_NCLS * PICK_NH;
    const int t = threadIdx.x;
    if (t < PICK_NH) {
        float z = b1[t];
        for (int k = 0; k < PICK_NFEAT; ++k) z += W1[t * PICK_NFEAT + k] * sm.feat[k];
        sm.hid[0][t] = fmaxf(z, 0.0f);
    }
    __syncthreads();
    if (t < PICK_NH) {
        float z = b2[t];
        for (int k = 0; k < PICK_NH; ++k) z += W2[t * PICK_NH + k] * sm.hid[0][k];
        sm.hid[1][t] = fmaxf(z, 0.0f);
    }
    __syncthreads();
    if (t < PICK_NCLS) {
        float z = b3[t];
        for (int k = 0; k < PICK_NH; ++k) z += W3[t * PICK_NH + k] * sm.hid[1][k];
        sm.logit[t] = z;
    }
    __syncthreads();
    int best = 0;
    for (int c = 1; c < PICK_NCLS; ++c)
        if (sm.logit[c] > sm.logit[best])
            best = c;
    __syncthreads();
    return best;
}


// Refinement at the precision of the current factor (T), from the iterate in
// X (the first solve); the single-system path's stopping rule: a column is
// done once eta <= tol and its last correction z_k (zeta_k = ||z_k|| /
// ||x_{k+1}||, rho_k = zeta_k / zeta_{k-1}, eta_k the backward error it was
// solved from) shows x accurate to binary64 level -- eta = 0 or
// zeta_k <= 2^-53; rho_k < 1/2 and rho_k/(1-rho_k) eta_k <= 2^-53; or
// rho_k >= 1/2 and eta_k <= 2^-51.  A binary64 factor's first solve is
// accepted at eta <= tol.  Divergence as before; max_iter corrections
// without success: no convergence.  Returns SPD_OK or SPD_ERR_NO_CONVERGENCE
// and fills the iteration counts and eta.
template <typename T, int WAVES>
SPD_DEV int b_refine(const BatchArgs &a, const double *A, const double *B, double *X, int n, int np, int m,
                     const BatchWs &w, double mu, spd_report &rep, SolveSmem &sm)
{
    constexpr double U = 0x1p-53, FLOOR = 0x1p-51;
    constexpr bool STABLE = sizeof(T) == 8;
    rep.iters_low = 1;
    rep.iters_high = 0;
    constexpr int MR = SPD_BATCH_MAXRHS;
    double eta0 = 0.0, anorm = 0.0;
    // identical in every thread
    double eta[MR], eprev[MR], zeta[MR], zprev[MR];
    bool done[MR];
#pragma unroll
    for (int c = 0; c < MR; ++c) {
        zeta[c] = zprev[c] = 1.0;
        eprev[c] = 0.0;
        done[c] = false;
    }
    int stalls = 0;
    for (;;) {
        const int first = (rep.iters_high == 0);
        const int k = rep.iters_high;  // corrections applied so far
        b_residual<WAVES>(A, w.Am, n, np, m, X, B, w.d, w.R, first, sm);
        rep.iters_high++;
        if (first)
            anorm = sm.norms[0];
        bool finite = isfinite(anorm), all = true;
        double worst = 0.0;
#pragma unroll
        for (int c = 0; c < MR; ++c) {
            if (c >= m)
                break;
            const double rn = sm.norms[1 + c], xn = sm.norms[1 + m + c], bn = sm.norms[1 + 2 * m + c];
            const double den = anorm * xn + bn;
            double v = (den > 0.0) ? rn / den : (rn > 0.0 ? __builtin_inf() : 0.0);
            if (!(rn == rn) || !(xn == xn))
                v = __builtin_nan("");
            eta[c] = v;
            if (!isfinite(v))
                finite = false;
            if (v > worst)
                worst = v;
            if (k > 0) {
                const double zn = __longlong_as_double((long long)sm.zmax[c]);
                zeta[c] = (zn == 0.0) ? 0.0 : zn / xn;
            }
            if (!done[c] && v <= a.tol) {
                if (v == 0.0 || zeta[c] <= U) {
                    done[c] = true;
                } else if (k == 0) {
                    done[c] = STABLE;
                } else {
                    const double rho = zeta[c] / zprev[c];
                    done[c] = (rho < 0.5) ? (rho / (1.0 - rho)) * eprev[c] <= U : eprev[c] <= FLOOR;
                }
            }
            all = all && done[c];
        }
        rep.eta = finite ? worst : __builtin_nan("");
        if (!finite)
            return SPD_ERR_NO_CONVERGENCE;
        if (all && worst <= a.tol)
            return SPD_OK;
        if (k == 0) {
            eta0 = worst;
        } else {
            bool all_slow = true;
#pragma unroll
            for (int c = 0; c < MR; ++c)
                if (c < m && !(eta[c] > 0.9 * eprev[c]))
                    all_slow = false;
            stalls = all_slow ? stalls + 1 : 0;
            if (worst > a.tol && (worst > eta0 || stalls >= 2))
                return SPD_ERR_NO_CONVERGENCE;
        }
        if (rep.iters_low > a.max_iter)
            return SPD_ERR_NO_CONVERGENCE;
#pragma unroll
        for (int c = 0; c < MR; ++c) {
            eprev[c] = eta[c];
            zprev[c] = zeta[c];
        }
        __syncthreads();
        if (threadIdx.x < m)
            sm.smax[threadIdx.x] = sm.norms[1 + 3 * m + threadIdx.x];
        __syncthreads();
        b_solve<T, WAVES>((const T *)w.L, (const T *)w.Winv, n, np, m, w.R, w.d, mu, X, 1, sm);
        rep.iters_low++;
    }
}

// smax[c] = max_i |d_i B[i][c]| (the first solve's scaling)
template <int WAVES>
SPD_DEV void b_rhs_max(const double *B, const double *d, int n, int m, SolveSmem &sm)
{
    double v[SPD_BATCH_MAXRHS];
#pragma unroll
    for (int c = 0; c < SPD_BATCH_MAXRHS; ++c) v[c] = 0.0;
    for (int i = threadIdx.x; i < n; i += WAVES * 64)
#pragma unroll
        for (int c = 0; c < SPD_BATCH_MAXRHS; ++c)
            if (c < m)
                v[c] = b_nanmax(v[c], fabs(d[i] * B[i + (int64_t)c * n]));
#pragma unroll
    for (int c = 0; c < SPD_BATCH_MAXRHS; ++c) {
        for (int off = 32; off > 0; off >>= 1) v[c] = b_nanmax(v[c], __shfl_xor(v[c], off));
        if ((threadIdx.x & 63) == 0)
            sm.red[threadIdx.x >> 6][c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < m) {
        double x = 0.0;
        for (int q = 0; q < WAVES; ++q) x = b_nanmax(x, sm.red[q][threadIdx.x]);
        sm.smax[threadIdx.x] = x;
    }
    __syncthreads();
}

// Factor in the factor type T at precision p (binary32 factor for BF16, FP16,
// FP32: equilibrated, mu for FP16, rounded update operands for the half
// formats; binary64 factor of A itself for FP64).  Returns the 1-based
// failing column (0 on success).
template <typename T, int WAVES>
SPD_DEV int b_factor_p(const BatchArgs &a, const double *A, int n, int np, const BatchWs &w, int p, double &mu,
                       SolveSmem &sm)
{
    if constexpr (sizeof(T) == 8) {
        mu = 1.0;
        b_convert<double, WAVES>(A, n, np, w.d, 1.0, 0, (double *)w.L, w.Am, sm);
        return b_factor<double, WAVES>((double *)w.L, np, (double *)w.Winv, HALF_NONE, sm);
    } else {
        mu = (p == SPD_FP16) ? a.mu16 : 1.0;
        b_convert<float, WAVES>(A, n, np, w.d, mu, a.equilibrate, (float *)w.L, w.Am, sm);
        const int half = (p == SPD_FP16) ? HALF_F16 : (p == SPD_BF16) ? HALF_BF16 : HALF_NONE;
        return b_factor<float, WAVES>((float *)w.L, np, (float *)w.Winv, half, sm);
    }
}

// One system through Algorithm 1 by one workgroup, at the precisions of the
// kernel's factor type: HI = false takes BF16, FP16 and FP32 requests (and
// the half -> binary32 fallback), HI = true the FP64 requests and every
// system the low-precision kernel handed over (a binary32 breakdown or
// non-convergence with fallback on: prec[s] = FP64, reps[s].fallbacks the
// count so far).  Systems of the other kernel are skipped; the
// low-precision kernel also reports invalid sizes.  ticks[s] (zeroed by the
// order kernel) accumulates every kernel's time on the system.
template <int WAVES, bool HI>
SPD_DEV void b_system(const BatchArgs &a, int64_t s, SolveSmem &sm)
{
    using T = typename std::conditional<HI, double, float>::type;
    const int n = a.n[s], m = a.nrhs[s];
    int p = a.prec[s];
    if (p == SPD_AUTO)
        p = SPD_FP32;
    const bool valid = n >= 0 && m >= 0 && n <= SPD_BATCH_NMAX && m <= SPD_BATCH_MAXRHS && p >= SPD_BF16 &&
                       p <= SPD_FP64;
    if (HI ? (!valid || p != SPD_FP64) : (valid && p == SPD_FP64)) {
        // the other kernel's system; the low-precision kernel starts its count
        if (!HI && threadIdx.x == 0)
            a.reps[s].fallbacks = 0;
        return;
    }
    const unsigned long long t0 = wall_clock64();
    spd_report rep;
    rep.status = SPD_OK;
    rep.prec_used = p;
    rep.iters_low = rep.iters_high = 0;
    rep.fallbacks = HI ? a.reps[s].fallbacks : 0;
    rep.info = 0;
    rep.eta = 0.0;
    bool handover = false;
    if (!valid) {
        rep.status = SPD_ERR_INVALID_ARG;
    } else if (n > 0 && m > 0) {
        const double *A = a.A + a.a_off[s];
        const double *B = a.B + a.b_off[s];
        double *X = a.X + a.b_off[s];
        const int np = ((n + BNB - 1) / BNB) * BNB;
        const BatchWs w = batch_ws(a);
        double mu = 1.0;
        int status = SPD_OK;
        for (;;) {
            const int info = b_factor_p<T, WAVES>(a, A, n, np, w, p, mu, sm);
            rep.info = info;
            rep.prec_used = p;
            int r;
            if (info) {
                r = SPD_ERR_NOT_SPD;
            } else {
                // first solve from B, then refinement
                b_rhs_max<WAVES>(B, w.d, n, m, sm);
                b_solve<T, WAVES>((const T *)w.L, (const T *)w.Winv, n, np, m, B, w.d, mu, X, 0, sm);
                r = b_refine<T, WAVES>(a, A, B, X, n, np, m, w, mu, rep, sm);
            }
            if (r == SPD_OK || !a.fallback || HI) {
                status = r;
                break;
            }
            // fallback: a half format retries in binary32 here; binary32 goes
            // to the binary64 kernel
            rep.fallbacks++;
            if (p == SPD_FP32) {
                handover = true;
                status = r;
                break;
            }
            p = SPD_FP32;
        }
        rep.status = status;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (handover) {
            a.reps[s].fallbacks = rep.fallbacks;
            a.prec[s] = SPD_FP64;
        } else {
            a.reps[s] = rep;
            a.prec[s] = rep.prec_used;
        }
        if (a.ticks)
            a.ticks[s] += (int64_t)(wall_clock64() - t0);
    }
}

// The precision picker for SPD_AUTO systems: features and perceptron by one
// workgroup per system; prec[s] becomes the chosen class.
__global__ __launch_bounds__(256, 3) void k_batch_pick(BatchArgs a)
{
    __shared__ PickSmem sm;
    __shared__ int s_q;
    for (;;) {
        if (threadIdx.x == 0)
            s_q = atomicAdd(a.queue + 0, 1);
        __syncthreads();
        const int64_t q = s_q;
        if (q >= a.batch)
            return;
        const int64_t s = a.order[q];
        const int n = a.n[s], m = a.nrhs[s];
        if (a.prec[s] == SPD_AUTO && n > 0 && m > 0 && n <= SPD_BATCH_NMAX && m <= SPD_BATCH_MAXRHS) {
            const unsigned long long t0 = wall_clock64();
            b_features<4>(a.A + a.a_off[s], n, m, sm);
            const int p = b_pick(a.picker, sm);
            if (threadIdx.x == 0) {
                a.prec[s] = p;
                if (a.ticks)
                    a.ticks[s] += (int64_t)(wall_clock64() - t0);
            }
        }
        __syncthreads();
    }
}

template <int WAVES, bool HI>
__global__ __launch_bounds__(WAVES * 64, 2) void k_batch(BatchArgs a)
{
    __shared__ SolveSmem sm;
    __shared__ int s_q;
    for (;;) {
        if (threadIdx.x == 0)
            s_q = atomicAdd(a.queue + (HI ? 2 : 1), 1);
        __syncthreads();
        const int64_t q = s_q;
        if (q >= a.batch)
            return;
        b_system<WAVES, HI>(a, a.order[q], sm);
        __syncthreads();
    }
}

// Features of every system (one workgroup each), for training the picker.
__global__ __launch_bounds__(256) void k_features(int64_t batch, const int32_t *__restrict__ n,
                                                  const int32_t *__restrict__ nrhs, const int64_t *__restrict__ a_off,
                                                  const double *__restrict__ A, float *__restrict__ feat)
{
    __shared__ PickSmem sm;
    for (int64_t s = blockIdx.x; s < batch; s += gridDim.x) {
        const int ns = n[s], ms = nrhs[s];
        if (ns >= 1 && ns <= SPD_BATCH_NMAX) {
            b_features<4>(A + a_off[s], ns, ms, sm);
            if (threadIdx.x < PICK_NFEAT)
                feat[s * PICK_NFEAT + threadIdx.x] = sm.feat[threadIdx.x];
        } else if (threadIdx.x < PICK_NFEAT) {
            feat[s * PICK_NFEAT + threadIdx.x] = 0.0f;
        }
        __syncthreads();
    }
}

// Order of work: systems sorted by decreasing n (counting sort, one
// workgroup); also clears the work-queue counter.
__global__ __launch_bounds__(1024) void k_batch_order(int64_t batch, const int32_t *__restrict__ n,
                                                      int32_t *__restrict__ order, int *queue, int64_t *ticks)
{
    constexpr int NBIN = SPD_BATCH_NMAX + 1;
    __shared__ int hist[NBIN], start[NBIN];
    const int tid = threadIdx.x;
    for (int b = tid; b < NBIN; b += 1024) hist[b] = 0;
    __syncthreads();
    for (int64_t s = tid; s < batch; s += 1024) {
        int v = n[s];
        v = (v < 0 || v > SPD_BATCH_NMAX) ? 0 : v;
        atomicAdd(&hist[SPD_BATCH_NMAX - v], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int b = 0; b < NBIN; ++b) {
            start[b] = acc;
            acc += hist[b];
        }
        queue[0] = queue[1] = queue[2] = 0;
    }
    if (ticks)
        for (int64_t s = tid; s < batch; s += 1024) ticks[s] = 0;
    __syncthreads();
    for (int64_t s = tid; s < batch; s += 1024) {
        int v = n[s];
        v = (v < 0 || v > SPD_BATCH_NMAX) ? 0 : v;
        const int pos = atomicAdd(&start[SPD_BATCH_NMAX - v], 1);
        order[pos] = (int32_t)s;
    }
}

namespace spd {

int64_t batch_ws_stride()
{
    int64_t b = (int64_t)SPD_BATCH_NMAX * SPD_BATCH_NMAX * 8 + (int64_t)SPD_BATCH_NMAX * BNB * 8 +
                (int64_t)SPD_BATCH_NMAX * 8 + (int64_t)SPD_BATCH_NMAX * SPD_BATCH_MAXRHS * 8 +
                (int64_t)SPD_BATCH_NMAX * SPD_BATCH_NMAX * 8;
    return (b + 255) / 256 * 256;
}

hipError_t launch_batch(const BatchLaunch &l, hipStream_t st)
{
    BatchArgs a;
    a.batch = l.batch;
    a.n = l.n;
    a.nrhs = l.nrhs;
    a.a_off = l.a_off;
    a.b_off = l.b_off;
    a.A = l.A;
    a.B = l.B;
    a.X = l.X;
    a.prec = l.prec;
    a.reps = l.reps;
    a.tol = l.tol;
    a.mu16 = l.mu16;
    a.max_iter = l.max_iter;
    a.fallback = l.fallback;
    a.equilibrate = l.equilibrate;
    a.order = l.order;
    a.queue = l.queue;
    a.ws = (char *)l.ws;
    a.ws_stride = batch_ws_stride();
    a.picker = l.picker;
    a.ticks = l.ticks;
    hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, st, l.batch, l.n, l.order, l.queue, l.ticks);
    // picker (AUTO systems), then the low-precision systems, then binary64
    // (requests and hand-overs); four wavefronts per workgroup
    if (l.picker)
        hipLaunchKernelGGL(k_batch_pick, dim3((unsigned)l.grid), dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_batch<4, false>), dim3((unsigned)l.grid), dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_batch<4, true>), dim3((unsigned)l.grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

void launch_features(int64_t batch, const int32_t *n, const int32_t *nrhs, const int64_t *a_off, const double *A,
                     float *feat, hipStream_t st)
{
    if (batch <= 0) return;
    const unsigned grid = (unsigned)(batch < 2048 ? batch : 2048);
    hipLaunchKernelGGL(k_features, dim3(grid), dim3(256), 0, st, batch, n, nrhs, a_off, A, feat);
}

}  // namespace spd
