// Binary64 residual R = B - A X and the norms of the backward error
// (Algorithm 1's residual steps, the ones it carries out in high precision).
//
// A is symmetric with only its lower triangle stored.  Workgroup (I, s) owns
// the 64-row block I and visits the 64-column blocks J = s, s + S, ...; each
// 64 x 64 tile of the full symmetric matrix is formed in LDS from the lower
// triangle (directly for J < I, transposed for J > I, mirrored for J == I)
// and multiplied by the matching rows of X.  Per-(s, row) partial sums are
// reduced in a fixed order by k_resid_reduce, so results are bitwise
// reproducible run to run.  The same pass can accumulate sum_j |a_ij| for
// ||A||_inf.
#include "common.h"
#include "internal.h"
#include <algorithm>

template <int MC, int RB, int CB, int JS>
__global__ __launch_bounds__(256) void k_resid_partial(const double *__restrict__ A, int64_t lda, int64_t n,
                                                       const double *__restrict__ X, int64_t ldx, int m, int c0, int S,
                                                       double *__restrict__ P, double *__restrict__ Pabs, int want_abs)
{
    constexpr int RG = 64 / RB, CG = MC / CB;
    static_assert(RG * CG * JS == 256, "thread layout");
    constexpr int TS = 65;
    __shared__ double Ts[64 * TS];
    __shared__ double Xs[MC * 64];
    const int tid = threadIdx.x;
    const int rg = tid % RG, cg = (tid / RG) % CG, js = tid / (RG * CG);
    const int I = blockIdx.x, s = blockIdx.y;
    const int64_t i0 = (int64_t)I * 64;
    const int nrb = (int)((n + 63) / 64);
    double acc[RB][CB];
    double aabs[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        aabs[r] = 0.0;
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[r][c] = 0.0;
    }
    const bool do_abs = want_abs && cg == 0;
    for (int J = s; J < nrb; J += S) {
        const int64_t j0 = (int64_t)J * 64;
        __syncthreads();
        if (J < I) {
            for (int idx = tid; idx < 4096; idx += 256) {
                const int i = idx & 63, j = idx >> 6;
                const int64_t gi = i0 + i, gj = j0 + j;
                Ts[j * TS + i] = (gi < n && gj < n) ? A[gi + gj * lda] : 0.0;
            }
        } else if (J > I) {
            for (int idx = tid; idx < 4096; idx += 256) {
                const int j = idx & 63, i = idx >> 6;
                const int64_t gi = i0 + i, gj = j0 + j;
                Ts[j * TS + i] = (gi < n && gj < n) ? A[gj + gi * lda] : 0.0;
            }
        } else {
            for (int idx = tid; idx < 4096; idx += 256) {
                const int i = idx & 63, j = idx >> 6;
                const int64_t gi = i0 + i, gj = j0 + j;
                Ts[j * TS + i] = (i >= j && gi < n && gj < n) ? A[gi + gj * lda] : 0.0;
            }
            __syncthreads();
            for (int idx = tid; idx < 4096; idx += 256) {
                const int i = idx & 63, j = idx >> 6;
                if (i < j)
                    Ts[j * TS + i] = Ts[i * TS + j];
            }
        }
        for (int idx = tid; idx < MC * 64; idx += 256) {
            const int j = idx & 63, c = idx >> 6;
            const int64_t gj = j0 + j;
            Xs[c * 64 + j] = (gj < n && c0 + c < m) ? X[gj + (int64_t)(c0 + c) * ldx] : 0.0;
        }
        __syncthreads();
        constexpr int JW = 64 / JS;
#pragma unroll 4
        for (int jj = 0; jj < JW; ++jj) {
            const int j = js * JW + jj;
            double a[RB], x[CB];
#pragma unroll
            for (int r = 0; r < RB; ++r) a[r] = Ts[j * TS + rg + RG * r];
#pragma unroll
            for (int c = 0; c < CB; ++c) x[c] = Xs[(cg * CB + c) * 64 + j];
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) acc[r][c] = fma(a[r], x[c], acc[r][c]);
            if (do_abs)
#pragma unroll
                for (int r = 0; r < RB; ++r) aabs[r] += fabs(a[r]);
        }
    }
    // combine the JS partial sums (fixed order) and store
    __syncthreads();
    double *red = Ts;  // reuse: JS * MC * 64 <= 64 * TS doubles
    if (JS > 1) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CB; ++c)
                red[(js * MC + cg * CB + c) * 64 + rg + RG * r] = acc[r][c];
    }
    __shared__ double redabs[JS * 64];
    if (do_abs)
#pragma unroll
        for (int r = 0; r < RB; ++r) redabs[js * 64 + rg + RG * r] = aabs[r];
    __syncthreads();
    if (js == 0) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = rg + RG * r;
            const int64_t gi = i0 + i;
            if (gi >= n)
                continue;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int cc = cg * CB + c;
                double v = acc[r][c];
                for (int q = 1; q < JS; ++q)
                    v += red[(q * MC + cc) * 64 + i];
                if (c0 + cc < m)
                    P[((int64_t)s * m + c0 + cc) * n + gi] = v;
            }
            if (do_abs) {
                double v = aabs[r];
                for (int q = 1; q < JS; ++q)
                    v += redabs[q * 64 + i];
                Pabs[(int64_t)s * n + gi] = v;
            }
        }
    }
}

// The same partial sums for 9..32 right-hand sides per chunk on binary64
// MFMA (v_mfma_f64_16x16x4f64): wave w owns rows 16 w .. 16 w + 15 of the
// tile and NT column tiles of 16; per k-step of 4 a lane feeds A(i, k) with
// i = lane % 16, k = lane / 16 from the LDS tile and X(k, c) with
// c = lane % 16 from the LDS copy of X (pitch 65: conflict-free columns).
// The accumulator holds row lane / 16 + 4 r, column lane % 16 in register r
// (the binary64 layout, unlike the binary32 16 x 16 one).
typedef double doublex4 __attribute__((ext_vector_type(4)));
template <int NT>
__global__ __launch_bounds__(256) void k_resid_mfma(const double *__restrict__ A, int64_t lda, int64_t n,
                                                    const double *__restrict__ X, int64_t ldx, int m, int c0, int S,
                                                    double *__restrict__ P, double *__restrict__ Pabs, int want_abs)
{
    constexpr int MC = 16 * NT, TS = 65, XU = MC * 64 / 256;
    __shared__ double Ts[64 * TS];
    __shared__ double Xs[MC * TS];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int I = blockIdx.x, s = blockIdx.y;
    const int64_t i0 = (int64_t)I * 64;
    const int nrb = (int)((n + 63) / 64);
    doublex4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    double aabs = 0.0;
    // The next tile's values are loaded into registers while the current
    // tile is multiplied.  Element u of a thread: idx = tid + 256 u; for a
    // tile left of the diagonal (and the diagonal tile, lower part only)
    // i = idx % 64, j = idx / 64 read along A's column j; right of it
    // j = idx % 64, i = idx / 64 read along A's column i (the transpose).
    double av[16], xv[XU];
    auto fetch = [&](int J) {
        const int64_t j0 = (int64_t)J * 64;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u;
            double v = 0.0;
            if (J <= I) {
                const int i = idx & 63, j = idx >> 6;
                const int64_t gi = i0 + i, gj = j0 + j;
                if (gi < n && gj < n && (J < I || i >= j)) v = A[gi + gj * lda];
            } else {
                const int j = idx & 63, i = idx >> 6;
                const int64_t gi = i0 + i, gj = j0 + j;
                if (gi < n && gj < n) v = A[gj + gi * lda];
            }
            av[u] = v;
        }
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int idx = tid + 256 * u;
            const int j = idx & 63, c = idx >> 6;
            const int64_t gj = j0 + j;
            xv[u] = (gj < n && c0 + c < m) ? X[gj + (int64_t)(c0 + c) * ldx] : 0.0;
        }
    };
    if (s < nrb) fetch(s);
    for (int J = s; J < nrb; J += S) {
        __syncthreads();  // the previous tile has been consumed
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u;
            if (J <= I)
                Ts[(idx >> 6) * TS + (idx & 63)] = av[u];
            else
                Ts[(idx & 63) * TS + (idx >> 6)] = av[u];
        }
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int idx = tid + 256 * u;
            Xs[(idx >> 6) * TS + (idx & 63)] = xv[u];
        }
        if (J == I) {  // mirror the lower triangle of the diagonal tile
            __syncthreads();
            for (int idx = tid; idx < 4096; idx += 256) {
                const int i = idx & 63, j = idx >> 6;
                if (i < j)
                    Ts[j * TS + i] = Ts[i * TS + j];
            }
        }
        __syncthreads();
        if (J + S < nrb) fetch(J + S);  // in flight during the products below
        if (want_abs && tid < 64)
            for (int j = 0; j < 64; ++j) aabs += fabs(Ts[j * TS + tid]);
#pragma unroll 4
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const double a = Ts[(k0 + kq) * TS + 16 * w + r16];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double b = Xs[(16 * t + r16) * TS + k0 + kq];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gi = i0 + 16 * w + kq + 4 * r;
            const int c = 16 * t + r16;
            if (gi < n && c0 + c < m) P[((int64_t)s * m + c0 + c) * n + gi] = acc[t][r];
        }
    if (want_abs && tid < 64 && i0 + tid < n) Pabs[(int64_t)s * n + i0 + tid] = aabs;
}

// Single pass over the lower triangle for a few right-hand sides.  Workgroup
// (J, q) walks tiles I = J + q CH .. of the 64-column strip J (contiguous in
// memory); wave w holds columns 16 w .. 16 w + 15 of the tile, lane l its row
// l.  Each stored a_ij (i > j) serves twice: a_ij x_j for row i (a row partial
// per tile, RP[I][J]) and a_ij x_i for row j (accumulated over the chunk in
// registers, CP[J][q]); a diagonal tile uses its lower triangle only (the
// diagonal once).  k_resid_sym_reduce then sums, per row of block I,
// RP[I][0..I] (as four interleaved sums) and CP[I][0..Q), in a fixed order.  With want_abs an extra
// "column" c = MC carries |a_ij| (row sums of |A|).
#define RSYM_CH 16
template <int MC, bool WA>
__global__ __launch_bounds__(256) void k_resid_sym(const double *__restrict__ A, int64_t lda, int64_t n,
                                                   const double *__restrict__ X, int64_t ldx, int m, int Q,
                                                   double *__restrict__ RP, double *__restrict__ CP)
{
    constexpr int NC = MC + 1;  // partial "columns" in the layout: MC right-hand sides + |A|
    constexpr int NA = WA ? NC : MC;  // the ones this variant computes
    constexpr bool want_abs = WA;
    __shared__ double xs[MC][64];
    __shared__ double red[4][NA][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int J = blockIdx.x, q = blockIdx.y;
    const int nrb = (int)((n + 63) / 64);
    const int I0 = J + q * RSYM_CH, I1 = min(I0 + RSYM_CH, nrb);
    if (I0 >= nrb)
        return;
    const int64_t j0 = (int64_t)J * 64;
    // x of the strip's columns, for the row partials
    for (int idx = threadIdx.x; idx < MC * 64; idx += 256) {
        const int c = idx / 64, j = idx % 64;
        xs[c][j] = (j0 + j < n && c < m) ? X[(j0 + j) + (int64_t)c * ldx] : 0.0;
    }
    __syncthreads();
    double cacc[16][NA];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
#pragma unroll
        for (int c = 0; c < NA; ++c) cacc[jj][c] = 0.0;
    // tile loads run one tile ahead of the arithmetic
    double an[16];
    auto load_tile = [&](int I) {
        const int64_t gi = (int64_t)I * 64 + lane;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int64_t gj = j0 + 16 * w + jj;
            an[jj] = (gi < n && gj < n) ? A[gi + gj * lda] : 0.0;
        }
    };
    load_tile(I0);
    for (int I = I0; I < I1; ++I) {
        const int64_t gi = (int64_t)I * 64 + lane;
        double a[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) a[jj] = an[jj];
        if (I + 1 < I1)
            load_tile(I + 1);
        if (I == J) {
#pragma unroll
            for (int jj = 0; jj < 16; ++jj)
                if (lane < 16 * w + jj)
                    a[jj] = 0.0;
        }
        double xi[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) xi[c] = (gi < n && c < m) ? X[gi + (int64_t)c * ldx] : 0.0;
        double racc[NA];
#pragma unroll
        for (int c = 0; c < NA; ++c) racc[c] = 0.0;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const bool strict = (I != J) || (lane > 16 * w + jj);
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                racc[c] = fma(a[jj], xs[c][16 * w + jj], racc[c]);
                if (strict)
                    cacc[jj][c] = fma(a[jj], xi[c], cacc[jj][c]);
            }
            if constexpr (WA) {
                racc[NA - 1] += fabs(a[jj]);
                if (strict)
                    cacc[jj][NA - 1] += fabs(a[jj]);
            }
        }
        // row partial of tile (I, J): sum over the 4 waves in order
#pragma unroll
        for (int c = 0; c < NA; ++c) red[w][c][lane] = racc[c];
        __syncthreads();
        for (int idx = threadIdx.x; idx < NA * 64; idx += 256) {
            const int c = idx / 64, i = idx % 64;
            RP[(((int64_t)I * nrb + J) * NC + c) * 64 + i] = ((red[0][c][i] + red[1][c][i]) + red[2][c][i]) + red[3][c][i];
        }
        __syncthreads();
    }
    // column partials: reduce each column's 64 lanes (fixed butterfly order)
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
#pragma unroll
        for (int c = 0; c < NA; ++c) {
            double v = cacc[jj][c];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0)
                CP[(((int64_t)J * Q + q) * NC + c) * 64 + 16 * w + jj] = v;
        }
}

SPD_DEV double nanmax2(double a, double b) { return (a > b || a != a) ? a : b; }
SPD_DEV double wave_max2(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v = nanmax2(v, __shfl_xor(v, off));
    return v;
}

__global__ __launch_bounds__(256) void k_resid_reduce(const double *__restrict__ B, int64_t ldb,
                                                      const double *__restrict__ X, int64_t ldx, int64_t n, int m,
                                                      int S, const double *__restrict__ P,
                                                      const double *__restrict__ Pabs, int want_abs,
                                                      const double *__restrict__ d, double *__restrict__ R,
                                                      int64_t ldr, double *norms)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    double vr = 0.0, vx = 0.0, vb = 0.0, vd = 0.0, va = 0.0;
    if (i < n) {
        double sum = 0.0;
        for (int s = 0; s < S; ++s)
            sum += P[((int64_t)s * m + c) * n + i];
        const double b = B[i + c * ldb];
        const double r = b - sum;
        R[i + c * ldr] = r;
        vr = fabs(r);
        vx = fabs(X[i + c * ldx]);
        vb = fabs(b);
        vd = d ? fabs(d[i] * r) : vr;
        if (want_abs && c == 0) {
            double a = 0.0;
            for (int s = 0; s < S; ++s)
                a += Pabs[(int64_t)s * n + i];
            va = a;
        }
    }
    vr = wave_max2(vr);
    vx = wave_max2(vx);
    vb = wave_max2(vb);
    vd = wave_max2(vd);
    if (want_abs && c == 0)
        va = wave_max2(va);
    if ((threadIdx.x & 63) == 0) {
        atomic_max_nonneg(norms + 1 + c, vr);
        atomic_max_nonneg(norms + 1 + m + c, vx);
        atomic_max_nonneg(norms + 1 + 2 * m + c, vb);
        atomic_max_nonneg(norms + 1 + 3 * m + c, vd);
        if (want_abs && c == 0)
            atomic_max_nonneg(norms, va);
    }
}

// R = B - (sum_J RP[I][J] + sum_q CP[I][q]) and the norms (as k_resid_reduce).
// Workgroup (I, c): 64 rows of block I, four waves; wave p sums the partials
// J = p, p + 4, ... (loads issued four at a time), and the four sums are
// added in the fixed order (s0 + s1) + (s2 + s3), then the column partials.
template <int MC>
__global__ __launch_bounds__(256) void k_resid_sym_reduce(const double *__restrict__ B, int64_t ldb,
                                                          const double *__restrict__ X, int64_t ldx, int64_t n, int m,
                                                          int Q, const double *__restrict__ RP,
                                                          const double *__restrict__ CP, int want_abs,
                                                          const double *__restrict__ d, double *__restrict__ R,
                                                          int64_t ldr, double *norms)
{
    constexpr int NC = MC + 1;
    __shared__ double part[2][4][64];
    const int il = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int I = blockIdx.x, c = blockIdx.y;
    const int nrb = (int)((n + 63) / 64);
    const bool wa = want_abs && c == 0;
    {
        const double *rp = RP + ((int64_t)I * nrb * NC + c) * 64 + il;
        const double *ra = RP + ((int64_t)I * nrb * NC + MC) * 64 + il;
        const int64_t st = (int64_t)NC * 64;  // stride between consecutive J
        double y = 0.0, ya = 0.0;
        int J = p;
        for (; J + 12 <= I; J += 16) {
            const double v0 = rp[J * st], v1 = rp[(J + 4) * st], v2 = rp[(J + 8) * st], v3 = rp[(J + 12) * st];
            if (wa) {
                const double a0 = ra[J * st], a1 = ra[(J + 4) * st], a2 = ra[(J + 8) * st], a3 = ra[(J + 12) * st];
                ya = (((ya + a0) + a1) + a2) + a3;
            }
            y = (((y + v0) + v1) + v2) + v3;
        }
        for (; J <= I; J += 4) {
            y += rp[J * st];
            if (wa)
                ya += ra[J * st];
        }
        part[0][p][il] = y;
        part[1][p][il] = ya;
    }
    __syncthreads();
    if (p != 0)
        return;
    const int64_t i = (int64_t)I * 64 + il;
    double vr = 0.0, vx = 0.0, vb = 0.0, vd = 0.0, va = 0.0;
    if (i < n) {
        double y = (part[0][0][il] + part[0][1][il]) + (part[0][2][il] + part[0][3][il]);
        double ya = (part[1][0][il] + part[1][1][il]) + (part[1][2][il] + part[1][3][il]);
        for (int q = 0; q < Q; ++q) {
            if (I + q * RSYM_CH >= nrb)
                break;
            y += CP[(((int64_t)I * Q + q) * NC + c) * 64 + il];
            if (wa)
                ya += CP[(((int64_t)I * Q + q) * NC + MC) * 64 + il];
        }
        const double b = B[i + c * ldb];
        const double r = b - y;
        R[i + c * ldr] = r;
        vr = fabs(r);
        vx = fabs(X[i + c * ldx]);
        vb = fabs(b);
        vd = d ? fabs(d[i] * r) : vr;
        va = ya;
    }
    vr = wave_max2(vr);
    vx = wave_max2(vx);
    vb = wave_max2(vb);
    vd = wave_max2(vd);
    if (wa)
        va = wave_max2(va);
    if (il == 0) {
        atomic_max_nonneg(norms + 1 + c, vr);
        atomic_max_nonneg(norms + 1 + m + c, vx);
        atomic_max_nonneg(norms + 1 + 2 * m + c, vb);
        atomic_max_nonneg(norms + 1 + 3 * m + c, vd);
        if (wa)
            atomic_max_nonneg(norms, va);
    }
}

namespace spd {

static int resid_splits(int64_t n)
{
    const int64_t nrb = (n + 63) / 64;
    int64_t S = 2048 / (nrb > 0 ? nrb : 1);
    if (S < 1) S = 1;
    if (S > nrb) S = nrb;
    if (S > 64) S = 64;
    return (int)(S < 1 ? 1 : S);
}

#define RSYM_MAX_M 2
static int rsym_mc(int m) { return m <= 1 ? 1 : 2; }

int64_t resid_scratch(int64_t n, int m)
{
    const int S = resid_splits(n);
    int64_t need = (int64_t)S * n * (m + 1);
    if (m <= RSYM_MAX_M) {
        const int64_t nrb = (n + 63) / 64, Q = (nrb + RSYM_CH - 1) / RSYM_CH, nc = rsym_mc(m) + 1;
        need = std::max<int64_t>(need, (nrb * nrb + nrb * Q) * nc * 64);
    }
    return need;
}

// eta[c] = ||r_c|| / (||A|| ||x_c|| + ||b_c||) from the residual's norms
// (norms[0] = ||A||, then max|r|, max|x|, max|b| per column), rounded as the
// host formula rounds it (no fused multiply-add)
__global__ void k_eta_from_norms(const double *__restrict__ norms, int m, double *__restrict__ eta)
{
#pragma clang fp contract(off)
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (c >= m)
        return;
    const double an = norms[0], rn = norms[1 + c], xn = norms[1 + m + c], bn = norms[1 + 2 * m + c];
    const double den = an * xn + bn;
    double v = (den > 0.0) ? rn / den : (rn > 0.0 ? __builtin_inf() : 0.0);
    if (!(rn == rn) || !(xn == xn) || !(an == an))
        v = __builtin_nan("");
    eta[c] = v;
}

template <int MC, int RB, int CB, int JS>
static void launch_partial(const double *A, int64_t lda, int64_t n, const double *X, int64_t ldx, int m, int c0,
                           int S, double *P, double *Pabs, int want_abs, hipStream_t st)
{
    const unsigned nrb = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL((k_resid_partial<MC, RB, CB, JS>), dim3(nrb, (unsigned)S), dim3(256), 0, st, A, lda, n, X,
                       ldx, m, c0, S, P, Pabs, want_abs);
}

void launch_eta_from_norms(const double *norms, int m, double *eta, hipStream_t st)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_eta_from_norms, dim3((unsigned)((m + 63) / 64)), dim3(64), 0, st, norms, m, eta);
}

void launch_residual(const double *A, int64_t lda, int64_t n, const double *X, int64_t ldx, const double *B,
                     int64_t ldb, int m, double *R, int64_t ldr, const double *d, double *norms, int want_anorm,
                     double *P, hipStream_t st)
{
    if (n <= 0 || m <= 0) return;
    if (m <= RSYM_MAX_M) {
        const int nrb = (int)((n + 63) / 64), Q = (nrb + RSYM_CH - 1) / RSYM_CH, mc = rsym_mc(m);
        double *RP = P, *CP = P + (int64_t)nrb * nrb * (mc + 1) * 64;
        const dim3 g((unsigned)nrb, (unsigned)Q), gr((unsigned)nrb, (unsigned)m);
        if (mc == 1) {
            if (want_anorm)
                hipLaunchKernelGGL((k_resid_sym<1, true>), g, dim3(256), 0, st, A, lda, n, X, ldx, m, Q, RP, CP);
            else
                hipLaunchKernelGGL((k_resid_sym<1, false>), g, dim3(256), 0, st, A, lda, n, X, ldx, m, Q, RP, CP);
            hipLaunchKernelGGL(k_resid_sym_reduce<1>, gr, dim3(256), 0, st, B, ldb, X, ldx, n, m, Q, RP, CP,
                               want_anorm, d, R, ldr, norms);
        } else {
            if (want_anorm)
                hipLaunchKernelGGL((k_resid_sym<2, true>), g, dim3(256), 0, st, A, lda, n, X, ldx, m, Q, RP, CP);
            else
                hipLaunchKernelGGL((k_resid_sym<2, false>), g, dim3(256), 0, st, A, lda, n, X, ldx, m, Q, RP, CP);
            hipLaunchKernelGGL(k_resid_sym_reduce<2>, gr, dim3(256), 0, st, B, ldb, X, ldx, n, m, Q, RP, CP,
                               want_anorm, d, R, ldr, norms);
        }
        return;
    }
    const int S = resid_splits(n);
    double *Pabs = P + (int64_t)S * n * m;
    const unsigned nrb = (unsigned)((n + 63) / 64);
    const int step = (m > 8) ? 32 : 64;  // MFMA chunks of up to 32 columns
    for (int c0 = 0; c0 < m; c0 += step) {
        const int mc = (m - c0 < step) ? (m - c0) : step;
        const int wa = (want_anorm && c0 == 0) ? 1 : 0;
        if (mc > 8) {
            if (mc <= 16)
                hipLaunchKernelGGL(k_resid_mfma<1>, dim3(nrb, (unsigned)S), dim3(256), 0, st, A, lda, n, X, ldx, m, c0,
                                   S, P, Pabs, wa);
            else
                hipLaunchKernelGGL(k_resid_mfma<2>, dim3(nrb, (unsigned)S), dim3(256), 0, st, A, lda, n, X, ldx, m, c0,
                                   S, P, Pabs, wa);
        } else if (mc <= 1)
            launch_partial<1, 1, 1, 4>(A, lda, n, X, ldx, m, c0, S, P, Pabs, wa, st);
        else if (mc <= 2)
            launch_partial<2, 1, 1, 2>(A, lda, n, X, ldx, m, c0, S, P, Pabs, wa, st);
        else if (mc <= 4)
            launch_partial<4, 1, 1, 1>(A, lda, n, X, ldx, m, c0, S, P, Pabs, wa, st);
        else
            launch_partial<8, 1, 2, 1>(A, lda, n, X, ldx, m, c0, S, P, Pabs, wa, st);
    }
    hipLaunchKernelGGL(k_resid_reduce, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, st, B, ldb, X,
                       ldx, n, m, S, P, Pabs, want_anorm, d, R, ldr, norms);
}

}  // namespace spd
