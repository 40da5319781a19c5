// Trailing update of the blocked factorisation in Algorithm 1's low-precision
// Cholesky (the Schur complement update of the low-precision factor),
//   H_ij -= L_ik L_jk^T   for the lower tiles of the trailing region,
// on MFMA: binary32 (k_syrk_update_f32), binary64 (k_syrk_update<double>),
// and binary16 / bfloat16 operands with binary32 accumulation
// (k_syrk_update_h).  Launched by the factorisation driver per group of
// panels (K = G NB) and within a group for its remaining panels.
#include "common.h"
#include "internal.h"
#include "half_ops.h"
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <type_traits>

// ---------------------------------------------------------------------------
// K4: trailing update H_ij -= L_ik L_jk^T on 128 x 128 lower tiles (MFMA).
// Tiles are numbered over the lower triangle of the trailing region (t tiles
// per side) restricted to tile columns [tj_lo, tj_hi): a range that stops
// short of the last tile column (or spans at most four) is walked column by
// column, a range reaching it as the lower triangle from (tj_lo, tj_lo) row
// by row.  Block indices are remapped so that consecutive tiles land on the
// same XCD (blocks are dispatched round-robin over the 8 XCDs).
SPD_DEV void decode_tile(int b, int t, int tj_lo, int tj_hi, int &ti, int &tj)
{
    if (tj_hi < t || tj_hi - tj_lo <= 4) {
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

// binary64 (binary32 has its own kernel below)
template <typename T> struct SyrkCfg;
template <> struct SyrkCfg<double> {
    static constexpr int KC = 16;
    using Acc = Acc32<double>;
    using Fr = Frag<double>;
};

template <typename T>
__global__ __launch_bounds__(256) void k_syrk_update(T *__restrict__ H, int64_t ld, int64_t k0, int nbk, int64_t r0,
                                                     int t, int tj_lo, int tj_hi, int ntiles,
                                                     const unsigned long long *info, int prio)
{
    constexpr int KC = SyrkCfg<T>::KC;
    using AccT = typename SyrkCfg<T>::Acc;
    using FragT = typename SyrkCfg<T>::Fr;
    constexpr int LDT = SPD_TILE + 4;  // LDS column stride
    __shared__ T As[2][KC * LDT];
    __shared__ T Bs[2][KC * LDT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    if (prio)
        __builtin_amdgcn_s_setprio(2);  // the lookahead part of the update
    // tiles of XCD x (blocks are dispatched round-robin over the 8 XCDs) are
    // the contiguous range [x chunk, (x + 1) chunk); a grid smaller than the
    // tile count loops (persistent), leaving compute-unit slots free
    const int per = gridDim.x / 8, chunk = (ntiles + 7) / 8;
    for (int it = blockIdx.x / 8; it < chunk; it += per) {
    const int logical = (blockIdx.x % 8) * chunk + it;
    if (logical >= ntiles)
        break;
    int ti, tj;
    decode_tile(logical, t, tj_lo, tj_hi, ti, tj);
    if (ti < 0)
        break;
    const int64_t crow = r0 + (int64_t)ti * SPD_TILE, ccol = r0 + (int64_t)tj * SPD_TILE;
    const T *pa = H + ccol + k0 * ld;  // rows of tile tj (D rows = C columns)
    const T *pb = H + crow + k0 * ld;  // rows of tile ti (D columns = C rows)
    const int wm = wave >> 1, wn = wave & 1;

    // The C tile is read once, up front, straight into the accumulators (so
    // its latency overlaps the K loop); the MFMA operands are negated.
    // Register j of tile (mi, ni) holds C[crow + 64 wn + 32 ni + col(j)][ccol + 64 wm + 32 mi + row(j)].
    AccT acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = AccT::row(j, lane), nn = AccT::col(j, lane);
                acc[mi][ni].set(j, H[(crow + 64 * wn + 32 * ni + nn) + (ccol + 64 * wm + 32 * mi + m) * ld]);
            }

    // 128 rows x KC columns of each operand per chunk, 16-byte vector loads,
    // staged through registers so the next chunk's loads overlap the MFMAs.
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int PER_COL = SPD_TILE / VEC;
    constexpr int NV = PER_COL * KC / 256;  // vectors per thread per operand
    static_assert(NV == 4, "staging layout");
    // per-thread staging slots: vector v covers column col_v, rows r_v..r_v+VEC-1
    int soff[NV];
    size_t goff[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int idx = tid + 256 * v;
        const int col = idx / PER_COL, r = (idx % PER_COL) * VEC;
        soff[v] = col * LDT + r;
        goff[v] = (size_t)col * ld + r;
    }
    V ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define SPD_GLOAD(kb)                                                       \
    do {                                                                    \
        const size_t o_ = (size_t)(kb) * ld;                                \
        ra0 = *(const V *)&pa[o_ + goff[0]]; rb0 = *(const V *)&pb[o_ + goff[0]]; \
        ra1 = *(const V *)&pa[o_ + goff[1]]; rb1 = *(const V *)&pb[o_ + goff[1]]; \
        ra2 = *(const V *)&pa[o_ + goff[2]]; rb2 = *(const V *)&pb[o_ + goff[2]]; \
        ra3 = *(const V *)&pa[o_ + goff[3]]; rb3 = *(const V *)&pb[o_ + goff[3]]; \
    } while (0)
#define SPD_SSTORE(buf)                                                     \
    do {                                                                    \
        *(V *)&As[buf][soff[0]] = ra0; *(V *)&Bs[buf][soff[0]] = rb0;       \
        *(V *)&As[buf][soff[1]] = ra1; *(V *)&Bs[buf][soff[1]] = rb1;       \
        *(V *)&As[buf][soff[2]] = ra2; *(V *)&Bs[buf][soff[2]] = rb2;       \
        *(V *)&As[buf][soff[3]] = ra3; *(V *)&Bs[buf][soff[3]] = rb3;       \
    } while (0)

    SPD_GLOAD(0);
    SPD_SSTORE(0);
    __syncthreads();
    int buf = 0;
    for (int kb = 0; kb < nbk; kb += KC) {
        // prefetch the next chunk (the last iteration re-reads its own chunk)
        const int kn = (kb + KC < nbk) ? kb + KC : kb;
        SPD_GLOAD(kn);
        // keep the next chunk's loads here, ahead of the MFMAs (the scheduler
        // would otherwise sink them to their LDS stores and expose their latency)
        __builtin_amdgcn_sched_barrier(0);
        const T *a0 = &As[buf][64 * wm];
        const T *b0 = &Bs[buf][64 * wn];
#pragma unroll
        for (int k = 0; k < KC; k += FragT::K) {
            FragT fa[2], fb[2];
            fa[0].load(a0 + k * LDT, LDT, lane);
            fa[1].load(a0 + 32 + k * LDT, LDT, lane);
            fb[0].load(b0 + k * LDT, LDT, lane);
            fb[1].load(b0 + 32 + k * LDT, LDT, lane);
            fa[0].negate();
            fa[1].negate();
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    mma(acc[mi][ni], fa[mi], fb[ni]);
        }
        __builtin_amdgcn_sched_barrier(0);
        SPD_SSTORE(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#undef SPD_GLOAD
#undef SPD_SSTORE
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = AccT::row(j, lane), nn = AccT::col(j, lane);
                H[(crow + 64 * wn + 32 * ni + nn) + (ccol + 64 * wm + 32 * mi + m) * ld] = acc[mi][ni].get(j);
            }
    __syncthreads();  // shared memory is reused by the next tile
    }
}

// ---------------------------------------------------------------------------
// K4, binary32: the same update written for v_mfma_f32_16x16x4f32.  One
// TS x TS tile (TS = 128 or 64): each wave owns a TS/2 x TS/2 block of
// D = C^T as NB x NB 16 x 16 accumulators holding -C (the sign is applied
// once on load and once on store, so the K loop only multiplies and adds).
// Shared memory holds KC columns of each operand as [k][row] with TS floats
// per k and the row index XOR-ed with 16 (k % 4): a fragment read (lane l:
// row 16 b + l%16, k = 4 s + l/16) then touches 64 distinct banks, and the
// 16-byte staging stores stay contiguous.  As and Bs are two staging
// buffers of KC x TS floats each; every wave has passed the final barrier
// when the function returns, so the next tile may restage at once.
template <int TS, int KC>
SPD_DEV void f32_update_tile(float *__restrict__ H, int64_t ld, int64_t k0, int nbk, int64_t crow, int64_t ccol,
                             float *__restrict__ As, float *__restrict__ Bs, int tid)
{
    constexpr int NB = TS / 32, NV = KC * TS / 1024;  // 16-blocks per wave side; staged float4 per thread
    constexpr int BUF = KC * TS;
    static_assert(NV == 2 || NV == 4, "staging layout");
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1, r = lane & 15, u = lane >> 4;
    const int ldi = (int)ld;  // offsets within a tile row block of <= 1024 columns fit in 32 bits
    // staging: thread covers rows 4 (tid % (TS/4)) .. +3 of columns tid / (TS/4) + (1024/TS) v
    constexpr int TPC = TS / 4, CSTEP = 256 / TPC;
    const int scol = tid / TPC, srow = (tid % TPC) * 4;
    const int goff = scol * ldi + srow;
    const int soff = scol * TS + (srow ^ (16 * (scol & 3)));  // CSTEP is a multiple of 4: col % 4 fixed
    // fragment offsets: row 16 b + r of the wave's TS/2 rows, k-slot u (+ 4 s TS for k-step s)
    int fa[NB], fb[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        fa[b] = u * TS + (((TS / 2) * wm + 16 * b) ^ (16 * u)) + r;
        fb[b] = u * TS + (((TS / 2) * wn + 16 * b) ^ (16 * u)) + r;
    }
    const int coff = r + 4 * u * ldi;
    const float *pa = H + ccol + k0 * ld;  // rows of tile tj (D rows = C columns)
    const float *pb = H + crow + k0 * ld;  // rows of tile ti (D columns = C rows)
    // register q of block (mi, ni): -C[crow + TS/2 wn + 16 ni + r][ccol + TS/2 wm + 16 mi + 4 u + q]
    float *cu = H + (crow + (TS / 2) * wn) + (ccol + (TS / 2) * wm) * ld;
    floatx4 c[NB][NB];
#pragma unroll
    for (int mi = 0; mi < NB; ++mi)
#pragma unroll
        for (int ni = 0; ni < NB; ++ni)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                c[mi][ni][q] = -cu[coff + 16 * ni + (16 * mi + q) * ldi];
    // staging registers (named, not an array, so that they stay registers)
    float4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define SPD_GL(o)                                                                         \
    do {                                                                                  \
        ra0 = *(const float4 *)&pa[(o) + goff];                                           \
        rb0 = *(const float4 *)&pb[(o) + goff];                                           \
        ra1 = *(const float4 *)&pa[(o) + goff + CSTEP * ldi];                             \
        rb1 = *(const float4 *)&pb[(o) + goff + CSTEP * ldi];                             \
        if constexpr (NV > 2) {                                                           \
            ra2 = *(const float4 *)&pa[(o) + goff + 2 * CSTEP * ldi];                     \
            rb2 = *(const float4 *)&pb[(o) + goff + 2 * CSTEP * ldi];                     \
            ra3 = *(const float4 *)&pa[(o) + goff + 3 * CSTEP * ldi];                     \
            rb3 = *(const float4 *)&pb[(o) + goff + 3 * CSTEP * ldi];                     \
        }                                                                                 \
    } while (0)
#define SPD_SS(bf)                                                                        \
    do {                                                                                  \
        float *as_ = As + (bf) * BUF, *bs_ = Bs + (bf) * BUF;                             \
        *(float4 *)&as_[soff] = ra0;                                                      \
        *(float4 *)&bs_[soff] = rb0;                                                      \
        *(float4 *)&as_[soff + CSTEP * TS] = ra1;                                         \
        *(float4 *)&bs_[soff + CSTEP * TS] = rb1;                                         \
        if constexpr (NV > 2) {                                                           \
            *(float4 *)&as_[soff + 2 * CSTEP * TS] = ra2;                                 \
            *(float4 *)&bs_[soff + 2 * CSTEP * TS] = rb2;                                 \
            *(float4 *)&as_[soff + 3 * CSTEP * TS] = ra3;                                 \
            *(float4 *)&bs_[soff + 3 * CSTEP * TS] = rb3;                                 \
        }                                                                                 \
    } while (0)
    SPD_GL(0);
    SPD_SS(0);
    lds_barrier();
    int buf = 0;
    for (int kb = 0; kb < nbk; kb += KC) {
        // prefetch the next chunk (the last iteration re-reads its own chunk)
        const int o = ((kb + KC < nbk) ? kb + KC : kb) * ldi;
        SPD_GL(o);
        __builtin_amdgcn_sched_barrier(0);
        const float *A0 = As + buf * BUF, *B0 = Bs + buf * BUF;
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            float a[NB], b[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                a[i] = A0[4 * ks * TS + fa[i]];
                b[i] = B0[4 * ks * TS + fb[i]];
            }
#pragma unroll
            for (int mi = 0; mi < NB; ++mi)
#pragma unroll
                for (int ni = 0; ni < NB; ++ni)
                    c[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mi], b[ni], c[mi][ni], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        SPD_SS(buf ^ 1);
        lds_barrier();
        buf ^= 1;
    }
#undef SPD_GL
#undef SPD_SS
#pragma unroll
    for (int mi = 0; mi < NB; ++mi)
#pragma unroll
        for (int ni = 0; ni < NB; ++ni)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                cu[coff + 16 * ni + (16 * mi + q) * ldi] = -c[mi][ni][q];
}

// A last round's 64-tile (chunks of 64 columns) in a function of its own, so
// that the 128-tile loop of the kernel keeps the register allocation and
// schedule it has without it.  The pointers are re-derived in their address
// spaces (global, shared), so the accesses stay GLOBAL and DS instructions.
__device__ __attribute__((noinline)) void f32_update_tail_tile(float *H, int64_t ld, int64_t k0, int nbk,
                                                               int64_t crow, int64_t ccol, float *As, float *Bs,
                                                               int tid)
{
    H = (float *)gmem(H);
    As = (float *)(__attribute__((address_space(3))) float *)As;
    Bs = (float *)(__attribute__((address_space(3))) float *)Bs;
    f32_update_tile<64, 64>(H, ld, k0, nbk, crow, ccol, As, Bs, tid);
}

// The binary32 update on TS x TS tiles (128, or 64 for the panel chain's
// single tile columns and for launches with too few 128-tiles to fill the
// chip).  Tiles are counted in TS units over the lower triangle of the
// trailing region (t tiles per side), tile columns [tj_lo, tj_hi).  Tiles
// [0, nfull) run whole, the same number per workgroup; with TS = 128 the
// remaining tiles [nfull, ntiles) -- a last round too small to fill the
// workgroups -- run as four 64-tiles each (the quarter above the diagonal
// of a diagonal tile skipped), with chunks of 64 columns, so that a last
// round costs about a quarter of a whole one.
template <int TS>
__global__ __launch_bounds__(256, 2) void k_syrk_update_f32(float *__restrict__ H, int64_t ld, int64_t k0, int nbk,
                                                           int64_t r0, int t, int tj_lo, int tj_hi, int ntiles,
                                                           int nfull, const unsigned long long *info, int prio)
{
    constexpr int KC = 32;
    __shared__ __align__(16) float As[2 * KC * TS];
    __shared__ __align__(16) float Bs[2 * KC * TS];
    const int tid = threadIdx.x;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    if (prio)
        __builtin_amdgcn_s_setprio(2);  // the lookahead part of the update
    const int per = gridDim.x / 8, chunk = (nfull + 7) / 8;
    for (int it = blockIdx.x / 8; it < chunk; it += per) {
        const int logical = (blockIdx.x % 8) * chunk + it;
        if (logical >= nfull)
            break;
        int ti, tj;
        decode_tile(logical, t, tj_lo, tj_hi, ti, tj);
        if (ti < 0)
            break;
        f32_update_tile<TS, KC>(H, ld, k0, nbk, r0 + (int64_t)ti * TS, r0 + (int64_t)tj * TS, As, Bs, tid);
    }
    if constexpr (TS == 128) {
        const int nsub = 4 * (ntiles - nfull), chunk2 = (nsub + 7) / 8;
        for (int it = blockIdx.x / 8; it < chunk2; it += per) {
            const int s = (blockIdx.x % 8) * chunk2 + it;
            if (s >= nsub)
                break;
            int ti, tj;
            decode_tile(nfull + (s >> 2), t, tj_lo, tj_hi, ti, tj);
            if (ti < 0)
                break;
            const int qi = (s >> 1) & 1, qj = s & 1;
            if (ti == tj && qi < qj)
                continue;  // above the diagonal
            f32_update_tail_tile(H, ld, k0, nbk, r0 + (int64_t)ti * 128 + 64 * qi, r0 + (int64_t)tj * 128 + 64 * qj, As,
                                 Bs, tid);
        }
    }
}

// ---------------------------------------------------------------------------
// K4, half-precision operands: H_ij -= round(L_ik) round(L_jk)^T with
// binary16 or bfloat16 operands and binary32 accumulation
// (v_mfma_f32_32x32x16_{f16,bf16}) on 128 x 128 tiles, np panels of K = 128
// each.  The operand panels are the fragment-layout copies written by the
// panel solve: row r (relative to the first row of the copy), column k at
//   ((r/32) (NB/16) + k/16) * 512 + (32 ((k%16)/8) + r%32) * 8 + k%8,
// so every fragment load is one contiguous 1 KiB per wave.  Panel p of the
// launch is the copy in ring slot (slot0 + p) % 16 (stride `sstride`
// fragments), with skip0 - 4 p 32-row blocks before row r0.
template <int HK>
__global__ __launch_bounds__(256) void k_syrk_update_h(float *__restrict__ H, int64_t ld, const void *__restrict__ Lh,
                                                       int slot0, int64_t sstride, int skip0, int np, int64_t r0,
                                                       int t, int tj_lo, int tj_hi, int ntiles,
                                                       const unsigned long long *info, int prio)
{
    using V8 = typename HalfT<HK>::V8;
    constexpr int KS = 128 / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    if (prio)
        __builtin_amdgcn_s_setprio(2);
    // tiles of XCD x (blocks are dispatched round-robin over the 8 XCDs) are
    // the contiguous range [x chunk, (x + 1) chunk); a grid smaller than the
    // tile count loops (persistent), leaving compute-unit slots free
    const V8 *base = (const V8 *)Lh;
    const int per = gridDim.x / 8, chunk = (ntiles + 7) / 8;
    for (int it = blockIdx.x / 8; it < chunk; it += per) {
    const int logical = (blockIdx.x % 8) * chunk + it;
    if (logical >= ntiles)
        break;
    int ti, tj;
    decode_tile(logical, t, tj_lo, tj_hi, ti, tj);
    if (ti < 0)
        break;
    const int64_t crow = r0 + (int64_t)ti * SPD_TILE, ccol = r0 + (int64_t)tj * SPD_TILE;
    const int wm = wave >> 1, wn = wave & 1;
    floatx16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = Acc32<float>::row(j, lane), nn = Acc32<float>::col(j, lane);
                acc[mi][ni][j] = H[(crow + 64 * wn + 32 * ni + nn) + (ccol + 64 * wm + 32 * mi + m) * ld];
            }
    for (int pnl = 0; pnl < np; ++pnl) {
        const V8 *lh = base + (int64_t)((slot0 + pnl) & 15) * sstride;
        const int skip = skip0 - 4 * pnl;
        // A operand: rows of tile tj (C columns); B operand: rows of tile ti (C rows)
        const V8 *pa0 = lh + (size_t)(skip + 4 * tj + 2 * wm) * KS * 64 + lane;
        const V8 *pb0 = lh + (size_t)(skip + 4 * ti + 2 * wn) * KS * 64 + lane;
        V8 fa[KS][2], fb[KS][2];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                fa[ks][q] = pa0[(q * KS + ks) * 64];
                fb[ks][q] = pb0[(q * KS + ks) * 64];
            }
        // all operand loads in flight before the first MFMA
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) {
                const V8 na = HalfT<HK>::neg(fa[ks][mi]);
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = HalfT<HK>::mma(na, fb[ks][ni], acc[mi][ni]);
            }
        }
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int m = Acc32<float>::row(j, lane), nn = Acc32<float>::col(j, lane);
                H[(crow + 64 * wn + 32 * ni + nn) + (ccol + 64 * wm + 32 * mi + m) * ld] = acc[mi][ni][j];
            }
    }
}

// ---------------------------------------------------------------------------
// K4, half-precision operands, 256 x 256 tiles: a whole group of np panels
// (K = 128 np, np <= 16) in one pass over each C tile, so the binary32 C tile
// crosses HBM once per group instead of once per one or two panels.  Each
// wave owns a 128 x 128 block of the tile as 4 x 4 accumulators of
// v_mfma_f32_32x32x16_{f16,bf16} (256 registers: one wave per SIMD), and
// streams its operand fragments straight from the panel copies -- one
// contiguous 1 KiB per fragment per wave -- with the next k-step's eight
// fragments in flight while the current step's sixteen MFMAs run.
// Panel p of the group is the copy in ring slot (slot0 + p) % 16 (slot
// stride `sstride` fragments); the copy of panel p starts 4 32-row blocks
// later than that of panel p - 1, so skip_p = skip0 - 4 p.
template <int HK>
__global__ __launch_bounds__(256, 1) void k_syrk_update_h256(float *__restrict__ H, int64_t ld,
                                                             const void *__restrict__ Lh, int slot0, int64_t sstride,
                                                             int skip0, int np, int64_t r0, int t, int tj_lo,
                                                             int tj_hi, int ntiles, const unsigned long long *info,
                                                             int prio)
{
    using V8 = typename HalfT<HK>::V8;
    constexpr int KS = 128 / 16;  // k-steps per panel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (*(volatile const unsigned long long *)info != (unsigned long long)SPD_INFO_NONE)
        return;
    if (prio)
        __builtin_amdgcn_s_setprio(2);
    const int wm = wave >> 1, wn = wave & 1;
    const V8 *base = (const V8 *)Lh;
    const int per = gridDim.x / 8, chunk = (ntiles + 7) / 8;
    for (int it = blockIdx.x / 8; it < chunk; it += per) {
        const int logical = (blockIdx.x % 8) * chunk + it;
        if (logical >= ntiles)
            break;
        int ti, tj;
        decode_tile(logical, t, tj_lo, tj_hi, ti, tj);
        if (ti < 0)
            break;
        const int64_t crow = r0 + (int64_t)ti * 256, ccol = r0 + (int64_t)tj * 256;
        // register j of acc[a][b] accumulates -sum L L^T for
        // C[crow + 128 wn + 32 b + col(j)][ccol + 128 wm + 32 a + row(j)];
        // C itself is added at the end (holding it through the K loop would
        // need a second register file)
        float *cb = H + (crow + 128 * wn) + (ccol + 128 * wm) * ld;
        const int ldi = (int)ld;  // byte offsets inside the wave's 128 x 128 block fit in 31 bits (ld < 2^22)
        floatx16 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    acc[a][b][j] = 0.0f;
        // operand 32-row blocks: A (C columns) 8 tj + 4 wm + a, B (C rows) 8 ti + 4 wn + b
        const int ba = 8 * tj + 4 * wm, bb = 8 * ti + 4 * wn;
        const int S = np * KS;
        V8 fa0[4], fb0[4], fa1[4], fb1[4];
        auto load = [&](int s, V8 *fa, V8 *fb) {
            const int p = s / KS, ks = s % KS;
            const V8 *lh = base + (int64_t)((slot0 + p) & 15) * sstride + lane;
            const int sk = skip0 - 4 * p;
#pragma unroll
            for (int a = 0; a < 4; ++a)
                fa[a] = lh[((int64_t)(sk + ba + a) * KS + ks) * 64];
#pragma unroll
            for (int b = 0; b < 4; ++b)
                fb[b] = lh[((int64_t)(sk + bb + b) * KS + ks) * 64];
        };
        auto step = [&](const V8 *fa, const V8 *fb) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const V8 na = HalfT<HK>::neg(fa[a]);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = HalfT<HK>::mma(na, fb[b], acc[a][b]);
            }
        };
        load(0, fa0, fb0);
        for (int s = 0; s < S; s += 2) {
            // S is even (KS = 8): steps s and s + 1 both exist
            load(s + 1, fa1, fb1);
            __builtin_amdgcn_sched_barrier(0);
            step(fa0, fb0);
            __builtin_amdgcn_sched_barrier(0);
            if (s + 2 < S)
                load(s + 2, fa0, fb0);
            __builtin_amdgcn_sched_barrier(0);
            step(fa1, fb1);
            __builtin_amdgcn_sched_barrier(0);
        }
        // C += acc, one 32 x 32 block at a time, the next block's C values
        // in flight while the current one is added and stored.  Buffer
        // loads/stores: the lane's part of the offset is one register, the
        // block's part a scalar (global addressing would keep a 64-bit
        // address per element alive through the K loop).
        // Offsets: register j of block (a, b) is at lane part + row part
        // (8 (j/4) + j%4) ldi (one register per j) + block part 32 a ldi
        // (scalar) + 32 b (immediate).  The asm statement keeps the compiler
        // from computing them before the K loop, where they would stay live.
        int rowb = ldi * 4;
        asm volatile("" : "+s"(rowb));
        const __amdgpu_buffer_rsrc_t rc =
            __builtin_amdgcn_make_buffer_rsrc(cb, (short)0, 0x7fffffff, SPD_BUFFER_RSRC_WORD3);
        const int voff = Acc32<float>::col(0, lane) * 4 + 4 * (lane >> 5) * rowb;
        int vj[16];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            vj[j] = voff + (8 * (j / 4) + j % 4) * rowb;
        float cv[2][16];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            cv[0][j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, vj[j], 0, 0));
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int a = q / 4, b = q % 4;
            if (q + 1 < 16) {
                const int a1 = (q + 1) / 4, b1 = (q + 1) % 4;
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    cv[(q + 1) & 1][j] = __builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(rc, vj[j] + 128 * b1, 32 * a1 * rowb, 0));
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, cv[q & 1][j] + acc[a][b][j]), rc,
                                                      vj[j] + 128 * b, 32 * a * rowb, 0);
        }
    }
}

namespace spd {

void launch_syrk_update_h256(float *H, int64_t ld, const void *Lh, int slot0, int64_t sstride, int skip0, int np,
                             int half, int64_t r0, int t, int tj_lo, int tj_hi, const unsigned long long *info,
                             hipStream_t st, int prio, int max_grid)
{
    if (t <= 0 || tj_lo >= tj_hi || np <= 0) return;
    int64_t ntiles = 0;
    for (int c = tj_lo; c < tj_hi; ++c) ntiles += t - c;
    int64_t grid = ((ntiles + 7) / 8) * 8;
    if (max_grid > 0 && grid > max_grid) grid = (max_grid / 8) * 8;
    if (half == HALF_F16)
        hipLaunchKernelGGL(k_syrk_update_h256<HALF_F16>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, Lh, slot0,
                           sstride, skip0, np, r0, t, tj_lo, tj_hi, (int)ntiles, info, prio);
    else
        hipLaunchKernelGGL(k_syrk_update_h256<HALF_BF16>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, Lh, slot0,
                           sstride, skip0, np, r0, t, tj_lo, tj_hi, (int)ntiles, info, prio);
}

void launch_syrk_update_half(float *H, int64_t ld, const void *Lh, int slot0, int64_t sstride, int skip0, int np,
                             int half, int64_t r0, int t, int tj_lo, int tj_hi, const unsigned long long *info,
                             hipStream_t st, int prio, int max_grid)
{
    if (t <= 0 || tj_lo >= tj_hi || np <= 0) return;
    int64_t ntiles = 0;
    for (int c = tj_lo; c < tj_hi; ++c) ntiles += t - c;
    int64_t grid = ((ntiles + 7) / 8) * 8;
    if (max_grid > 0 && grid > max_grid) grid = (max_grid / 8) * 8;
    if (half == HALF_F16)
        hipLaunchKernelGGL(k_syrk_update_h<HALF_F16>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, Lh, slot0,
                           sstride, skip0, np, r0, t, tj_lo, tj_hi, (int)ntiles, info, prio);
    else
        hipLaunchKernelGGL(k_syrk_update_h<HALF_BF16>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, Lh, slot0,
                           sstride, skip0, np, r0, t, tj_lo, tj_hi, (int)ntiles, info, prio);
}

// Below this many 128-tiles a binary32 update runs on 64-tiles (SPD_SMALL_TILES overrides).
static int small_update_tiles()
{
    static const int v = [] {
        const char *e = std::getenv("SPD_SMALL_TILES");
        return e ? std::atoi(e) : 512;
    }();
    return v;
}
#define kSmallUpdateTiles small_update_tiles()

// Workgroups of the binary32 128-tile update resident at once on the current
// device (two per compute unit), or 0 when the last round is not to be split
// into 64-tiles (SPD_TAIL_SPLIT=0).
static int update_slots()
{
    static const bool off = [] {
        const char *e = std::getenv("SPD_TAIL_SPLIT");
        return e && std::atoi(e) == 0;
    }();
    if (off) return 0;
    static std::atomic<int> cache[64];  // per device; threads that race store the same value
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (!v) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            return 0;
        v = 2 * cus;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Whole rounds of 128-tiles over P workgroups (P = the cap, else every
// resident slot); when the last round has at most P/2 tiles, those run as
// 64-tiles inside the same launch (at most two per workgroup).  An uncapped
// launch of more than two rounds keeps one workgroup per tile: the hardware
// hands tiles to slots as they free up, which balances better than fixed
// rounds once other streams hold some slots.  Returns the tiles that run
// whole; *grid is the launch's workgroup count.
static int64_t update_split(int64_t ntiles, int64_t max_grid, int64_t *grid)
{
    *grid = ((ntiles + 7) / 8) * 8;
    if (max_grid > 0 && *grid > max_grid) *grid = (max_grid / 8) * 8;
    const int slots = update_slots();
    if (slots < 8 || (max_grid <= 0 && ntiles > 2 * (int64_t)slots)) return ntiles;
    int64_t P = (max_grid > 0) ? std::min<int64_t>(max_grid, slots) : slots;
    P = (P / 8) * 8;
    if (P < 8) return ntiles;
    const int64_t per = P / 8, rounds = ((ntiles + 7) / 8 + per - 1) / per;
    const int64_t nfull = (rounds - 1) * 8 * per, rem = ntiles - nfull;
    if (rem > P / 2) return ntiles;
    *grid = (nfull > 0) ? P : std::min<int64_t>(P, ((4 * rem + 7) / 8) * 8);
    return nfull;
}

template <typename T>
void launch_syrk_update(T *H, int64_t ld, int64_t k0, int nbk, int64_t r0, int t, int tj_lo, int tj_hi,
                        const unsigned long long *info, hipStream_t st, int prio, int max_grid, bool small_tiles)
{
    if (t <= 0 || tj_lo >= tj_hi) return;
    int64_t ntiles = 0;
    for (int c = tj_lo; c < tj_hi; ++c) ntiles += t - c;
    int64_t grid = ((ntiles + 7) / 8) * 8;
    if (max_grid > 0 && grid > max_grid) grid = (max_grid / 8) * 8;
    if constexpr (sizeof(T) == 4) {
        if (small_tiles && ntiles < kSmallUpdateTiles && max_grid == 0) {
            // too few 128-tiles for the chip: 64-tiles, four times as many workgroups
            const int t2 = 2 * t, lo2 = 2 * tj_lo, hi2 = 2 * tj_hi;
            int64_t n2 = 0;
            for (int c = lo2; c < hi2; ++c) n2 += t2 - c;
            const int64_t g2 = ((n2 + 7) / 8) * 8;
            hipLaunchKernelGGL(k_syrk_update_f32<64>, dim3((unsigned)g2), dim3(256), 0, st, H, ld, k0, nbk, r0, t2,
                               lo2, hi2, (int)n2, (int)n2, info, prio);
        } else {
            const int64_t nfull = update_split(ntiles, max_grid, &grid);
            hipLaunchKernelGGL(k_syrk_update_f32<128>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, k0, nbk, r0,
                               t, tj_lo, tj_hi, (int)ntiles, (int)nfull, info, prio);
        }
    } else
        hipLaunchKernelGGL(k_syrk_update<T>, dim3((unsigned)grid), dim3(256), 0, st, H, ld, k0, nbk, r0, t, tj_lo,
                           tj_hi, (int)ntiles, info, prio);
}
template void launch_syrk_update<float>(float *, int64_t, int64_t, int, int64_t, int, int, int,
                                        const unsigned long long *, hipStream_t, int, int, bool);
template void launch_syrk_update<double>(double *, int64_t, int64_t, int, int64_t, int, int, int,
                                         const unsigned long long *, hipStream_t, int, int, bool);

}  // namespace spd
