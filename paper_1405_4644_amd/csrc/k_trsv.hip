// Triangular solves with the low-precision factor (Eq. (3): forward L y = b,
// backward L^T x = y), blocked by big diagonal blocks of NBS (1024) rows.
//
// Set-up, once per factorisation: W_k = L_kk^{-1} for every big diagonal
// block, built from the 128-wide block inverses by repeated doubling,
//   [W11 0; W21 W22] with W21 = -W22 (L21 W11),
// two batched MFMA products per doubling level.
//
// Solve, one persistent launch per direction.  With K big blocks the forward
// solve is z_k = W_k (b_k - sum_{j<k} L_kj z_j).  It is cut into tasks of R
// rows (32 binary32 / 16 binary64):
//   U(j, i, c): P_ij[c] = L_ij[rows c] z_j          (j < i)
//   Z(i, c)   : z_i[c]  = W_i[rows c] (b_i - sum_j P_ij)
// handed out by an atomic counter column by column (Z(j), U(j, j+1), ...,
// U(j, K-1)), which is a topological order: every task waits only on tasks
// handed out before it, so progress never depends on how many workgroups are
// resident, and the bandwidth-bound U tasks run well ahead of the chain.
// A task loads its matrix block into registers before it waits, so the wait
// hides the load.  Z(i) sums the partials of blocks j <= i-2 (finished a step
// earlier) before it waits for the newest ones, U(i-1, i), so the critical
// path per big block is one Z and one U task.  Partials are summed in a fixed
// order: results do not depend on timing.  The backward solve is the mirror
// image with transposed blocks (x_k = W_k^T (y_k - sum_{j>k} L_jk^T x_j)).
//
// Waits are bounded: after ~1 s without progress a workgroup raises the
// error flag and leaves; every other waiter sees the flag and leaves too.
//
// Publishing a task's results: each XCD has its own L2, and a release fence
// at agent scope writes that whole cache back to memory; once per task it
// cuts the kernel's streaming rate about threefold.  Results that other
// workgroups read are therefore written with agent-scope stores (coherent
// across the L2s by themselves), and publishing waits only for those stores
// to complete before the counter is raised.  The waiting side reads them
// with agent-scope loads in turn, so it needs no acquire fence (an L2
// invalidate) either.
#include "common.h"
#include "internal.h"

#define TRSV_NBS 1024                    // big diagonal block
#define TRSV_NCRIT 64                    // workgroups on the chain's tasks
#define TRSV_NBULK 192                   // workgroups streaming the other blocks
#define TRSV_CDEPTH 1                    // U(p, p+d) tasks taken by the chain: d <= this

// thread 0 only: wait until *addr >= want, or give up after `tmo` ticks of
// wall_clock64 (100 MHz on gfx9) or as soon as another wait has given up.
// The polling loads are relaxed agent-scope atomics (coherent loads that do
// not invalidate the caches).
SPD_DEV bool wait_ge(int *addr, int want, int *err, unsigned long long tmo)
{
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        if (wall_clock64() - t0 > tmo) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// a result that other workgroups read (agent-coherent store), and its read
template <typename T>
SPD_DEV void store_shared(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
SPD_DEV T load_shared(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Big-block inverses.
// WB holds K blocks of nbs x nbs (column-major, leading dimension nbs); block
// k covers rows [k nbs, k nbs + s_k), s_k = min(nbs, npad - k nbs).
__global__ __launch_bounds__(256) void k_inv_init_f(const float *__restrict__ W128, int64_t npad, int nbs,
                                                    float *__restrict__ WB)
{
    // one workgroup per 128-block b: WB_kb[128 i + r][128 i + c] = W128_b[r][c]
    const int64_t b = blockIdx.x, g = b * 128, kb = g / nbs, i = (g - kb * nbs) / 128;
    float *dst = WB + kb * nbs * nbs + 128 * i + 128 * i * nbs;
    const float *src = W128 + b * 128 * 128;
    for (int idx = threadIdx.x; idx < 128 * 128; idx += 256)
        dst[(idx % 128) + (int64_t)(idx / 128) * nbs] = src[idx];
}
__global__ __launch_bounds__(256) void k_inv_init_d(const double *__restrict__ W128, int64_t npad, int nbs,
                                                    double *__restrict__ WB)
{
    const int64_t b = blockIdx.x, g = b * 128, kb = g / nbs, i = (g - kb * nbs) / 128;
    double *dst = WB + kb * nbs * nbs + 128 * i + 128 * i * nbs;
    const double *src = W128 + b * 128 * 128;
    for (int idx = threadIdx.x; idx < 128 * 128; idx += 256)
        dst[(idx % 128) + (int64_t)(idx / 128) * nbs] = src[idx];
}

// One doubling level of width s.  Workgroup (x, y, z): output tile (x, y) of
// pair p of big block kb (z = kb * ppb + p); the pair is [a0, a1) + [a1, b1)
// inside the block.  PHASE 1: Tk = L21 W11 (W11 lower: k >= 128 y);
// PHASE 2: W21 = -W22 Tk (W22 lower: k < 128 (x + 1)).  128 x 128 tiles on
// MFMA, computed transposed so that each lane stores contiguous rows.
template <typename T, int PHASE>
__global__ __launch_bounds__(256) void k_inv_merge(const T *__restrict__ L, int64_t ld, int64_t npad,
                                                   T *__restrict__ WB, int nbs, int s, T *__restrict__ Tb)
{
    constexpr int KC = sizeof(T) == 4 ? 32 : 16;
    constexpr int LDA = 128 + 4, LDB = KC + 1;
    __shared__ T As[KC * LDA];   // As[k * LDA + m]
    __shared__ T Bs[128 * LDB];  // Bs[n * LDB + k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ppb = (nbs + 2 * s - 1) / (2 * s);
    const int kb = blockIdx.z / ppb, p = blockIdx.z % ppb;
    const int64_t o = (int64_t)kb * nbs;
    const int sk = (int)((npad - o) < nbs ? (npad - o) : nbs);
    const int a0 = 2 * p * s, a1 = a0 + s, b1 = (a0 + 2 * s < sk) ? a0 + 2 * s : sk;
    if (a1 >= sk)
        return;
    const int M = b1 - a1;
    const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
    if (m0 >= M)
        return;
    T *Wk = WB + (int64_t)kb * nbs * nbs;
    T *Tk = Tb + (int64_t)blockIdx.z * s * s;
    const T *A, *B;
    T *Cp;
    int64_t lda, ldb, ldc;
    int kbeg, kend;
    T alpha;
    if (PHASE == 1) {
        A = L + (o + a1) + (o + a0) * ld;
        lda = ld;
        B = Wk + a0 + (int64_t)a0 * nbs;
        ldb = nbs;
        Cp = Tk;
        ldc = s;
        kbeg = n0;
        kend = s;
        alpha = (T)1;
    } else {
        A = Wk + a1 + (int64_t)a1 * nbs;
        lda = nbs;
        B = Tk;
        ldb = s;
        Cp = Wk + a1 + (int64_t)a0 * nbs;
        ldc = nbs;
        kbeg = 0;
        kend = (m0 + 128 < M) ? m0 + 128 : M;
        alpha = (T)-1;
    }
    const int wn = wave >> 1, wm = wave & 1;
    Acc32<T> acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b].zero();
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
        __syncthreads();
        copy_g2s<T, 128, 256, 8>(As, LDA, A + m0 + (int64_t)k0 * lda, lda, KC, tid);
        copy_g2s<T, KC, 256, 8>(Bs, LDB, B + k0 + (int64_t)n0 * ldb, ldb, 128, tid);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KC; kk += Frag<T>::K) {
            if constexpr (sizeof(T) == 4) {
                float fa[2], fb[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    fa[q] = Bs[(64 * wn + 32 * q + (lane & 31)) * LDB + kk + (lane >> 5)];
                    fb[q] = As[(kk + (lane >> 5)) * LDA + 64 * wm + 32 * q + (lane & 31)];
                }
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi) acc[ni][mi].mma(fa[ni], fb[mi]);
            } else {
                double fa[2][2], fb[2][2];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        fa[q][h] = Bs[(64 * wn + 32 * q + 16 * h + (lane & 15)) * LDB + kk + (lane >> 4)];
                        fb[q][h] = As[(kk + (lane >> 4)) * LDA + 64 * wm + 32 * q + 16 * h + (lane & 15)];
                    }
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi) acc[ni][mi].mma(fa[ni], fb[mi]);
            }
        }
    }
    // register j of acc[ni][mi]: n = 64 wn + 32 ni + row(j), m = 64 wm + 32 mi + col(j)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int n = 64 * wn + 32 * ni + Acc32<T>::row(j, lane);
                const int m = 64 * wm + 32 * mi + Acc32<T>::col(j, lane);
                Cp[(m0 + m) + (int64_t)(n0 + n) * ldc] = alpha * acc[ni][mi].get(j);
            }
}

// ---------------------------------------------------------------------------
// Register-resident block times vector.
//   FWD (rows form):  out[r] = sum_c M[r][c] v[c], R rows, columns [0, ncols)
//   BWD (cols form):  out[c] = sum_r M[r][c] v[r0 + r], R columns, rows [0, nrows)
// M is column-major (leading dimension ld).  VEC elements per 16-byte load;
// R = 8 VEC; every thread holds E = NBS / 32 vectors.
template <typename T> struct VecOf;
template <> struct VecOf<float> { using V = float4; static constexpr int N = 4; };
template <> struct VecOf<double> { using V = double2; static constexpr int N = 2; };

template <typename T>
SPD_DEV T vget(const typename VecOf<T>::V &v, int r)
{
    if constexpr (sizeof(T) == 4)
        return r == 0 ? v.x : r == 1 ? v.y : r == 2 ? v.z : v.w;
    else
        return r == 0 ? v.x : v.y;
}

template <typename T, int MC, bool FWD, int NBS>
struct BlockVec {
    using V = typename VecOf<T>::V;
    static constexpr int VEC = VecOf<T>::N;
    static constexpr int R = 8 * VEC;      // rows (FWD) / columns (BWD) per task
    static constexpr int E = NBS / 32;     // vectors per thread
    static constexpr int TPC = 256 / R;    // BWD: threads per column
    V m[E];

    // FWD: thread t covers rows VEC (t % 8) .. +VEC of columns t / 8 + 32 e.
    // BWD: thread t covers column t / TPC, rows VEC (t % TPC) + 32 e .. +VEC.
    SPD_DEV void load(const T *base, int64_t ld, int len, int tid)
    {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (FWD) {
                const int col = tid / 8 + 32 * e;
                if (col < len)
                    m[e] = *(const V *)(base + VEC * (tid % 8) + (int64_t)col * ld);
            } else {
                const int row = VEC * (tid % TPC) + 32 * e;
                if (row < len)
                    m[e] = *(const V *)(base + row + (int64_t)(tid / TPC) * ld);
            }
        }
    }

    // out[r][cc] for r < R (valid in thread tid < R * MC as (tid % R, tid / R)
    // for FWD; in the thread with tid % TPC == 0 for column tid / TPC for BWD)
    SPD_DEV void apply(const T (*vs)[NBS], int len, int r0, T (*red)[R][MC], T out[MC], int tid)
    {
        const int lane = tid & 63, wave = tid >> 6;
        if constexpr (FWD) {
            T acc[VEC][MC];
#pragma unroll
            for (int r = 0; r < VEC; ++r)
#pragma unroll
                for (int cc = 0; cc < MC; ++cc) acc[r][cc] = (T)0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int col = tid / 8 + 32 * e;
                if (col < len) {
#pragma unroll
                    for (int cc = 0; cc < MC; ++cc) {
                        const T x = vs[cc][col];
#pragma unroll
                        for (int r = 0; r < VEC; ++r) acc[r][cc] += vget<T>(m[e], r) * x;
                    }
                }
            }
            // sum over the 8 column groups of this wave (lane bits 3..5), then over waves
#pragma unroll
            for (int sh = 8; sh < 64; sh <<= 1)
#pragma unroll
                for (int r = 0; r < VEC; ++r)
#pragma unroll
                    for (int cc = 0; cc < MC; ++cc) acc[r][cc] += __shfl_xor(acc[r][cc], sh);
            if (lane < 8) {
#pragma unroll
                for (int r = 0; r < VEC; ++r)
#pragma unroll
                    for (int cc = 0; cc < MC; ++cc) red[wave][VEC * lane + r][cc] = acc[r][cc];
            }
            __syncthreads();
            if (tid < R * MC) {
                const int r = tid % R, cc = tid / R;
                out[0] = ((red[0][r][cc] + red[1][r][cc]) + red[2][r][cc]) + red[3][r][cc];
            }
        } else {
            T acc[MC];
#pragma unroll
            for (int cc = 0; cc < MC; ++cc) acc[cc] = (T)0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int row = VEC * (tid % TPC) + 32 * e;
                if (row < len) {
#pragma unroll
                    for (int r = 0; r < VEC; ++r) {
                        const T a = vget<T>(m[e], r);
#pragma unroll
                        for (int cc = 0; cc < MC; ++cc) acc[cc] += a * vs[cc][r0 + row + r];
                    }
                }
            }
#pragma unroll
            for (int sh = 1; sh < TPC; sh <<= 1)
#pragma unroll
                for (int cc = 0; cc < MC; ++cc) acc[cc] += __shfl_xor(acc[cc], sh);
#pragma unroll
            for (int cc = 0; cc < MC; ++cc) out[cc] = acc[cc];
        }
    }
};

// geometry of big block k
SPD_DEV void big_block(int64_t npad, int nbs, int k, int64_t &o, int &sz)
{
    o = (int64_t)k * nbs;
    sz = (int)((npad - o) < nbs ? (npad - o) : nbs);
}

template <typename T, int MC, bool FWD>
__global__ __launch_bounds__(256) void k_trsv_blk(const T *__restrict__ L, int64_t ld, const T *__restrict__ WB,
                                                  int64_t npad, int nbs, int K, const T *__restrict__ Yin,
                                                  T *__restrict__ Zout, int64_t ldy, int c0, int m,
                                                  T *__restrict__ P, int *ctl, int *err, int ncrit, int cdepth,
                                                  unsigned long long tmo)
{
    constexpr int NBS = TRSV_NBS;
    using BV = BlockVec<T, MC, FWD, NBS>;
    constexpr int R = BV::R;
    // vector entries per thread, and partials summed per batch of loads
    constexpr int PER = MC * NBS / 256, QB = PER >= 32 ? 1 : 32 / PER;
    __shared__ T vs[MC][NBS];
    __shared__ T red[4][R][MC];
    __shared__ int s_task, s_ok, s_crit;
    const int tid = threadIdx.x;
    int *qcrit = ctl, *qbulk = ctl + 1, *ticket = ctl + 2;
    int *cntA = ctl + 3, *cntB = ctl + 3 + K, *cntZ = ctl + 3 + 2 * K;
    const int mc = min(MC, m - c0);
    BV bv;
    // Blocks in processing order p (FWD: block p; BWD: block K-1-p); only
    // block K-1 may be shorter than nbs.
    const int slast = (int)(npad - (int64_t)(K - 1) * nbs);
    auto proc_size = [&](int p) -> int { return (FWD ? p == K - 1 : p == 0) ? slast : nbs; };
    auto rows_before = [&](int p) -> int64_t {
        return FWD ? (int64_t)p * nbs : (p == 0 ? 0 : slast + (int64_t)(p - 1) * nbs);
    };
    auto proc_locate = [&](int64_t pos, int &p, int &off) {
        if (FWD) {
            p = (int)(pos / nbs);
            off = (int)(pos - (int64_t)p * nbs);
        } else if (pos < slast) {
            p = 0;
            off = (int)pos;
        } else {
            p = 1 + (int)((pos - slast) / nbs);
            off = (int)((pos - slast) % nbs);
        }
    };

    // The first ncrit workgroups to start take the chain's tasks in step
    // order: every Z(p), the U(p, p+1) that feeds the next Z, and the U(p,
    // p+d) for d <= cdepth; the others take the remaining U tasks column by
    // column.  A workgroup that has started is resident, so the chain never
    // waits for a workgroup that cannot run.
    if (tid == 0)
        s_crit = atomicAdd(ticket, 1) < ncrit;
    __syncthreads();
    const bool crit = s_crit != 0;
    for (;;) {
        if (tid == 0)
            s_task = atomicAdd(crit ? qcrit : qbulk, 1);
        __syncthreads();
        int rem = s_task, pi = -1, pj = -1, c = 0;
        if (crit) {
            // step p: Z(p, 0..), then U(p, p+d, 0..) for d = 1 .. cdepth
            for (int p = 0; p < K && pi < 0; ++p) {
                for (int d = 0; d <= cdepth && p + d < K; ++d) {
                    const int nt = proc_size(p + d) / R;
                    if (rem < nt) {
                        pj = p;
                        pi = p + d;
                        c = rem;
                        break;
                    }
                    rem -= nt;
                }
            }
        } else {
            // column q: U(q, pi, 0..) for the blocks pi from q+1+cdepth on
            for (int q = 0; q + 1 + cdepth < K; ++q) {
                const int cnt = (int)((npad - rows_before(q + 1 + cdepth)) / R);
                if (rem < cnt) {
                    int off;
                    proc_locate(rows_before(q + 1 + cdepth) + (int64_t)rem * R, pi, off);
                    pj = q;
                    c = off / R;
                    break;
                }
                rem -= cnt;
            }
        }
        if (pi < 0)
            return;
        const int nc = proc_size(pi) / R;
        const bool ztask = (pj == pi);
        const int ki = FWD ? pi : K - 1 - pi, kj = FWD ? pj : K - 1 - pj;
        int64_t oi, oj;
        int si, sj;
        big_block(npad, nbs, ki, oi, si);
        big_block(npad, nbs, kj, oj, sj);
        T *Pbase = P + ((int64_t)pi * (pi - 1) / 2) * NBS * MC;  // partials of row pi
        const T *Wk = WB + (int64_t)ki * nbs * nbs;

        // The task's matrix block, loaded before any wait:
        //   U: the block of L coupling ki and kj (entries c R .. +R of block ki);
        //   Z: rows (FWD) / columns (BWD) c R .. +R of W_ki.
        // Vector range it needs: U [0, sj); Z FWD [0, (c+1) R), BWD [c R, si).
        const T *mb;
        int64_t mld;
        int lo, hi;
        if (!ztask) {
            mb = FWD ? L + (oi + c * R) + oj * ld : L + oj + (oi + c * R) * ld;
            mld = ld;
            lo = 0;
            hi = sj;
        } else {
            mb = FWD ? Wk + c * R : Wk + c * R + (int64_t)(c * R) * nbs;
            mld = nbs;
            lo = FWD ? 0 : c * R;
            hi = FWD ? (c + 1) * R : si;
        }
        bv.load(mb, mld, hi - lo, tid);

        if (!ztask) {
            if (tid == 0)
                s_ok = wait_ge(&cntZ[pj], sj / R, err, tmo) ? 1 : 0;
            __syncthreads();
            if (!s_ok)
                return;
            // all of this thread's loads issued before the first use
            T zv[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int t = (tid + 256 * k) % NBS, cc = (tid + 256 * k) / NBS;
                zv[k] = (t < sj && cc < mc) ? load_shared(&Zout[(oj + t) + (int64_t)(c0 + cc) * ldy]) : (T)0;
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int t = (tid + 256 * k) % NBS, cc = (tid + 256 * k) / NBS;
                if (t < sj)
                    vs[cc][t] = zv[k];
            }
        } else {
            if (pi >= 2) {
                if (tid == 0)
                    s_ok = wait_ge(&cntA[pi], (pi - 1) * nc, err, tmo) ? 1 : 0;
                __syncthreads();
                if (!s_ok)
                    return;
            }
            // v = y - (sum of the partials of blocks finished a step ago), in
            // order of q; the loads go out QB partials at a time
            T sA[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) sA[k] = (T)0;
            for (int q0 = 0; q0 + 1 < pi; q0 += QB) {
                T pv[QB][PER];
#pragma unroll
                for (int u = 0; u < QB; ++u)
#pragma unroll
                    for (int k = 0; k < PER; ++k) {
                        const int t = (tid + 256 * k) % NBS, cc = (tid + 256 * k) / NBS;
                        pv[u][k] = (q0 + u + 1 < pi && t >= lo && t < hi)
                                       ? load_shared(&Pbase[(int64_t)(q0 + u) * NBS * MC + cc * NBS + t])
                                       : (T)0;
                    }
#pragma unroll
                for (int u = 0; u < QB; ++u)
#pragma unroll
                    for (int k = 0; k < PER; ++k)
                        if (q0 + u + 1 < pi)
                            sA[k] += pv[u][k];
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int t = (tid + 256 * k) % NBS, cc = (tid + 256 * k) / NBS;
                if (t >= lo && t < hi)
                    vs[cc][t] = (cc < mc) ? Yin[(oi + t) + (int64_t)(c0 + cc) * ldy] - sA[k] : (T)0;
            }
            if (pi >= 1) {
                if (tid == 0)
                    s_ok = wait_ge(&cntB[pi], nc, err, tmo) ? 1 : 0;
                __syncthreads();
                if (!s_ok)
                    return;
                const T *pB = Pbase + (int64_t)(pi - 1) * NBS * MC;
                T bv_[PER];
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int t = (tid + 256 * k) % NBS, cc = (tid + 256 * k) / NBS;
                    bv_[k] = (t >= lo && t < hi) ? load_shared(&pB[cc * NBS + t]) : (T)0;
                }
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int t = (tid + 256 * k) % NBS, cc = (tid + 256 * k) / NBS;
                    if (t >= lo && t < hi)
                        vs[cc][t] -= bv_[k];
                }
            }
        }
        __syncthreads();
        T out[MC];
        bv.apply(vs, hi - lo, lo, red, out, tid);

        // results: U -> partial P_{pi,pj}; Z -> solution entries of block ki
        T *dst;
        int64_t dcol;
        int nvalid;
        if (!ztask) {
            dst = Pbase + (int64_t)pj * NBS * MC + c * R;
            dcol = NBS;
            nvalid = MC;
        } else {
            dst = Zout + oi + c * R + (int64_t)c0 * ldy;
            dcol = ldy;
            nvalid = mc;
        }
        if (FWD) {
            if (tid < R * MC && tid / R < nvalid)
                store_shared(&dst[tid % R + (tid / R) * dcol], out[0]);
        } else if (tid % BV::TPC == 0) {
#pragma unroll
            for (int cc = 0; cc < MC; ++cc)
                if (cc < nvalid)
                    store_shared(&dst[tid / BV::TPC + cc * dcol], out[cc]);
        }
        // every thread's result stores complete, then one relaxed increment
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            int *ctr = ztask ? &cntZ[pi] : (pj == pi - 1 ? &cntB[pi] : &cntA[pi]);
            __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_zero_int(int *p, int count)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < count)
        p[i] = 0;
}

namespace spd {

int solve_nbs(int64_t npad) { return (int)(npad < TRSV_NBS ? npad : TRSV_NBS); }
int solve_nblocks(int64_t npad) { return (int)((npad + solve_nbs(npad) - 1) / solve_nbs(npad)); }

int64_t solve_winv_elems(int64_t npad)
{
    const int64_t nbs = solve_nbs(npad);
    return solve_nblocks(npad) * nbs * nbs;
}

int64_t solve_tmp_elems(int64_t npad)
{
    const int nbs = solve_nbs(npad), K = solve_nblocks(npad);
    int64_t mx = 1;
    for (int s = 128; s < nbs; s *= 2) {
        const int64_t ppb = (nbs + 2 * s - 1) / (2 * s);
        mx = std::max<int64_t>(mx, K * ppb * (int64_t)s * s);
    }
    return mx;
}

int64_t trsv_scratch_elems(int64_t npad)
{
    const int64_t K = solve_nblocks(npad);
    return std::max<int64_t>(K * (K - 1) / 2, 1) * TRSV_NBS * TRSV_MC;
}

// counters of one direction, padded to 256 bytes (a caller keeping one set
// per direction back to back keeps each on lines of its own)
int trsv_ctl_ints(int64_t npad) { return (3 + 3 * solve_nblocks(npad) + 63) & ~63; }

template <typename T>
void launch_build_winv(const T *L, int64_t ld, int64_t npad, const T *W128, T *WB, T *Tb, hipStream_t st)
{
    const int nbs = solve_nbs(npad), K = solve_nblocks(npad);
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL(k_inv_init_f, dim3((unsigned)(npad / 128)), dim3(256), 0, st, W128, npad, nbs, WB);
    else
        hipLaunchKernelGGL(k_inv_init_d, dim3((unsigned)(npad / 128)), dim3(256), 0, st, W128, npad, nbs, WB);
    for (int s = 128; s < nbs; s *= 2) {
        const int ppb = (nbs + 2 * s - 1) / (2 * s);
        const dim3 grid((unsigned)(s / 128), (unsigned)(s / 128), (unsigned)(K * ppb));
        hipLaunchKernelGGL((k_inv_merge<T, 1>), grid, dim3(256), 0, st, L, ld, npad, WB, nbs, s, Tb);
        hipLaunchKernelGGL((k_inv_merge<T, 2>), grid, dim3(256), 0, st, L, ld, npad, WB, nbs, s, Tb);
    }
}
template void launch_build_winv<float>(const float *, int64_t, int64_t, const float *, float *, float *,
                                       hipStream_t);
template void launch_build_winv<double>(const double *, int64_t, int64_t, const double *, double *, double *,
                                        hipStream_t);

template <typename T, bool FWD>
static void launch_dir(const T *L, int64_t ld, const T *WB, int64_t npad, int m, const T *Yin, T *Zout,
                       int64_t ldy, T *P, int *ctl, bool ctl_zeroed, int *err, unsigned long long tmo,
                       hipStream_t st)
{
    const int nbs = solve_nbs(npad), K = solve_nblocks(npad);
    constexpr int R = 8 * VecOf<T>::N;
    // chain tasks: every Z and U(p, p+d), d <= TRSV_CDEPTH; the other U
    // tasks stream
    const int cdepth = TRSV_CDEPTH;
    int64_t ncrit_tasks = 0, nbulk_tasks = 0;
    for (int p = 0; p < K; ++p) {
        const int64_t o = (int64_t)p * nbs, sz = std::min<int64_t>(nbs, npad - o);
        ncrit_tasks += (1 + std::min(p, cdepth)) * (sz / R);
        nbulk_tasks += std::max(p - cdepth, 0) * (sz / R);
    }
    const int ncrit = (int)std::min<int64_t>(ncrit_tasks, TRSV_NCRIT);
    const int grid = ncrit + (int)std::min<int64_t>(nbulk_tasks, TRSV_NBULK);
    const int nctl = trsv_ctl_ints(npad);
    for (int c0 = 0; c0 < m; c0 += TRSV_MC) {
        if (c0 > 0 || !ctl_zeroed)
            hipLaunchKernelGGL(k_zero_int, dim3((nctl + 255) / 256), dim3(256), 0, st, ctl, nctl);
        const int mc = m - c0;
        if (mc == 1)
            hipLaunchKernelGGL((k_trsv_blk<T, 1, FWD>), dim3(grid), dim3(256), 0, st, L, ld, WB, npad, nbs, K, Yin,
                               Zout, ldy, c0, m, P, ctl, err, ncrit, cdepth, tmo);
        else if (mc == 2)
            hipLaunchKernelGGL((k_trsv_blk<T, 2, FWD>), dim3(grid), dim3(256), 0, st, L, ld, WB, npad, nbs, K, Yin,
                               Zout, ldy, c0, m, P, ctl, err, ncrit, cdepth, tmo);
        else if (mc <= 4)
            hipLaunchKernelGGL((k_trsv_blk<T, 4, FWD>), dim3(grid), dim3(256), 0, st, L, ld, WB, npad, nbs, K, Yin,
                               Zout, ldy, c0, m, P, ctl, err, ncrit, cdepth, tmo);
        else
            hipLaunchKernelGGL((k_trsv_blk<T, TRSV_MC, FWD>), dim3(grid), dim3(256), 0, st, L, ld, WB, npad, nbs, K,
                               Yin, Zout, ldy, c0, m, P, ctl, err, ncrit, cdepth, tmo);
    }
}

template <typename T>
void launch_trsv(const T *L, int64_t ld, const T *WB, int64_t npad, int m, T *Y, T *Z, int64_t ldy, T *P, int *ctl,
                 bool ctl_zeroed, int *err, unsigned long long wait_ticks, hipStream_t st)
{
    // each direction has its own counters (ctl, ctl + trsv_ctl_ints)
    launch_dir<T, true>(L, ld, WB, npad, m, Y, Z, ldy, P, ctl, ctl_zeroed, err, wait_ticks, st);
    launch_dir<T, false>(L, ld, WB, npad, m, Z, Y, ldy, P, ctl + trsv_ctl_ints(npad), ctl_zeroed, err, wait_ticks,
                         st);
}
template void launch_trsv<float>(const float *, int64_t, const float *, int64_t, int, float *, float *, int64_t,
                                 float *, int *, bool, int *, unsigned long long, hipStream_t);
template void launch_trsv<double>(const double *, int64_t, const double *, int64_t, int, double *, double *, int64_t,
                                  double *, int *, bool, int *, unsigned long long, hipStream_t);

}  // namespace spd
