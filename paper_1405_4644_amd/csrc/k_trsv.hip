// Triangular solves with the low-precision factor in one persistent launch
// per direction (Eq. (3): forward L y = b, backward L^T x = y).
//
// The factor is cut into SB x SB blocks (ns = npad / SB block rows).  The
// forward solve needs z_k = W_kk (b_k - sum_{j<k} L_kj z_j), W_kk = L_kk^{-1}
// (the diagonal blocks of the stored per-panel inverses).  Work items:
//   item 0          : z_0 = W_00 b_0
//   item (k, j), j<k: P_kj = L_kj z_j ; the item with j = k-1 is "designated":
//                     it also waits for the other partials of row k, forms
//                     z_k = W_kk (b_k - sum_j P_kj) and publishes z_k.
// Items are handed out by an atomic counter in column-major order of the
// strictly lower block triangle, which is a topological order: every item
// waits only on items handed out before it, so progress does not depend on
// how many workgroups are resident.  The backward solve is the mirror image
// with transposed blocks (x_k = W_kk^T (y_k - sum_{j>k} L_jk^T x_j)).
//
// Waits are bounded: after ~1 s without progress a workgroup raises the
// error flag and leaves; every other waiter sees the flag and leaves too.
#include "common.h"
#include "internal.h"

#define TRSV_TIMEOUT_TICKS 100000000ULL  // wall_clock64 runs at 100 MHz on gfx9

// thread 0 only: wait until *addr >= want, or give up.  The polling loads are
// relaxed agent-scope atomics (coherent loads that do not invalidate the
// caches); the caller issues one acquire fence after a successful wait.
SPD_DEV bool wait_ge(int *addr, int want, int *err)
{
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        if (wall_clock64() - t0 > TRSV_TIMEOUT_TICKS) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// every thread: make this workgroup's global stores complete, then thread 0
// publishes with one release operation
SPD_DEV void publish_barrier()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// item q >= 1 -> (r, c), r > c, column-major over the strictly lower triangle of ns x ns
SPD_DEV void decode_item(int q, int ns, int &r, int &c)
{
    // prefix(c) = c (2 ns - 1 - c) / 2 items precede column c
    const double b = 2.0 * ns - 1.0;
    int j = (int)((b - sqrt(b * b - 8.0 * q)) * 0.5);
    if (j < 0) j = 0;
    while (j > 0 && (long long)j * (2 * ns - 1 - j) / 2 > q) --j;
    while ((long long)(j + 1) * (2 * ns - 2 - j) / 2 <= q) ++j;
    c = j;
    r = j + 1 + (q - (int)((long long)j * (2 * ns - 1 - j) / 2));
}

// Stage an SB x SB block (column-major source, leading dimension ld) into LDS
// as Ms[c * (SB + 1) + r] = M[r][c].
template <typename T, int SB>
SPD_DEV void stage(T *Ms, const T *src, int64_t ld, int tid)
{
    copy_g2s<T, SB, 256, 16>(Ms, SB + 1, src, ld, SB, tid);
}

// out[i] = sum_t M(i, t) v[t] for the MC columns of v (vs[cc][t]); M in LDS.
// TRANS: M(i, t) = Ms^T, i.e. out = M^T v.  Result for row i is returned to
// the thread with (tid % SB) == i and tid < SB (others get garbage).
template <typename T, int SB, int MC, bool TRANS>
SPD_DEV void block_gemv(const T *Ms, const T (*vs)[SB], T (*red)[MC][SB], T out[MC], int tid)
{
    constexpr int PARTS = 256 / SB, SPAN = SB / PARTS;
    const int i = tid % SB, part = tid / SB;
    T acc[MC];
#pragma unroll
    for (int cc = 0; cc < MC; ++cc) acc[cc] = (T)0;
#pragma unroll 8
    for (int tt = 0; tt < SPAN; ++tt) {
        const int t = part * SPAN + tt;
        const T a = TRANS ? Ms[i * (SB + 1) + t] : Ms[t * (SB + 1) + i];
#pragma unroll
        for (int cc = 0; cc < MC; ++cc) acc[cc] += a * vs[cc][t];
    }
#pragma unroll
    for (int cc = 0; cc < MC; ++cc) red[part][cc][i] = acc[cc];
    __syncthreads();
    if (tid < SB) {
#pragma unroll
        for (int cc = 0; cc < MC; ++cc) {
            T s = red[0][cc][i];
#pragma unroll
            for (int p = 1; p < PARTS; ++p) s += red[p][cc][i];
            out[cc] = s;
        }
    }
}

template <typename T, int SB, int MC, bool FWD>
__global__ __launch_bounds__(256) void k_trsv_persist(const T *__restrict__ L, int64_t ld, const T *__restrict__ W,
                                                      int nbw, int ns, const T *__restrict__ Yin,
                                                      T *__restrict__ Zout, int64_t ldy, int c0, int m,
                                                      T *__restrict__ P, int *ctl, int *flags, int epoch,
                                                      int *err)
{
    __shared__ T Ms[SB * (SB + 1)];
    __shared__ T Ws[SB * (SB + 1)];
    __shared__ T vs[MC][SB];
    __shared__ T red[256 / SB][MC][SB];
    __shared__ int s_item, s_ok;
    const int tid = threadIdx.x;
    int *qhead = ctl, *cnt = ctl + 1;
    const int total = 1 + ns * (ns - 1) / 2;
    const int mc = min(MC, m - c0);

    for (;;) {
        if (tid == 0)
            s_item = atomicAdd(qhead, 1);
        __syncthreads();
        const int q = s_item;
        if (q >= total)
            return;
        // (row, col) of the item in the solve's own orientation
        int k, j;  // k: block row being accumulated; j: block whose solution is consumed
        bool diag_only = (q == 0), designated;
        if (diag_only) {
            k = FWD ? 0 : ns - 1;
            j = -1;
            designated = true;
        } else {
            int r, c;
            decode_item(q - 1, ns, r, c);
            k = FWD ? r : ns - 1 - r;
            j = FWD ? c : ns - 1 - c;
            designated = FWD ? (j == k - 1) : (j == k + 1);
        }
        // prefetch: the off-diagonal block and, for a designated item, W_kk
        if (!diag_only) {
            // forward: L_kj (rows k, cols j); backward: L_jk (rows j, cols k), used transposed
            const T *src = FWD ? L + (int64_t)k * SB + (int64_t)j * SB * ld : L + (int64_t)j * SB + (int64_t)k * SB * ld;
            stage<T, SB>(Ms, src, ld, tid);
        }
        if (designated) {
            const int64_t g = (int64_t)k * SB, b = g / nbw, o = g - b * nbw;
            stage<T, SB>(Ws, W + b * nbw * nbw + o + o * nbw, nbw, tid);
        }
        const int pk = FWD ? k : ns - 1 - k;  // row index in the forward-style triangle
        const int others = (diag_only || !designated) ? 0 : pk - 1;
        // a designated item first collects the other partials of its row
        // (usually ready long before the newest block), in a fixed order
        T psum[MC];
#pragma unroll
        for (int cc = 0; cc < MC; ++cc) psum[cc] = (T)0;
        if (others > 0) {
            if (tid == 0)
                s_ok = wait_ge(&cnt[k], others, err) ? 1 : 0;
            __syncthreads();
            if (!s_ok)
                return;
            if (tid < SB) {
                const T *pp = P + ((int64_t)pk * (pk - 1) / 2) * MC * SB + tid;
                for (int pj = 0; pj < others; ++pj)
#pragma unroll
                    for (int cc = 0; cc < MC; ++cc) psum[cc] += pp[(int64_t)pj * MC * SB + cc * SB];
            }
        }
        T own[MC];
#pragma unroll
        for (int cc = 0; cc < MC; ++cc) own[cc] = (T)0;
        if (!diag_only) {
            if (tid == 0)
                s_ok = wait_ge(&flags[j], epoch, err) ? 1 : 0;
            __syncthreads();
            if (!s_ok)
                return;
            for (int idx = tid; idx < MC * SB; idx += 256) {
                const int t = idx % SB, cc = idx / SB;
                vs[cc][t] = (cc < mc) ? Zout[((int64_t)j * SB + t) + (int64_t)(c0 + cc) * ldy] : (T)0;
            }
            __syncthreads();
            block_gemv<T, SB, MC, !FWD>(Ms, vs, red, own, tid);
        }
        if (!designated) {
            const int pj = FWD ? j : ns - 1 - j;
            T *pp = P + ((int64_t)pk * (pk - 1) / 2 + pj) * MC * SB;
            if (tid < SB)
#pragma unroll
                for (int cc = 0; cc < MC; ++cc) pp[cc * SB + tid] = own[cc];
            publish_barrier();
            if (tid == 0)
                __hip_atomic_fetch_add(&cnt[k], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        __syncthreads();  // red[] and vs[] reuse below
        if (tid < SB) {
            // v = y_k - (sum of the other partials + own)
#pragma unroll
            for (int cc = 0; cc < MC; ++cc) {
                const T y = (cc < mc) ? Yin[((int64_t)k * SB + tid) + (int64_t)(c0 + cc) * ldy] : (T)0;
                vs[cc][tid] = y - (psum[cc] + own[cc]);
            }
        }
        __syncthreads();
        T z[MC];
        block_gemv<T, SB, MC, !FWD>(Ws, vs, red, z, tid);
        if (tid < SB)
            for (int cc = 0; cc < mc; ++cc)
                Zout[((int64_t)k * SB + tid) + (int64_t)(c0 + cc) * ldy] = z[cc];
        publish_barrier();
        if (tid == 0)
            __hip_atomic_store(&flags[k], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_zero_int(int *p, int count)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < count)
        p[i] = 0;
}

namespace spd {

template <typename T> struct SolveBlk;
template <> struct SolveBlk<float> { static constexpr int SB = 128; };
template <> struct SolveBlk<double> { static constexpr int SB = 64; };

int trsv_block(int elem) { return elem == 4 ? SolveBlk<float>::SB : SolveBlk<double>::SB; }

int64_t trsv_scratch_elems(int64_t npad, int elem)
{
    const int64_t ns = npad / trsv_block(elem);
    return ns * (ns - 1) / 2 * TRSV_MC * trsv_block(elem);
}

template <typename T, bool FWD>
static int launch_dir(const T *L, int64_t ld, const T *W, int nbw, int64_t npad, int m, const T *Yin, T *Zout,
                      int64_t ldy, T *P, int *ctl, int *flags, int epoch, int *err, hipStream_t st)
{
    constexpr int SB = SolveBlk<T>::SB;
    const int ns = (int)(npad / SB);
    const int total = 1 + ns * (ns - 1) / 2;
    const int grid = total < 256 ? total : 256;  // one workgroup per CU fits the LDS budget
    for (int c0 = 0; c0 < m; c0 += TRSV_MC) {
        hipLaunchKernelGGL(k_zero_int, dim3((ns + 1 + 255) / 256), dim3(256), 0, st, ctl, ns + 1);
        const int mc = m - c0;
        if (mc == 1)
            hipLaunchKernelGGL((k_trsv_persist<T, SB, 1, FWD>), dim3(grid), dim3(256), 0, st, L, ld, W, nbw, ns, Yin,
                               Zout, ldy, c0, m, P, ctl, flags, epoch, err);
        else if (mc == 2)
            hipLaunchKernelGGL((k_trsv_persist<T, SB, 2, FWD>), dim3(grid), dim3(256), 0, st, L, ld, W, nbw, ns, Yin,
                               Zout, ldy, c0, m, P, ctl, flags, epoch, err);
        else if (mc <= 4)
            hipLaunchKernelGGL((k_trsv_persist<T, SB, 4, FWD>), dim3(grid), dim3(256), 0, st, L, ld, W, nbw, ns, Yin,
                               Zout, ldy, c0, m, P, ctl, flags, epoch, err);
        else
            hipLaunchKernelGGL((k_trsv_persist<T, SB, TRSV_MC, FWD>), dim3(grid), dim3(256), 0, st, L, ld, W, nbw,
                               ns, Yin, Zout, ldy, c0, m, P, ctl, flags, epoch, err);
        ++epoch;
    }
    return epoch;
}

template <typename T>
int launch_trsv_persist(const T *L, int64_t ld, const T *W, int nbw, int64_t npad, int m, T *Y, T *Z, int64_t ldy,
                        T *P, int *ctl, int *flags, int epoch, int *err, hipStream_t st)
{
    epoch = launch_dir<T, true>(L, ld, W, nbw, npad, m, Y, Z, ldy, P, ctl, flags, epoch, err, st);
    epoch = launch_dir<T, false>(L, ld, W, nbw, npad, m, Z, Y, ldy, P, ctl, flags, epoch, err, st);
    return epoch;
}
template int launch_trsv_persist<float>(const float *, int64_t, const float *, int, int64_t, int, float *, float *,
                                        int64_t, float *, int *, int *, int, int *, hipStream_t);
template int launch_trsv_persist<double>(const double *, int64_t, const double *, int, int64_t, int, double *,
                                         double *, int64_t, double *, int *, int *, int, int *, hipStream_t);

}  // namespace spd
