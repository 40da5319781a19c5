// Triangular solves with the low-precision factor (Eq. (3); Algorithm 1,
// lines 2 and 5) and the binary64 scaling/update around them (line 6).
//
// A correction is z = s mu D L^{-T} L^{-1} round(D r / s): the right-hand
// side is scaled by D and by a power of two s per column (so its largest
// entry is in [1/2, 1] before rounding), solved in the factor's precision,
// then mapped back and added to x in binary64.
//
// The substitutions are blocked by the panel width NB: with W_k = L_kk^{-1},
//   forward:  z_k = W_k y_k;      y_i -= L_ik z_k          (i > k)
//   backward: x_k = W_k^T z_k;    z_j -= L_kj^T x_k        (j < k)
// one launch for the diagonal product and one for the panel product per
// block.
#include "common.h"
#include "internal.h"

#define SOLVE_MC 8  // right-hand sides per workgroup

SPD_DEV double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

SPD_DEV double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v = nanmax(v, __shfl_xor(v, off));
    return v;
}

__global__ __launch_bounds__(256) void k_rhs_max(const double *__restrict__ R, int64_t ldr, int64_t n,
                                                 const double *__restrict__ d, double *smax)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    double v = (i < n) ? fabs(d[i] * R[i + c * ldr]) : 0.0;
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0)
        atomic_max_nonneg(smax + c, v);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rhs_scale(const double *__restrict__ R, int64_t ldr, int64_t n,
                                                   int64_t npad, const double *__restrict__ d,
                                                   const double *__restrict__ smax, T *__restrict__ Y, int64_t ldy)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= npad)
        return;
    const double s = pow2_ceil(smax[c]);
    Y[i + c * ldy] = (i < n) ? (T)(d[i] * R[i + c * ldr] / s) : (T)0;
}

// z_k = W_k y_k for rhs chunk blockIdx.x; thread r = row of the block.
template <typename T, int NB>
__global__ __launch_bounds__(NB) void k_fwd_diag(const T *__restrict__ Wk, const T *__restrict__ Y,
                                                 T *__restrict__ Z, int64_t ldy, int64_t k0, int m)
{
    __shared__ T ys[SOLVE_MC][NB];
    const int r = threadIdx.x, c0 = blockIdx.x * SOLVE_MC;
    const int mc = min(SOLVE_MC, m - c0);
    for (int c = 0; c < mc; ++c)
        ys[c][r] = Y[(k0 + r) + (c0 + c) * ldy];
    __syncthreads();
    T acc[SOLVE_MC];
#pragma unroll
    for (int c = 0; c < SOLVE_MC; ++c) acc[c] = (T)0;
    for (int t = 0; t <= r; ++t) {
        const T w = Wk[r + (size_t)t * NB];
#pragma unroll
        for (int c = 0; c < SOLVE_MC; ++c)
            acc[c] += w * ys[c][t];
    }
    for (int c = 0; c < mc; ++c)
        Z[(k0 + r) + (c0 + c) * ldy] = acc[c];
}

// Y[rows] -= L[rows, k0:k0+NB] z_k ; rows = row0 + 64 blockIdx.x + [0, 64)
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_fwd_panel(const T *__restrict__ L, int64_t ld, const T *__restrict__ Z,
                                                   T *__restrict__ Y, int64_t ldy, int64_t k0, int64_t row0, int m)
{
    __shared__ T zs[SOLVE_MC][NB];
    __shared__ T red[4][SOLVE_MC][64];
    const int tid = threadIdx.x, row = tid & 63, q = tid >> 6;
    const int c0 = blockIdx.y * SOLVE_MC;
    const int mc = min(SOLVE_MC, m - c0);
    for (int idx = tid; idx < NB * SOLVE_MC; idx += 256) {
        const int t = idx % NB, c = idx / NB;
        zs[c][t] = (c < mc) ? Z[(k0 + t) + (c0 + c) * ldy] : (T)0;
    }
    __syncthreads();
    const int64_t gr = row0 + (int64_t)blockIdx.x * 64 + row;
    T acc[SOLVE_MC];
#pragma unroll
    for (int c = 0; c < SOLVE_MC; ++c) acc[c] = (T)0;
    const T *lp = L + gr + (k0 + q * (NB / 4)) * ld;
#pragma unroll 4
    for (int t = 0; t < NB / 4; ++t) {
        const T l = lp[t * ld];
#pragma unroll
        for (int c = 0; c < SOLVE_MC; ++c)
            acc[c] += l * zs[c][q * (NB / 4) + t];
    }
#pragma unroll
    for (int c = 0; c < SOLVE_MC; ++c) red[q][c][row] = acc[c];
    __syncthreads();
    if (q == 0) {
        for (int c = 0; c < mc; ++c) {
            const T s = (red[0][c][row] + red[1][c][row]) + (red[2][c][row] + red[3][c][row]);
            Y[gr + (c0 + c) * ldy] -= s;
        }
    }
}

// x_k = W_k^T z_k (W staged through LDS 32 rows at a time for coalescing).
template <typename T, int NB>
__global__ __launch_bounds__(NB) void k_bwd_diag(const T *__restrict__ Wk, const T *__restrict__ Z,
                                                 T *__restrict__ Y, int64_t ldy, int64_t k0, int m)
{
    __shared__ T zs[SOLVE_MC][NB];
    __shared__ T ws[NB * 33];
    const int r = threadIdx.x, c0 = blockIdx.x * SOLVE_MC;
    const int mc = min(SOLVE_MC, m - c0);
    for (int c = 0; c < SOLVE_MC; ++c)
        zs[c][r] = (c < mc) ? Z[(k0 + r) + (c0 + c) * ldy] : (T)0;
    T acc[SOLVE_MC];
#pragma unroll
    for (int c = 0; c < SOLVE_MC; ++c) acc[c] = (T)0;
    for (int t0 = 0; t0 < NB; t0 += 32) {
        __syncthreads();
        // ws[col * 33 + tt] = W[t0 + tt][col]
        for (int idx = r; idx < 32 * NB; idx += NB) {
            const int tt = idx & 31, col = idx >> 5;
            ws[col * 33 + tt] = Wk[(t0 + tt) + (size_t)col * NB];
        }
        __syncthreads();
#pragma unroll 4
        for (int tt = 0; tt < 32; ++tt) {
            const T w = ws[r * 33 + tt];  // W[t0+tt][r], zero above the diagonal
#pragma unroll
            for (int c = 0; c < SOLVE_MC; ++c)
                acc[c] += w * zs[c][t0 + tt];
        }
    }
    for (int c = 0; c < mc; ++c)
        Y[(k0 + r) + (c0 + c) * ldy] = acc[c];
}

// Z[cols] -= L[k0:k0+NB, cols]^T x_k for output rows cols = 64 blockIdx.x + [0, 64) < k0
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_bwd_panel(const T *__restrict__ L, int64_t ld, const T *__restrict__ Y,
                                                   T *__restrict__ Z, int64_t ldy, int64_t k0, int m)
{
    __shared__ T xs[SOLVE_MC][NB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = blockIdx.y * SOLVE_MC;
    const int mc = min(SOLVE_MC, m - c0);
    for (int idx = tid; idx < NB * SOLVE_MC; idx += 256) {
        const int t = idx % NB, c = idx / NB;
        xs[c][t] = (c < mc) ? Y[(k0 + t) + (c0 + c) * ldy] : (T)0;
    }
    __syncthreads();
    for (int o = 0; o < 16; ++o) {
        const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + o;
        if (col >= k0)
            break;
        T acc[SOLVE_MC];
#pragma unroll
        for (int c = 0; c < SOLVE_MC; ++c) acc[c] = (T)0;
        const T *lp = L + k0 + col * ld;
#pragma unroll
        for (int i = 0; i < NB / 64; ++i) {
            const int r = lane + 64 * i;
            const T l = lp[r];
#pragma unroll
            for (int c = 0; c < SOLVE_MC; ++c)
                acc[c] += l * xs[c][r];
        }
#pragma unroll
        for (int c = 0; c < SOLVE_MC; ++c) {
            T v = acc[c];
            for (int off = 32; off > 0; off >>= 1)
                v += __shfl_xor(v, off);
            acc[c] = v;
        }
        if (lane == 0)
            for (int c = 0; c < mc; ++c)
                Z[col + (c0 + c) * ldy] -= acc[c];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_update_x(double *__restrict__ X, int64_t ldx, int64_t n,
                                                  const T *__restrict__ Y, int64_t ldy, const double *__restrict__ d,
                                                  double mu, const double *__restrict__ smax, int accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n)
        return;
    const double s = pow2_ceil(smax[c]);
    const double z = ((s * mu) * d[i]) * (double)Y[i + c * ldy];
    double *px = X + i + c * ldx;
    *px = accumulate ? *px + z : z;
}

__global__ void k_zero(double *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count)
        p[i] = 0.0;
}

namespace spd {

void launch_rhs_max(const double *R, int64_t ldr, int64_t n, int m, const double *d, double *smax, hipStream_t st)
{
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(k_rhs_max, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, st, R, ldr, n, d,
                       smax);
}

template <typename T>
void launch_rhs_scale(const double *R, int64_t ldr, int64_t n, int64_t npad, int m, const double *d,
                      const double *smax, T *Y, int64_t ldy, hipStream_t st)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_rhs_scale<T>, dim3((unsigned)((npad + 255) / 256), (unsigned)m), dim3(256), 0, st, R, ldr,
                       n, npad, d, smax, Y, ldy);
}
template void launch_rhs_scale<float>(const double *, int64_t, int64_t, int64_t, int, const double *,
                                      const double *, float *, int64_t, hipStream_t);
template void launch_rhs_scale<double>(const double *, int64_t, int64_t, int64_t, int, const double *,
                                       const double *, double *, int64_t, hipStream_t);

template <typename T>
void launch_trsv_fwd(const T *L, int64_t ld, const T *W, int64_t npad, int m, T *Y, T *Z, int64_t ldy,
                     hipStream_t st)
{
    const int64_t nt = npad / SPD_NB;
    const unsigned mch = (unsigned)((m + SOLVE_MC - 1) / SOLVE_MC);
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t k0 = k * SPD_NB;
        hipLaunchKernelGGL((k_fwd_diag<T, SPD_NB>), dim3(mch), dim3(SPD_NB), 0, st, W + (size_t)k * SPD_NB * SPD_NB,
                           Y, Z, ldy, k0, m);
        const int64_t row0 = k0 + SPD_NB, rows = npad - row0;
        if (rows > 0)
            hipLaunchKernelGGL((k_fwd_panel<T, SPD_NB>), dim3((unsigned)(rows / 64), mch), dim3(256), 0, st, L, ld,
                               Z, Y, ldy, k0, row0, m);
    }
}
template void launch_trsv_fwd<float>(const float *, int64_t, const float *, int64_t, int, float *, float *, int64_t,
                                     hipStream_t);
template void launch_trsv_fwd<double>(const double *, int64_t, const double *, int64_t, int, double *, double *,
                                      int64_t, hipStream_t);

template <typename T>
void launch_trsv_bwd(const T *L, int64_t ld, const T *W, int64_t npad, int m, T *Z, T *Y, int64_t ldy,
                     hipStream_t st)
{
    const int64_t nt = npad / SPD_NB;
    const unsigned mch = (unsigned)((m + SOLVE_MC - 1) / SOLVE_MC);
    for (int64_t k = nt - 1; k >= 0; --k) {
        const int64_t k0 = k * SPD_NB;
        hipLaunchKernelGGL((k_bwd_diag<T, SPD_NB>), dim3(mch), dim3(SPD_NB), 0, st, W + (size_t)k * SPD_NB * SPD_NB,
                           Z, Y, ldy, k0, m);
        if (k0 > 0)
            hipLaunchKernelGGL((k_bwd_panel<T, SPD_NB>), dim3((unsigned)((k0 + 63) / 64), mch), dim3(256), 0, st,
                               L, ld, Y, Z, ldy, k0, m);
    }
}
template void launch_trsv_bwd<float>(const float *, int64_t, const float *, int64_t, int, float *, float *, int64_t,
                                     hipStream_t);
template void launch_trsv_bwd<double>(const double *, int64_t, const double *, int64_t, int, double *, double *,
                                      int64_t, hipStream_t);

template <typename T>
void launch_update_x(double *X, int64_t ldx, int64_t n, int m, const T *Y, int64_t ldy, const double *d, double mu,
                     const double *smax, int accumulate, hipStream_t st)
{
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(k_update_x<T>, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, st, X, ldx, n, Y,
                       ldy, d, mu, smax, accumulate);
}
template void launch_update_x<float>(double *, int64_t, int64_t, int, const float *, int64_t, const double *, double,
                                     const double *, int, hipStream_t);
template void launch_update_x<double>(double *, int64_t, int64_t, int, const double *, int64_t, const double *,
                                      double, const double *, int, hipStream_t);

void launch_zero(double *p, int64_t count, hipStream_t st)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count);
}

}  // namespace spd
