// Triangular solves with the low-precision factor (Eq. (3); Algorithm 1's
// first solve and correction solves) and the binary64 scaling and update of
// x around them.
//
// A correction is z = s mu D L^{-T} L^{-1} round(D r / s): the right-hand
// side is scaled by D and by a power of two s per column (so its largest
// entry is in [1/2, 1] before rounding), solved in the factor's precision,
// then mapped back and added to x in binary64.
//
// The substitutions themselves are in k_trsv.hip.
#include "common.h"
#include "internal.h"

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
                                                   const double *__restrict__ smax, T *__restrict__ Y, int64_t ldy,
                                                   double *__restrict__ zd, int64_t nzd, int *__restrict__ zi,
                                                   int64_t nzi)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (c == 0) {
        // clears what the kernels after this one start from (the next
        // residual's norms, the triangular solves' counters); no other
        // kernel of the launch reads them
        const int64_t stride = (int64_t)gridDim.x * 256;
        for (int64_t j = i; j < nzd; j += stride)
            zd[j] = 0.0;
        for (int64_t j = i; j < nzi; j += stride)
            zi[j] = 0;
    }
    if (i >= npad)
        return;
    const double s = pow2_ceil(smax[c]);
    Y[i + c * ldy] = (i < n) ? (T)(d[i] * R[i + c * ldr] / s) : (T)0;
}

// x += z (or x = z) with z = s mu d_i Y_i; with zmax, also max_i |z_i| per
// column (the correction's size, read by the stopping rule)
template <typename T>
__global__ __launch_bounds__(256) void k_update_x(double *__restrict__ X, int64_t ldx, int64_t n,
                                                  const T *__restrict__ Y, int64_t ldy, const double *__restrict__ d,
                                                  double mu, const double *__restrict__ smax, int accumulate,
                                                  double *zmax)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    double z = 0.0;
    if (i < n) {
        const double s = pow2_ceil(smax[c]);
        z = ((s * mu) * d[i]) * (double)Y[i + c * ldy];
        double *px = X + i + c * ldx;
        *px = accumulate ? *px + z : z;
    }
    if (zmax) {
        const double v = wave_max(fabs(z));
        if ((threadIdx.x & 63) == 0)
            atomic_max_nonneg(zmax + c, v);
    }
}

// out[c] raised to max_i |X[i][c] - S[i][c]| (a correction taken as the
// change of x); then S = X
__global__ __launch_bounds__(256) void k_col_maxdiff(const double *__restrict__ X, int64_t ldx, double *__restrict__ S,
                                                     int64_t lds, int64_t n, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    double v = 0.0;
    if (i < n) {
        const double x = X[i + c * ldx];
        v = fabs(x - S[i + c * lds]);
        S[i + c * lds] = x;
    }
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0)
        atomic_max_nonneg(out + c, v);
}

// tuning input: a_ii = 2, a_ij = a_ji = h(min, max) / n with h a 32-bit
// integer hash mapped to (-1, 1): symmetric and diagonally dominant (SPD)
// (columns j = blockIdx.y, blockIdx.y + gridDim.y, ...)
__global__ __launch_bounds__(256) void k_tune_matrix(double *A, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        double v = 2.0;
        if (i != j) {
            uint32_t h = (uint32_t)(i < j ? i : j) * 0x9E3779B1u ^ (uint32_t)(i < j ? j : i) * 0x85EBCA77u;
            h ^= h >> 15;
            h *= 0x2C1B3C6Du;
            h ^= h >> 12;
            v = ((double)h / 4294967296.0 * 2.0 - 1.0) / (double)n;
        }
        A[i + j * n] = v;
    }
}

__global__ void k_zero(double *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count)
        p[i] = 0.0;
}

// the refinement's per-iteration read-back: the norms, the triangular
// solves' timeout flag and, when asked, the factorisation's info word, copied
// by one workgroup into host-visible memory
__global__ __launch_bounds__(256) void k_publish(const double *__restrict__ src, int64_t count,
                                                 const int *__restrict__ flag, const unsigned long long *__restrict__ info,
                                                 double *__restrict__ dst, int *__restrict__ dflag,
                                                 unsigned long long *__restrict__ dinfo)
{
    for (int64_t i = threadIdx.x; i < count; i += 256)
        dst[i] = src[i];
    if (threadIdx.x == 0) {
        *dflag = *flag;
        if (dinfo)
            *dinfo = *info;
    }
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
                      const double *smax, T *Y, int64_t ldy, double *zd, int64_t nzd, int *zi, int64_t nzi,
                      hipStream_t st)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_rhs_scale<T>, dim3((unsigned)((npad + 255) / 256), (unsigned)m), dim3(256), 0, st, R, ldr,
                       n, npad, d, smax, Y, ldy, zd, zd ? nzd : 0, zi, zi ? nzi : 0);
}
template void launch_rhs_scale<float>(const double *, int64_t, int64_t, int64_t, int, const double *,
                                      const double *, float *, int64_t, double *, int64_t, int *, int64_t,
                                      hipStream_t);
template void launch_rhs_scale<double>(const double *, int64_t, int64_t, int64_t, int, const double *,
                                       const double *, double *, int64_t, double *, int64_t, int *, int64_t,
                                       hipStream_t);

template <typename T>
void launch_update_x(double *X, int64_t ldx, int64_t n, int m, const T *Y, int64_t ldy, const double *d, double mu,
                     const double *smax, int accumulate, double *zmax, hipStream_t st)
{
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(k_update_x<T>, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, st, X, ldx, n, Y,
                       ldy, d, mu, smax, accumulate, zmax);
}
template void launch_update_x<float>(double *, int64_t, int64_t, int, const float *, int64_t, const double *, double,
                                     const double *, int, double *, hipStream_t);
template void launch_update_x<double>(double *, int64_t, int64_t, int, const double *, int64_t, const double *,
                                      double, const double *, int, double *, hipStream_t);

void launch_col_maxdiff(const double *X, int64_t ldx, double *S, int64_t lds, int64_t n, int m, double *out,
                        hipStream_t st)
{
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(k_col_maxdiff, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, st, X, ldx, S,
                       lds, n, out);
}

void launch_tune_matrix(double *A, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tune_matrix, dim3((unsigned)((n + 255) / 256), (unsigned)std::min<int64_t>(n, 4096)),
                       dim3(256), 0, st, A, n);
}

void launch_publish(const double *src, int64_t count, const int *flag, const unsigned long long *info, double *dst,
                    int *dflag, unsigned long long *dinfo, hipStream_t st)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, st, src, count, flag, info, dst, dflag, dinfo);
}

void launch_zero(double *p, int64_t count, hipStream_t st)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count);
}

}  // namespace spd
