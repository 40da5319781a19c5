// Conjugate gradients with iterative refinement (Algorithm 2, Section 3.2):
// the binary32 operator A~ (dense, or the band |i - j| <= k of Section 4),
// its product with the search directions, and the binary64 vector steps.
//
// Storage.  Dense A~: binary32, ldt x ldt column-major (ldt = n rounded up to
// 256, zero outside n x n), both triangles written so that column i is row i
// and every product reads whole columns contiguously.  Band A~:
// Bd[(d + k) ldt + i] = A~(i, i + d) for d = -k..k (zero where i + d falls
// outside 0..n-1, and in rows n..ldt-1).  Search directions: P (binary64,
// n x m, ld n) and its binary32 rounding Pf (ldt x m, zero rows n..ldt-1).
//
// Reductions are deterministic: every kernel that needs a dot product
// writes one partial per workgroup, and k_cg_scalars sums them for each
// column in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace {

constexpr int CG_MAXK_BAND = 4096;  // largest half-bandwidth kept in band storage

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_sumf(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// fixed-order sum of one value per thread over a 256-thread block
__device__ inline double block_sum256(double v, double *red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// dense A~ = fl32(A), both triangles, zero padding to ldt x ldt
__global__ __launch_bounds__(256) void k_cg_dense(const double *__restrict__ A, int64_t lda, int64_t n,
                                                  float *__restrict__ At, int64_t ldt)
{
    __shared__ double tile[64][65];
    const int64_t I = (int64_t)blockIdx.x * 64, J = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t i = I + tx;
    if (I > J) {  // strictly below the diagonal: a straight copy
        for (int r = ty; r < 64; r += 4) {
            const int64_t j = J + r;
            At[i + j * ldt] = (i < n && j < n) ? (float)A[i + j * lda] : 0.0f;
        }
        return;
    }
    // diagonal or above: element (i, j) with i < j is A(j, i), read through
    // the tile A[J.., I..] (lower triangle, coalesced along J)
    for (int r = ty; r < 64; r += 4) {
        const int64_t ii = I + r, jj = J + tx;
        tile[r][tx] = (jj < n && ii < n && jj >= ii) ? A[jj + ii * lda] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = J + r;
        float v = 0.0f;
        if (i < n && j < n) v = (float)((i >= j) ? A[i + j * lda] : tile[tx][r]);
        At[i + j * ldt] = v;
    }
}

// band A~: Bd[(d + k) ldt + i] = fl32(A(i, i + d)), zero outside the matrix
__global__ __launch_bounds__(256) void k_cg_band(const double *__restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                 float *__restrict__ Bd, int64_t ldt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t d = (int64_t)blockIdx.y - k;
    if (i >= ldt) return;
    const int64_t j = i + d;
    float v = 0.0f;
    if (i < n && j >= 0 && j < n) v = (float)((i >= j) ? A[i + j * lda] : A[j + i * lda]);
    Bd[(d + k) * ldt + i] = v;
}

// any column of the block [c0, c0 + cnt) still active?
__device__ inline bool any_active(const int *act, int c0, int cnt)
{
    bool a = false;
    for (int c = 0; c < cnt; ++c) a |= act[c0 + c] != 0;
    return a;
}

// z = A~ p for up to 4 right-hand sides on the VALU: one wave per 4
// columns of A~ (= rows of z), lanes along the column (float4 each), then a
// wave reduction.  One binary64 partial of p^T z per workgroup and column.
template <int MB>
__global__ __launch_bounds__(256) void k_cg_mv_valu(const float *__restrict__ At, int64_t ldt, int64_t n,
                                                    const float *__restrict__ Pf, const double *__restrict__ P,
                                                    double *__restrict__ Z, double *__restrict__ part, int64_t npart,
                                                    const int *__restrict__ act)
{
    __shared__ double red[4][MB];
    if (!any_active(act, 0, MB)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * 16 + w * 4;
    float acc[4][MB];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[c][b] = 0.0f;
    const float4 *a4[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a4[c] = reinterpret_cast<const float4 *>(At + (i0 + c) * ldt);
    const int64_t nt = ldt / 256;
#pragma unroll 2
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t q = t * 64 + lane;
        float4 p4[MB];
#pragma unroll
        for (int b = 0; b < MB; ++b) p4[b] = reinterpret_cast<const float4 *>(Pf + b * ldt)[q];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float4 a = a4[c][q];
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                acc[c][b] += a.x * p4[b].x;
                acc[c][b] += a.y * p4[b].y;
                acc[c][b] += a.z * p4[b].z;
                acc[c][b] += a.w * p4[b].w;
            }
        }
    }
    double pz[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) pz[b] = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t i = i0 + c;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            const double z = (double)wave_sumf(acc[c][b]);
            if (i < n) {
                if (lane == 0) Z[i + b * n] = z;
                pz[b] += P[i + b * n] * z;
            }
        }
    }
    if (lane == 0)
#pragma unroll
        for (int b = 0; b < MB; ++b) red[w][b] = pz[b];
    __syncthreads();
    if (threadIdx.x < MB) {
        const int b = threadIdx.x;
        part[blockIdx.x + b * npart] = ((red[0][b] + red[1][b]) + red[2][b]) + red[3][b];
    }
}

// z = A~ p for 5..32 right-hand sides per launch row (blockIdx.y picks the
// block of 32) on v_mfma_f32_32x32x2f32: a workgroup owns 32 rows of z, its
// four waves split the columns' length, and each lane streams one column of
// A~ (the MFMA's A operand, lanes 0-31 taking k-slot 0, lanes 32-63 k-slot 1)
// against the matching rows of Pf (the B operand); the k order is the same
// permutation on both operands.
__global__ __launch_bounds__(256) void k_cg_mv_mfma(const float *__restrict__ At, int64_t ldt, int64_t n, int m,
                                                    const float *__restrict__ Pf, const double *__restrict__ P,
                                                    double *__restrict__ Z, double *__restrict__ part, int64_t npart,
                                                    const int *__restrict__ act)
{
    __shared__ float red[3][16][64];
    const int c0 = blockIdx.y * 32;
    const int mc = min(32, m - c0);
    if (!any_active(act, c0, mc)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t i0 = (int64_t)blockIdx.x * 32;
    const int64_t kq = ldt / 4;  // each wave: rows [w kq, (w + 1) kq) of the columns
    const float *acol = At + (i0 + l32) * ldt + w * kq + 8 * h;
    const bool bvalid = l32 < mc;
    const float *bcol = Pf + (int64_t)(c0 + (bvalid ? l32 : 0)) * ldt + w * kq + 8 * h;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll 2
    for (int64_t j = 0; j < kq; j += 16) {
        const float4 a0 = *reinterpret_cast<const float4 *>(acol + j);
        const float4 a1 = *reinterpret_cast<const float4 *>(acol + j + 4);
        float4 b0 = *reinterpret_cast<const float4 *>(bcol + j);
        float4 b1 = *reinterpret_cast<const float4 *>(bcol + j + 4);
        if (!bvalid) b0 = b1 = make_float4(0.f, 0.f, 0.f, 0.f);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, b0.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, b0.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.z, b0.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.w, b0.w, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.x, b1.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.y, b1.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.z, b1.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.w, b1.w, acc, 0, 0, 0);
    }
    if (w > 0)
#pragma unroll
        for (int r = 0; r < 16; ++r) red[w - 1][r][lane] = acc[r];
    __syncthreads();
    if (w != 0) return;
    // register r of lane l: row 8(r/4) + 4(l/32) + r%4 of the tile, column l%32
    const int c = c0 + l32;
    double pz = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float s = ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
        const int64_t i = i0 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (bvalid && i < n) {
            const double z = (double)s;
            Z[i + (int64_t)c * n] = z;
            pz += P[i + (int64_t)c * n] * z;
        }
    }
    pz += __shfl_xor(pz, 32, 64);
    if (h == 0 && bvalid) part[blockIdx.x + (int64_t)c * npart] = pz;
}

// z = A~ p on the band: a thread per row, the rows' slice of Pf (with its
// k-wide halo) staged in LDS per right-hand side
__global__ __launch_bounds__(256) void k_cg_mv_band(const float *__restrict__ Bd, int64_t ldt, int64_t n, int64_t k,
                                                    int m, const float *__restrict__ Pf,
                                                    const double *__restrict__ P, double *__restrict__ Z,
                                                    double *__restrict__ part, int64_t npart,
                                                    const int *__restrict__ act)
{
    extern __shared__ float pl[];  // 256 + 2k
    __shared__ double red[4];
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    const int64_t i = i0 + threadIdx.x;
    const int64_t span = 256 + 2 * k;
    for (int b = 0; b < m; ++b) {
        if (!act[b]) continue;  // uniform across the block
        __syncthreads();
        for (int64_t s = threadIdx.x; s < span; s += 256) {
            const int64_t j = i0 - k + s;
            pl[s] = (j >= 0 && j < n) ? Pf[j + (int64_t)b * ldt] : 0.0f;
        }
        __syncthreads();
        float acc = 0.0f;
        if (i < n)
            for (int64_t d = -k; d <= k; ++d) acc += Bd[(d + k) * ldt + i] * pl[threadIdx.x + k + d];
        double pz = 0.0;
        if (i < n) {
            const double z = (double)acc;
            Z[i + (int64_t)b * n] = z;
            pz = P[i + (int64_t)b * n] * z;
        }
        pz = block_sum256(pz, red);
        if (threadIdx.x == 0) part[blockIdx.x + (int64_t)b * npart] = pz;
    }
}

// P = R, Pf = fl32(R) and a partial of r^T r, for the columns starting a phase
__global__ __launch_bounds__(256) void k_cg_start(int64_t n, int m, const double *__restrict__ R,
                                                  double *__restrict__ P, float *__restrict__ Pf, int64_t ldt,
                                                  double *__restrict__ part, int64_t npart, const int *__restrict__ go)
{
    __shared__ double red[4];
    for (int b = 0; b < m; ++b) {
        if (!go[b]) continue;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = (int64_t)blockIdx.x * 1024 + u * 256 + threadIdx.x;
            if (i < n) {
                const double r = R[i + (int64_t)b * n];
                P[i + (int64_t)b * n] = r;
                Pf[i + (int64_t)b * ldt] = (float)r;
                s += r * r;
            }
        }
        s = block_sum256(s, red);
        if (threadIdx.x == 0) part[blockIdx.x + (int64_t)b * npart] = s;
    }
}

// x += alpha p, r -= alpha z and a partial of the new r^T r (active columns)
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int m, const double *__restrict__ alpha,
                                               const double *__restrict__ P, const double *__restrict__ Z,
                                               double *__restrict__ X, int64_t ldx, double *__restrict__ R,
                                               double *__restrict__ part, int64_t npart, const int *__restrict__ act)
{
    __shared__ double red[4];
    for (int b = 0; b < m; ++b) {
        if (!act[b]) continue;
        const double al = alpha[b];
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = (int64_t)blockIdx.x * 1024 + u * 256 + threadIdx.x;
            if (i < n) {
                X[i + (int64_t)b * ldx] += al * P[i + (int64_t)b * n];
                const double r = R[i + (int64_t)b * n] - al * Z[i + (int64_t)b * n];
                R[i + (int64_t)b * n] = r;
                s += r * r;
            }
        }
        s = block_sum256(s, red);
        if (threadIdx.x == 0) part[blockIdx.x + (int64_t)b * npart] = s;
    }
}

// p = r + beta p, Pf = fl32(p) (columns still active)
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, int m, const double *__restrict__ beta,
                                              const double *__restrict__ R, double *__restrict__ P,
                                              float *__restrict__ Pf, int64_t ldt, const int *__restrict__ act)
{
    for (int b = 0; b < m; ++b) {
        if (!act[b]) continue;
        const double be = beta[b];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = (int64_t)blockIdx.x * 1024 + u * 256 + threadIdx.x;
            if (i < n) {
                const double p = R[i + (int64_t)b * n] + be * P[i + (int64_t)b * n];
                P[i + (int64_t)b * n] = p;
                Pf[i + (int64_t)b * ldt] = (float)p;
            }
        }
    }
}

// Per-column scalars from the partials (one block per column):
//   CG_START: rho = r^T r, thr = inner_tol^2 rho, cnt = 0,
//             act = go && max_inner > 0 && rho > thr
//   CG_ALPHA: alpha = rho / p^T z                      (active columns)
//   CG_BETA:  rho' = r^T r, beta = rho' / rho, rho = rho', ++cnt,
//             act = cnt < max_inner && rho' > thr      (active columns)
__global__ __launch_bounds__(256) void k_cg_scalars(int mode, const double *__restrict__ part, int64_t npart,
                                                    double *__restrict__ sc, int *__restrict__ act,
                                                    const int *__restrict__ go, int *__restrict__ cnt,
                                                    double inner_tol2, int max_inner, int m)
{
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (mode != spd::CG_START && !act[b]) return;
    if (mode == spd::CG_START && !go[b]) {
        if (threadIdx.x == 0) act[b] = 0;
        return;
    }
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < npart; q += 256) s += part[q + (int64_t)b * npart];
    s = block_sum256(s, red);
    if (threadIdx.x != 0) return;
    double *rho = sc, *thr = sc + m, *alpha = sc + 2 * m, *beta = sc + 3 * m;
    if (mode == spd::CG_START) {
        rho[b] = s;
        thr[b] = inner_tol2 * s;
        cnt[b] = 0;
        act[b] = (max_inner > 0 && s > thr[b]) ? 1 : 0;
    } else if (mode == spd::CG_ALPHA) {
        alpha[b] = rho[b] / s;
    } else {
        beta[b] = s / rho[b];
        rho[b] = s;
        cnt[b] += 1;
        act[b] = (cnt[b] < max_inner && s > thr[b]) ? 1 : 0;
    }
}

}  // namespace

namespace spd {

int64_t cg_ldt(int64_t n) { return ((std::max<int64_t>(n, 1) + 255) / 256) * 256; }
int cg_band_ok(int64_t k) { return k >= 0 && k <= CG_MAXK_BAND; }

void launch_cg_dense(const double *A, int64_t lda, int64_t n, float *At, int64_t ldt, hipStream_t st)
{
    dim3 g((unsigned)(ldt / 64), (unsigned)(ldt / 64));
    hipLaunchKernelGGL(k_cg_dense, g, dim3(256), 0, st, A, lda, n, At, ldt);
}

void launch_cg_band(const double *A, int64_t lda, int64_t n, int64_t k, float *Bd, int64_t ldt, hipStream_t st)
{
    dim3 g((unsigned)(ldt / 256), (unsigned)(2 * k + 1));
    hipLaunchKernelGGL(k_cg_band, g, dim3(256), 0, st, A, lda, n, k, Bd, ldt);
}

int64_t cg_mv_parts(int64_t n, int64_t ldt, int64_t k, int m)
{
    if (k >= 0) return (n + 255) / 256;
    return (m <= 4) ? ldt / 16 : ldt / 32;
}

void launch_cg_mv(const float *At, int64_t ldt, int64_t n, int64_t k, int m, const float *Pf, const double *P,
                  double *Z, double *part, int64_t npart, const int *act, hipStream_t st)
{
    if (k >= 0) {
        const size_t lds = (size_t)(256 + 2 * k) * sizeof(float);
        hipLaunchKernelGGL(k_cg_mv_band, dim3((unsigned)((n + 255) / 256)), dim3(256), lds, st, At, ldt, n, k, m,
                           Pf, P, Z, part, npart, act);
        return;
    }
    const dim3 blk(256);
    switch (m) {
    case 1: hipLaunchKernelGGL(k_cg_mv_valu<1>, dim3((unsigned)(ldt / 16)), blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    case 2: hipLaunchKernelGGL(k_cg_mv_valu<2>, dim3((unsigned)(ldt / 16)), blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    case 3: hipLaunchKernelGGL(k_cg_mv_valu<3>, dim3((unsigned)(ldt / 16)), blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    case 4: hipLaunchKernelGGL(k_cg_mv_valu<4>, dim3((unsigned)(ldt / 16)), blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    default:
        hipLaunchKernelGGL(k_cg_mv_mfma, dim3((unsigned)(ldt / 32), (unsigned)((m + 31) / 32)), blk, 0, st, At, ldt,
                           n, m, Pf, P, Z, part, npart, act);
    }
}

int64_t cg_vec_parts(int64_t n) { return std::max<int64_t>((n + 1023) / 1024, 1); }

void launch_cg_start(int64_t n, int m, const double *R, double *P, float *Pf, int64_t ldt, double *part,
                     int64_t npart, const int *go, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_start, dim3((unsigned)npart), dim3(256), 0, st, n, m, R, P, Pf, ldt, part, npart, go);
}

void launch_cg_xr(int64_t n, int m, const double *alpha, const double *P, const double *Z, double *X, int64_t ldx,
                  double *R, double *part, int64_t npart, const int *act, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_xr, dim3((unsigned)npart), dim3(256), 0, st, n, m, alpha, P, Z, X, ldx, R, part, npart,
                       act);
}

void launch_cg_p(int64_t n, int m, const double *beta, const double *R, double *P, float *Pf, int64_t ldt,
                 const int *act, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_p, dim3((unsigned)cg_vec_parts(n)), dim3(256), 0, st, n, m, beta, R, P, Pf, ldt, act);
}

void launch_cg_scalars(int mode, const double *part, int64_t npart, double *sc, int *act, const int *go, int *cnt,
                       double inner_tol2, int max_inner, int m, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_scalars, dim3((unsigned)m), dim3(256), 0, st, mode, part, npart, sc, act, go, cnt,
                       inner_tol2, max_inner, m);
}

}  // namespace spd
