// Conjugate gradients with iterative refinement (Algorithm 2, Section 3.2):
// the binary32 operator A~ (dense, or the band |i - j| <= k of Section 4),
// its product with the search directions, and the binary64 vector steps.
//
// Storage.  Dense A~: binary32, ldt x ldt (ldt = n rounded up to 256, zero
// outside n x n), both triangles, in the MFMA fragment order of frag_off so
// that each product streams it with fully coalesced loads.  Band A~:
// Bd[(d + k) ldt + i] = A~(i, i + d) for d = -k..k (zero where i + d falls
// outside 0..n-1, and in rows n..ldt-1).  Search directions: P (binary64,
// n x m, ld n) and its binary32 rounding Pf (layout of pf_off, zero in rows
// n..ldt-1 and in the padding columns of the last block).
//
// Reductions are deterministic: every kernel that needs a dot product
// writes one partial per workgroup, and its consumers sum them for each
// column in a fixed order (every workgroup of a consumer the same way).
// One CG iteration is three launches (four for the dense 5..32-column
// product, which adds its slice sum): product, x/r update, p update.
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

// Offset of A~(j, i) in the dense fragment order: column block I = i / 32,
// row block J = j / 16 (512 values, contiguous, blocks of one column block
// consecutive along J); inside a block, value e of the float4 number s of
// lane l, with l = 32 h + i % 32 and j % 16 = 8 h + 4 s + e.  A wave's float4
// load of one (s) half of a block is then 1 KB contiguous, and lane l holds
// exactly the MFMA operand values of row i % 32 at k-slot h.
__device__ inline int64_t frag_off(int64_t j, int64_t i, int64_t nJ)
{
    const int64_t jj = j & 15;
    const int h = (int)(jj >> 3), s = (int)((jj >> 2) & 1), e = (int)(jj & 3);
    return ((i >> 5) * nJ + (j >> 4)) * 512 + s * 256 + (h * 32 + (int)(i & 31)) * 4 + e;
}

// Offset of the binary32 direction value (j, c): right-hand sides in blocks
// of W columns (W = m for m <= 4, else 32), each block ldt x W stored with
// the column index inside groups of four consecutive rows:
// ((j / 4) W + c % W) 4 + j % 4.  A lane's four consecutive rows of one
// column are one float4.
__device__ inline int64_t pf_off(int64_t j, int c, int W, int64_t ldt)
{
    return (int64_t)(c / W) * ldt * W + ((j >> 2) * W + (c % W)) * 4 + (j & 3);
}

// dense A~ = fl32(A) in fragment order, zero outside n x n; one 64 x 64
// tile of the symmetric A per workgroup, read along A's columns
__global__ __launch_bounds__(256) void k_cg_dense(const double *__restrict__ A, int64_t lda, int64_t n,
                                                  float *__restrict__ Af, int64_t ldt)
{
    __shared__ float tile[64][65];  // tile[jl][il] = A~(J0 + jl, I0 + il)
    const int64_t I0 = (int64_t)blockIdx.x * 64, J0 = (int64_t)blockIdx.y * 64;
    const int t = threadIdx.x;
    if (J0 >= I0 + 64) {  // every jj > ii: A[jj + ii lda], contiguous along jj
        for (int r = 0; r < 16; ++r) {
            const int il = (t >> 6) + 4 * r, jl = t & 63;
            const int64_t ii = I0 + il, jj = J0 + jl;
            tile[jl][il] = (ii < n && jj < n) ? (float)A[jj + ii * lda] : 0.0f;
        }
    } else if (I0 >= J0 + 64) {  // every ii > jj: A[ii + jj lda], contiguous along ii
        for (int r = 0; r < 16; ++r) {
            const int jl = (t >> 6) + 4 * r, il = t & 63;
            const int64_t ii = I0 + il, jj = J0 + jl;
            tile[jl][il] = (ii < n && jj < n) ? (float)A[ii + jj * lda] : 0.0f;
        }
    } else {  // diagonal tile
        for (int r = 0; r < 16; ++r) {
            const int il = (t >> 6) + 4 * r, jl = t & 63;
            const int64_t ii = I0 + il, jj = J0 + jl;
            float v = 0.0f;
            if (ii < n && jj < n) v = (float)((jj >= ii) ? A[jj + ii * lda] : A[ii + jj * lda]);
            tile[jl][il] = v;
        }
    }
    __syncthreads();
    // the tile is 2 column blocks x 4 row blocks of 512 values
    const int64_t nJ = ldt / 16;
    for (int r = 0; r < 16; ++r) {
        const int f = t + 256 * r;          // 0..4095
        const int blk = f >> 9, w = f & 511;
        const int bi = blk >> 2, bj = blk & 3;
        const int s = w >> 8, lane = (w >> 2) & 63, e = w & 3;
        const int il = bi * 32 + (lane & 31), jl = bj * 16 + (lane >> 5) * 8 + s * 4 + e;
        const int64_t I = (I0 >> 5) + bi, J = (J0 >> 4) + bj;
        Af[(I * nJ + J) * 512 + w] = tile[jl][il];
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

// z = A~ p for up to 4 right-hand sides on the VALU.  A workgroup owns the
// 32 rows of z of one column block; its four waves split the block's row
// blocks, every lane accumulates row i % 32 over its k-slot's rows, with the
// direction values loaded as broadcast float4s.  The halves and the waves
// are summed in a fixed order; one binary64 partial of p^T z per column.
template <int MB>
__global__ __launch_bounds__(256) void k_cg_mv_valu(const float *__restrict__ Af, int64_t ldt, int64_t n,
                                                    const float *__restrict__ Pf, const double *__restrict__ P,
                                                    double *__restrict__ Z, double *__restrict__ part, int64_t npart,
                                                    const int *__restrict__ act)
{
    __shared__ float red[3][MB][64];
    if (!any_active(act, 0, MB)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t nJ = ldt / 16, jq = nJ / 4;
    const int64_t I = blockIdx.x;
    const float *ab = Af + (I * nJ + w * jq) * 512 + lane * 4;
    // rows J 16 + 8 h + 0..3 and + 4..7 of right-hand side b: float4 number
    // (4 J + 2 h) W + b and the next group
    const float4 *pb = reinterpret_cast<const float4 *>(Pf) + (w * jq * 4 + 2 * h) * MB;
    float acc[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) acc[b] = 0.0f;
#pragma unroll 4
    for (int64_t J = 0; J < jq; ++J) {
        const float4 a0 = *reinterpret_cast<const float4 *>(ab + J * 512);
        const float4 a1 = *reinterpret_cast<const float4 *>(ab + J * 512 + 256);
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            const float4 p0 = pb[J * 4 * MB + b], p1 = pb[J * 4 * MB + MB + b];
            acc[b] += a0.x * p0.x;
            acc[b] += a0.y * p0.y;
            acc[b] += a0.z * p0.z;
            acc[b] += a0.w * p0.w;
            acc[b] += a1.x * p1.x;
            acc[b] += a1.y * p1.y;
            acc[b] += a1.z * p1.z;
            acc[b] += a1.w * p1.w;
        }
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) acc[b] += __shfl_xor(acc[b], 32, 64);
    if (w > 0)
#pragma unroll
        for (int b = 0; b < MB; ++b) red[w - 1][b][lane] = acc[b];
    __syncthreads();
    if (w != 0) return;
    const int64_t i = I * 32 + l32;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const float zf = ((acc[b] + red[0][b][lane]) + red[1][b][lane]) + red[2][b][lane];
        double pz = 0.0;
        if (h == 0 && i < n) {
            const double z = (double)zf;
            Z[i + (int64_t)b * n] = z;
            pz = P[i + (int64_t)b * n] * z;
        }
        pz = wave_sum(pz);
        if (lane == 0) part[blockIdx.x + (int64_t)b * npart] = pz;
    }
}

// z = A~ p for 5..32 right-hand sides per launch row (blockIdx.y picks the
// block of 32) on v_mfma_f32_32x32x2f32, split along k over CG_KS slices.
// Workgroup b owns the 32 rows of z of column block b / CG_KS and the
// row-block slice b % CG_KS; its four waves split the slice.  Per row block a
// lane loads two float4s of A~ (its MFMA A-operand values for k-slot h) and
// the matching two float4s of the directions (B operand: column c =
// lane % 32, the same eight rows), both fully coalesced.  Workgroups are
// dealt to the eight XCDs round-robin, so with CG_KS = 8 every XCD streams
// one eighth of the binary32 directions, which fits its L2, instead of all
// of them (9 MB at n = 70000, 32 columns).  Each slice writes its binary32
// partial z to Zp[slice][c][i]; k_cg_mv_ksum adds the slices in order.
constexpr int CG_KS = 8;
__global__ __launch_bounds__(256) void k_cg_mv_mfma_ks(const float *__restrict__ Af, int64_t ldt, int64_t n, int m,
                                                       const float *__restrict__ Pf, float *__restrict__ Zp,
                                                       const int *__restrict__ act)
{
    __shared__ float red[3][16][64];
    const int c0 = blockIdx.y * 32;
    const int mc = min(32, m - c0);
    if (!any_active(act, c0, mc)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t nJ = ldt / 16;
    const int64_t I = blockIdx.x / CG_KS, sl = blockIdx.x % CG_KS;
    const int64_t js = nJ * sl / CG_KS, je = nJ * (sl + 1) / CG_KS;
    const int64_t jb = js + (je - js) * w / 4, jend = js + (je - js) * (w + 1) / 4;
    const float *ab = Af + (I * nJ) * 512 + lane * 4;
    const float4 *pb = reinterpret_cast<const float4 *>(Pf + (int64_t)blockIdx.y * ldt * 32) + (2 * h) * 32 + l32;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll 2
    for (int64_t J = jb; J < jend; ++J) {
        const float4 a0 = *reinterpret_cast<const float4 *>(ab + J * 512);
        const float4 a1 = *reinterpret_cast<const float4 *>(ab + J * 512 + 256);
        const float4 b0 = pb[J * 128], b1 = pb[J * 128 + 32];
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
    const int c = c0 + l32;
    if (l32 >= mc) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float s = ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
        const int64_t i = I * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (i < n) Zp[(sl * m + c) * n + i] = s;
    }
}

// z = sum of the CG_KS slices (binary32, slice order), widened; one partial
// of p^T z per workgroup and column (blockIdx.y = column)
__global__ __launch_bounds__(256) void k_cg_mv_ksum(int64_t n, int m, const float *__restrict__ Zp,
                                                    const double *__restrict__ P, double *__restrict__ Z,
                                                    double *__restrict__ part, int64_t npart,
                                                    const int *__restrict__ act)
{
    __shared__ double red[4];
    const int c = blockIdx.y;
    if (!act[c]) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double pz = 0.0;
    if (i < n) {
        float s = Zp[(int64_t)c * n + i];
#pragma unroll
        for (int q = 1; q < CG_KS; ++q) s += Zp[((int64_t)q * m + c) * n + i];
        const double z = (double)s;
        Z[i + (int64_t)c * n] = z;
        pz = P[i + (int64_t)c * n] * z;
    }
    pz = block_sum256(pz, red);
    if (threadIdx.x == 0) part[blockIdx.x + (int64_t)c * npart] = pz;
}

// z = A~ p on the band: a thread per row; the directions of up to CB
// right-hand sides over the workgroup's rows and their k-wide halo staged
// in LDS column by column (pitch span + 1), each band value loaded once and
// applied to all of them
template <int CB>
__global__ __launch_bounds__(256) void k_cg_mv_band(const float *__restrict__ Bd, int64_t ldt, int64_t n, int64_t k,
                                                    int m, int W, const float *__restrict__ Pf,
                                                    const double *__restrict__ P, double *__restrict__ Z,
                                                    double *__restrict__ part, int64_t npart,
                                                    const int *__restrict__ act)
{
    extern __shared__ float pl[];  // CB x (span + 1)
    __shared__ double redc[4 * CB];
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    const int t = threadIdx.x;
    const int64_t i = i0 + t;
    const int64_t span = 256 + 2 * k, pitch = span + 1;
    for (int cb = 0; cb < m; cb += CB) {
        const int cnt = min(CB, m - cb);
        if (!any_active(act, cb, cnt)) continue;  // uniform across the block
        __syncthreads();
        const int64_t total = (int64_t)cnt * span;
        for (int64_t q0 = t; q0 < total; q0 += 256 * 8) {  // eight loads in flight per thread
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t q = q0 + 256 * u;
                v[u] = 0.0f;
                if (q < total) {
                    const int c = (int)(q / span);
                    const int64_t j = i0 - k + (q - (int64_t)c * span);
                    if (j >= 0 && j < n) v[u] = Pf[pf_off(j, cb + c, W, ldt)];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t q = q0 + 256 * u;
                if (q < total) {
                    const int c = (int)(q / span);
                    pl[c * pitch + (q - (int64_t)c * span)] = v[u];
                }
            }
        }
        __syncthreads();
        float acc[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c] = 0.0f;
        if (i < n)
#pragma unroll 4
            for (int64_t d = -k; d <= k; ++d) {
                const float a = Bd[(d + k) * ldt + i];
                const float *col = pl + t + k + d;
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < cnt) acc[c] += a * col[c * pitch];
            }
        // z, and p^T z per column: wave sums, then the four waves in order
        double pz[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            pz[c] = 0.0;
            if (c < cnt && i < n) {
                const double z = (double)acc[c];
                Z[i + (int64_t)(cb + c) * n] = z;
                pz[c] = P[i + (int64_t)(cb + c) * n] * z;
            }
            pz[c] = wave_sum(pz[c]);
        }
        __syncthreads();
        if ((t & 63) == 0)
#pragma unroll
            for (int c = 0; c < CB; ++c) redc[(t >> 6) * CB + c] = pz[c];
        __syncthreads();
        if (t < cnt)
            part[blockIdx.x + (int64_t)(cb + t) * npart] =
                ((redc[t] + redc[CB + t]) + redc[2 * CB + t]) + redc[3 * CB + t];
    }
}

// P = R, Pf = fl32(R) and a partial of r^T r, for the columns starting a
// phase (blockIdx.y = column)
__global__ __launch_bounds__(256) void k_cg_start(int64_t n, int m, int W, const double *__restrict__ R,
                                                  double *__restrict__ P, float *__restrict__ Pf, int64_t ldt,
                                                  double *__restrict__ part, int64_t npart, const int *__restrict__ go)
{
    __shared__ double red[4];
    const int b = blockIdx.y;
    if (!go[b]) return;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = (int64_t)blockIdx.x * 1024 + u * 256 + threadIdx.x;
        if (i < n) {
            const double r = R[i + (int64_t)b * n];
            P[i + (int64_t)b * n] = r;
            Pf[pf_off(i, b, W, ldt)] = (float)r;
            s += r * r;
        }
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) part[blockIdx.x + (int64_t)b * npart] = s;
}

// fixed-order sum of column b's npart partials; the same value in every block
__device__ inline double sum_parts(const double *part, int64_t npart, int b, double *red)
{
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < npart; q += 256) s += part[q + (int64_t)b * npart];
    return block_sum256(s, red);
}

// Scalar state per column, double-buffered by iteration parity `par`:
// rho[par][b] = r^T r of the current iterate, act[par][b] = column still
// iterating; thr[b] = inner_tol^2 rho_0 and cnt[b] = products this phase.
// Iteration `par` reads slot par and its last kernel writes slot par ^ 1, so
// no kernel reads a slot that it also writes.

// alpha = rho / p^T z (from the product's partials, summed identically in
// every block), x += alpha p, r -= alpha z, and a partial of the new r^T r
// (blockIdx.y = column)
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int m, const double *__restrict__ pzp, int64_t npz,
                                               const double *__restrict__ rho, const double *__restrict__ P,
                                               const double *__restrict__ Z, double *__restrict__ X, int64_t ldx,
                                               double *__restrict__ R, double *__restrict__ part, int64_t npart,
                                               const int *__restrict__ act)
{
    __shared__ double red[4];
    const int b = blockIdx.y;
    if (!act[b]) return;
    const double al = rho[b] / sum_parts(pzp, npz, b, red);
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

// rho' = r^T r (partials of k_cg_xr), beta = rho' / rho, p = r + beta p,
// Pf = fl32(p) (blockIdx.y = column); block (0, b) advances the column's
// state into slot par ^ 1: rho', ++cnt, act' = cnt < max_inner && rho' > thr
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, int m, int W, const double *__restrict__ rrp, int64_t nrr,
                                              double *__restrict__ sc, int par, const double *__restrict__ R,
                                              double *__restrict__ P, float *__restrict__ Pf, int64_t ldt,
                                              int *__restrict__ act, int *__restrict__ cnt, int max_inner)
{
    __shared__ double red[4];
    const int b = blockIdx.y;
    const double *rho = sc + (int64_t)par * m;
    double *rho_next = sc + (int64_t)(par ^ 1) * m;
    const double *thr = sc + 2 * (int64_t)m;
    const int *a_cur = act + (int64_t)par * m;
    int *a_next = act + (int64_t)(par ^ 1) * m;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!a_cur[b]) {
        if (lead) {
            a_next[b] = 0;
            rho_next[b] = rho[b];
        }
        return;
    }
    const double rr = sum_parts(rrp, nrr, b, red);
    const double be = rr / rho[b];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = (int64_t)blockIdx.x * 1024 + u * 256 + threadIdx.x;
        if (i < n) {
            const double p = R[i + (int64_t)b * n] + be * P[i + (int64_t)b * n];
            P[i + (int64_t)b * n] = p;
            Pf[pf_off(i, b, W, ldt)] = (float)p;
        }
    }
    if (lead) {
        rho_next[b] = rr;
        const int c = cnt[b] + 1;
        cnt[b] = c;
        a_next[b] = (c < max_inner && rr > thr[b]) ? 1 : 0;
    }
}

// Start of a phase (one block per column): rho = r^T r into slot 0,
// thr = inner_tol^2 rho, cnt = 0, act[0] = go && max_inner > 0 && rho > thr
__global__ __launch_bounds__(256) void k_cg_begin(const double *__restrict__ part, int64_t npart,
                                                  double *__restrict__ sc, int *__restrict__ act,
                                                  const int *__restrict__ go, int *__restrict__ cnt,
                                                  double inner_tol2, int max_inner, int m)
{
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (!go[b]) {
        if (threadIdx.x == 0) {
            act[b] = 0;
            cnt[b] = 0;
        }
        return;
    }
    const double s = sum_parts(part, npart, b, red);
    if (threadIdx.x != 0) return;
    sc[b] = s;
    sc[2 * (int64_t)m + b] = inner_tol2 * s;
    cnt[b] = 0;
    act[b] = (max_inner > 0 && s > inner_tol2 * s) ? 1 : 0;
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

int cg_pf_width(int m) { return (m <= 4) ? std::max(m, 1) : 32; }
int64_t cg_pf_elems(int64_t ldt, int m)
{
    const int W = cg_pf_width(m);
    return (int64_t)((m + W - 1) / W) * W * ldt;
}

int64_t cg_mv_parts(int64_t n, int64_t ldt, int64_t k, int m)
{
    if (k >= 0) return (n + 255) / 256;
    return (m <= 4) ? ldt / 32 : (n + 255) / 256;
}

int64_t cg_zp_elems(int64_t n, int m) { return (m > 4) ? (int64_t)CG_KS * m * n : 0; }

void launch_cg_mv(const float *At, int64_t ldt, int64_t n, int64_t k, int m, const float *Pf, const double *P,
                  double *Z, double *part, int64_t npart, const int *act, float *Zp, hipStream_t st)
{
    const int W = cg_pf_width(m);
    if (k >= 0) {
        const int64_t pitch = 256 + 2 * k + 1;
        const dim3 g((unsigned)((n + 255) / 256));
        // dynamic LDS for 32 columns, plus the kernel's static reduction
        // space (1 KB), within the 64 KB a workgroup may use
        if (m > 1 && pitch * 32 * (int64_t)sizeof(float) + 1024 <= 65536)
            hipLaunchKernelGGL(k_cg_mv_band<32>, g, dim3(256), (size_t)pitch * 32 * sizeof(float), st, At, ldt, n, k,
                               m, W, Pf, P, Z, part, npart, act);
        else
            hipLaunchKernelGGL(k_cg_mv_band<1>, g, dim3(256), (size_t)pitch * sizeof(float), st, At, ldt, n, k, m, W,
                               Pf, P, Z, part, npart, act);
        return;
    }
    const dim3 blk(256), g((unsigned)(ldt / 32));
    switch (m) {
    case 1: hipLaunchKernelGGL(k_cg_mv_valu<1>, g, blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    case 2: hipLaunchKernelGGL(k_cg_mv_valu<2>, g, blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    case 3: hipLaunchKernelGGL(k_cg_mv_valu<3>, g, blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    case 4: hipLaunchKernelGGL(k_cg_mv_valu<4>, g, blk, 0, st, At, ldt, n, Pf, P, Z, part, npart, act); break;
    default:
        hipLaunchKernelGGL(k_cg_mv_mfma_ks, dim3((unsigned)(ldt / 32 * CG_KS), (unsigned)((m + 31) / 32)), blk, 0, st,
                           At, ldt, n, m, Pf, Zp, act);
        hipLaunchKernelGGL(k_cg_mv_ksum, dim3((unsigned)((n + 255) / 256), (unsigned)m), blk, 0, st, n, m, Zp, P, Z,
                           part, npart, act);
    }
}

int64_t cg_vec_parts(int64_t n) { return std::max<int64_t>((n + 1023) / 1024, 1); }

void launch_cg_start(int64_t n, int m, const double *R, double *P, float *Pf, int64_t ldt, double *part,
                     int64_t npart, const int *go, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_start, dim3((unsigned)npart, (unsigned)m), dim3(256), 0, st, n, m, cg_pf_width(m), R, P,
                       Pf, ldt, part, npart, go);
}

void launch_cg_xr(int64_t n, int m, const double *pzp, int64_t npz, const double *sc, int par, const double *P,
                  const double *Z, double *X, int64_t ldx, double *R, double *part, int64_t npart, const int *act,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_xr, dim3((unsigned)npart, (unsigned)m), dim3(256), 0, st, n, m, pzp, npz,
                       sc + (int64_t)par * m, P, Z, X, ldx, R, part, npart, act + (int64_t)par * m);
}

void launch_cg_p(int64_t n, int m, const double *rrp, int64_t nrr, double *sc, int par, const double *R, double *P,
                 float *Pf, int64_t ldt, int *act, int *cnt, int max_inner, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_p, dim3((unsigned)cg_vec_parts(n), (unsigned)m), dim3(256), 0, st, n, m, cg_pf_width(m),
                       rrp, nrr, sc, par, R, P, Pf, ldt, act, cnt, max_inner);
}

void launch_cg_begin(const double *part, int64_t npart, double *sc, int *act, const int *go, int *cnt,
                     double inner_tol2, int max_inner, int m, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_begin, dim3((unsigned)m), dim3(256), 0, st, part, npart, sc, act, go, cnt, inner_tol2,
                       max_inner, m);
}

}  // namespace spd
