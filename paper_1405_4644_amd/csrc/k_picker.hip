// Training kernels of the precision picker: a 16 -> 64 -> 64 -> 4 perceptron
// (ReLU hidden layers, softmax cross-entropy), binary32.  Parameters are one
// flat vector: W1 (64 x 16), b1, W2 (64 x 64), b2, W3 (4 x 64), b3, weight
// matrices row-major [out][in].  Samples X are row-major N x 16.
//
//   k_mlp_forward  logits of every sample (one thread per sample, the
//                  parameters staged in shared memory);
//   k_mlp_grad     per block of 64 samples: forward, backward and the block's
//                  parameter gradient (sums over its samples) and loss;
//   k_mlp_reduce   sums the block partials in block order (deterministic);
//   k_adam         one Adam step (bias-corrected moments).
#include "common.h"
#include "internal.h"

#define NF 16
#define NHID 64
#define NC 4
#define OFF_B1 (NHID * NF)
#define OFF_W2 (OFF_B1 + NHID)
#define OFF_B2 (OFF_W2 + NHID * NHID)
#define OFF_W3 (OFF_B2 + NHID)
#define OFF_B3 (OFF_W3 + NC * NHID)
#define GB 64  // samples per gradient block

__global__ __launch_bounds__(64) void k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X,
                                                    int64_t N, float *__restrict__ logits)
{
    __shared__ float Ps[PICK_NPARAM];
    for (int k = threadIdx.x; k < PICK_NPARAM; k += 64) Ps[k] = P[k];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (s >= N)
        return;
    float x[NF], h1[NHID], z[NC];
#pragma unroll
    for (int k = 0; k < NF; ++k) x[k] = X[s * NF + k];
#pragma unroll
    for (int u = 0; u < NHID; ++u) {
        float a = Ps[OFF_B1 + u];
#pragma unroll
        for (int k = 0; k < NF; ++k) a += Ps[u * NF + k] * x[k];
        h1[u] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) z[c] = Ps[OFF_B3 + c];
    for (int u = 0; u < NHID; ++u) {
        float a = Ps[OFF_B2 + u];
#pragma unroll
        for (int k = 0; k < NHID; ++k) a += Ps[OFF_W2 + u * NHID + k] * h1[k];
        const float h2 = fmaxf(a, 0.0f);
#pragma unroll
        for (int c = 0; c < NC; ++c) z[c] += Ps[OFF_W3 + c * NHID + u] * h2;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) logits[s * NC + c] = z[c];
}

// Block b owns samples [64 b, 64 b + 64): partial[b][k] = sum over its samples
// of d(loss_s)/d(param k) / N, loss_part[b] = sum of its losses / N.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                  const int32_t *__restrict__ y, int64_t N,
                                                  float *__restrict__ partial, float *__restrict__ loss_part)
{
    __shared__ float Ps[PICK_NPARAM];
    __shared__ float Xs[GB][NF];
    __shared__ float H1[GB][NHID + 1], H2[GB][NHID + 1], G1[GB][NHID + 1], G2[GB][NHID + 1];
    __shared__ float G3[GB][NC];
    __shared__ float Ls[GB];
    const int tid = threadIdx.x;
    for (int k = tid; k < PICK_NPARAM; k += 256) Ps[k] = P[k];
    const int64_t s0 = (int64_t)blockIdx.x * GB;
    for (int idx = tid; idx < GB * NF; idx += 256) {
        const int s = idx / NF, k = idx % NF;
        Xs[s][k] = (s0 + s < N) ? X[(s0 + s) * NF + k] : 0.0f;
    }
    __syncthreads();
    const float invN = 1.0f / (float)N;
    // forward and backward, one thread per sample
    if (tid < GB) {
        const int s = tid;
        const bool valid = s0 + s < N;
#pragma unroll 4
        for (int u = 0; u < NHID; ++u) {
            float a = Ps[OFF_B1 + u];
            for (int k = 0; k < NF; ++k) a += Ps[u * NF + k] * Xs[s][k];
            H1[s][u] = fmaxf(a, 0.0f);
        }
        float z[NC];
        for (int c = 0; c < NC; ++c) z[c] = Ps[OFF_B3 + c];
        for (int u = 0; u < NHID; ++u) {
            float a = Ps[OFF_B2 + u];
            for (int k = 0; k < NHID; ++k) a += Ps[OFF_W2 + u * NHID + k] * H1[s][k];
            const float h2 = fmaxf(a, 0.0f);
            H2[s][u] = h2;
            for (int c = 0; c < NC; ++c) z[c] += Ps[OFF_W3 + c * NHID + u] * h2;
        }
        float zmax = z[0];
        for (int c = 1; c < NC; ++c) zmax = fmaxf(zmax, z[c]);
        float e[NC], se = 0.0f;
        for (int c = 0; c < NC; ++c) {
            e[c] = expf(z[c] - zmax);
            se += e[c];
        }
        const int lab = valid ? y[s0 + s] : 0;
        float g3[NC];
        for (int c = 0; c < NC; ++c) {
            const float pc = e[c] / se;
            g3[c] = valid ? (pc - (c == lab ? 1.0f : 0.0f)) * invN : 0.0f;
            G3[s][c] = g3[c];
        }
        Ls[s] = valid ? -(z[lab] - zmax - logf(se)) * invN : 0.0f;
        for (int u = 0; u < NHID; ++u) {
            float g = 0.0f;
            for (int c = 0; c < NC; ++c) g += Ps[OFF_W3 + c * NHID + u] * g3[c];
            G2[s][u] = (H2[s][u] > 0.0f) ? g : 0.0f;
        }
        for (int k = 0; k < NHID; ++k) {
            float g = 0.0f;
            for (int u = 0; u < NHID; ++u) g += Ps[OFF_W2 + u * NHID + k] * G2[s][u];
            G1[s][k] = (H1[s][k] > 0.0f) ? g : 0.0f;
        }
    }
    __syncthreads();
    // block gradient: every parameter is a sum over the 64 samples, in order
    float *out = partial + (int64_t)blockIdx.x * PICK_NPARAM;
    for (int k = tid; k < PICK_NPARAM; k += 256) {
        float g = 0.0f;
        if (k < OFF_B1) {
            const int u = k / NF, i = k % NF;
            for (int s = 0; s < GB; ++s) g += G1[s][u] * Xs[s][i];
        } else if (k < OFF_W2) {
            const int u = k - OFF_B1;
            for (int s = 0; s < GB; ++s) g += G1[s][u];
        } else if (k < OFF_B2) {
            const int u = (k - OFF_W2) / NHID, i = (k - OFF_W2) % NHID;
            for (int s = 0; s < GB; ++s) g += G2[s][u] * H1[s][i];
        } else if (k < OFF_W3) {
            const int u = k - OFF_B2;
            for (int s = 0; s < GB; ++s) g += G2[s][u];
        } else if (k < OFF_B3) {
            const int c = (k - OFF_W3) / NHID, i = (k - OFF_W3) % NHID;
            for (int s = 0; s < GB; ++s) g += G3[s][c] * H2[s][i];
        } else {
            const int c = k - OFF_B3;
            for (int s = 0; s < GB; ++s) g += G3[s][c];
        }
        out[k] = g;
    }
    if (tid == 0) {
        float l = 0.0f;
        for (int s = 0; s < GB; ++s) l += Ls[s];
        loss_part[blockIdx.x] = l;
    }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial,
                                                    const float *__restrict__ loss_part, int nblk,
                                                    float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < PICK_NPARAM) {
        float g = 0.0f;
        for (int b = 0; b < nblk; ++b) g += partial[(int64_t)b * PICK_NPARAM + k];
        grad[k] = g;
    }
    if (k == 0 && loss) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += loss_part[b];
        *loss = l;
    }
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int64_t count, float lr,
                                              float b1, float b2, float eps, float c1, float c2)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count)
        return;
    const float mk = b1 * m[k] + (1.0f - b1) * g[k];
    const float vk = b2 * v[k] + (1.0f - b2) * g[k] * g[k];
    m[k] = mk;
    v[k] = vk;
    P[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

namespace spd {

void launch_mlp_forward(const float *P, const float *X, int64_t N, float *logits, hipStream_t st)
{
    if (N <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((N + 63) / 64)), dim3(64), 0, st, P, X, N, logits);
}

int64_t mlp_grad_scratch(int64_t N)
{
    const int64_t nblk = (N + GB - 1) / GB;
    return nblk * PICK_NPARAM + nblk;
}

void launch_mlp_grad(const float *P, const float *X, const int32_t *y, int64_t N, float *grad, float *loss,
                     float *scratch, hipStream_t st)
{
    if (N <= 0) return;
    const int nblk = (int)((N + GB - 1) / GB);
    float *partial = scratch, *loss_part = scratch + (int64_t)nblk * PICK_NPARAM;
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)nblk), dim3(256), 0, st, P, X, y, N, partial, loss_part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((PICK_NPARAM + 255) / 256), dim3(256), 0, st, partial, loss_part, nblk,
                       grad, loss);
}

void launch_adam(float *P, const float *g, float *m, float *v, int64_t count, int step, float lr, float b1, float b2,
                 float eps, hipStream_t st)
{
    if (count <= 0) return;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, P, g, m, v, count, lr, b1,
                       b2, eps, c1, c2);
}

}  // namespace spd
