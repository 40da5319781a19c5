// Shared device-side definitions for libspd (gfx950 / CDNA4 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

#define SPD_DEV __device__ __forceinline__

// Global-memory views of generic pointers.  In a device function that is not
// inlined into its kernel the compiler cannot tell global from shared memory
// and emits FLAT accesses, which count against the shared-memory wait
// counter as well: a shared-memory read then waits for every global load in
// flight, so loads issued ahead never overlap the work between.  Accesses
// through these views are GLOBAL instructions.
template <typename T>
SPD_DEV __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
template <typename T>
SPD_DEV const __attribute__((address_space(1))) T *gmem(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}

// Panel width of the blocked factorisation and tile sizes.
#define SPD_IB 32           // inner strip width inside a diagonal block
#define SPD_TILE 128        // trailing-update tile (rows and columns)
#define SPD_INFO_NONE 0x7fffffffffffffffLL

// ---------------------------------------------------------------------------
// 32x32 output tile per wavefront: acc += A(32 x K) * B(32 x K)^T.
// The MFMA lane layouts (checked on the device):
//  * v_mfma_f32_32x32x2f32: lane l supplies A[l%32][k0 + l/32] and
//    B[l%32][k0 + l/32]; accumulator register j holds
//    C[8*(j/4) + 4*(l/32) + j%4][l%32].
//  * v_mfma_f64_16x16x4f64: lane l supplies A[l%16][k0 + l/16] and
//    B[l%16][k0 + l/16]; register j holds C[4*j + l/16][l%16].
// A 32x32 binary64 tile is 2x2 such 16x16 blocks.
// ---------------------------------------------------------------------------
template <typename T> struct Acc32;
template <> struct Acc32<float> {
    floatx16 v;
    SPD_DEV void zero() { for (int j = 0; j < 16; ++j) v[j] = 0.f; }
    // One k-step of 2 (float32): a = A[l%32][k0+l/32], b = B[l%32][k0+l/32]
    SPD_DEV void mma(float a, float b) { v = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, v, 0, 0, 0); }
    // (row, col) of register j for lane l
    static SPD_DEV int row(int j, int l) { return 8 * (j / 4) + 4 * (l / 32) + (j % 4); }
    static SPD_DEV int col(int j, int l) { return l % 32; }
    static constexpr int NREG = 16;
    SPD_DEV float get(int j) const { return v[j]; }
    SPD_DEV void set(int j, float x) { v[j] = x; }
};
template <> struct Acc32<double> {
    doublex4 v[2][2];
    SPD_DEV void zero() {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int j = 0; j < 4; ++j) v[a][b][j] = 0.0;
    }
    // One k-step of 4 (float64): a[mi] = A[16 mi + l%16][k0 + l/16], b[ni] likewise
    SPD_DEV void mma(const double a[2], const double b[2]) {
        for (int mi = 0; mi < 2; ++mi)
            for (int ni = 0; ni < 2; ++ni)
                v[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], v[mi][ni], 0, 0, 0);
    }
    // flattened register index j in [0,16): mi = j/8, ni = (j/4)%2, r = j%4
    static SPD_DEV int row(int j, int l) { return 16 * (j / 8) + 4 * (j % 4) + l / 16; }
    static SPD_DEV int col(int j, int l) { return 16 * ((j / 4) % 2) + l % 16; }
    static constexpr int NREG = 16;
    SPD_DEV double get(int j) const { return v[j / 8][(j / 4) % 2][j % 4]; }
    SPD_DEV void set(int j, double x) { v[j / 8][(j / 4) % 2][j % 4] = x; }
};

// One k-step fragment of a 32-row operand block whose rows are contiguous in
// memory (element (r, k) at p[r + k*ks]).  binary32: one value per lane
// (rows l%32, k-step 2); binary64: two values per lane (rows l%16 and
// 16 + l%16, k-step 4).
template <typename T> struct Frag;
template <> struct Frag<float> {
    static constexpr int K = 2;
    float v;
    SPD_DEV void load(const float *p, int ks, int lane) { v = p[(lane & 31) + (lane >> 5) * ks]; }
    SPD_DEV void negate() { v = -v; }
};
template <> struct Frag<double> {
    static constexpr int K = 4;
    double v[2];
    SPD_DEV void load(const double *p, int ks, int lane)
    {
        const int r = lane & 15, kk = lane >> 4;
        v[0] = p[r + kk * ks];
        v[1] = p[16 + r + kk * ks];
    }
    SPD_DEV void negate() { v[0] = -v[0]; v[1] = -v[1]; }
};
SPD_DEV void mma(Acc32<float> &acc, const Frag<float> &a, const Frag<float> &b) { acc.mma(a.v, b.v); }

SPD_DEV void mma(Acc32<double> &acc, const Frag<double> &a, const Frag<double> &b) { acc.mma(a.v, b.v); }

// acc += A(32 x kc) * B(32 x kc)^T with A(r,k) = pa[r + k*aks], B(r,k) = pb[r + k*bks];
// kc a multiple of Frag<T>::K.
template <typename T>
SPD_DEV void mma_tile(Acc32<T> &acc, const T *pa, int aks, const T *pb, int bks, int kc, int lane)
{
#pragma unroll 4
    for (int k = 0; k < kc; k += Frag<T>::K) {
        Frag<T> a, b;
        a.load(pa + (size_t)k * aks, aks, lane);
        b.load(pb + (size_t)k * bks, bks, lane);
        mma(acc, a, b);
    }
}

// Cooperative copy of a ROWS x cols column-major block (leading dimension ld)
// into LDS as dst[c * dld + r].  Each thread issues UNROLL global loads
// before storing any of them, so load latency overlaps instead of
// serialising on every element.  NT = threads taking part (tid < NT).
template <typename T, int ROWS, int NT, int UNROLL>
SPD_DEV void copy_g2s(T *dst, int dld, const T *__restrict__ src, int64_t ld, int cols, int tid)
{
    const int total = ROWS * cols;
    for (int base = 0; base < total; base += NT * UNROLL) {
        T v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int idx = base + u * NT + tid;
            if (idx < total)
                v[u] = src[(idx % ROWS) + (int64_t)(idx / ROWS) * ld];
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int idx = base + u * NT + tid;
            if (idx < total)
                dst[(idx / ROWS) * dld + (idx % ROWS)] = v[u];
        }
    }
}

// Workgroup barrier that orders shared-memory accesses only: unlike
// __syncthreads() it does not wait for the wave's global stores to complete.
SPD_DEV void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Word 3 of a raw buffer resource on gfx950 (32-bit data format, no
// swizzle): used with __builtin_amdgcn_make_buffer_rsrc.
#define SPD_BUFFER_RSRC_WORD3 0x00020000

// Monotone atomic max of a non-negative double via its bit pattern (NaN,
// whose bits exceed +inf's, wins -- so a NaN anywhere propagates).
SPD_DEV void atomic_max_nonneg(double *addr, double v)
{
    unsigned long long bits = __double_as_longlong(v);
    atomicMax(reinterpret_cast<unsigned long long *>(addr), bits);
}

// Smallest power of two s with v <= s (1 for v == 0, inf or NaN).
SPD_DEV double pow2_ceil(double v)
{
    if (!(v > 0.0) || v == __builtin_inf())
        return 1.0;
    int e;
    double f = frexp(v, &e);
    return (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}
