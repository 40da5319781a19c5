// Binary16 / bfloat16 operand types of the half-precision trailing update
// and of the panel solve's rounded copy (device code; after common.h and
// internal.h).
#pragma once
#include "common.h"
#include "internal.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int HK> struct HalfT;
template <> struct HalfT<HALF_F16> {
    using E = _Float16;
    using V8 = halfx8;
    static SPD_DEV V8 neg(V8 v) { return __builtin_bit_cast(V8, __builtin_bit_cast(u32x4, v) ^ 0x80008000u); }
    static SPD_DEV floatx16 mma(V8 a, V8 b, floatx16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};
template <> struct HalfT<HALF_BF16> {
    using E = __bf16;
    using V8 = bf16x8;
    static SPD_DEV V8 neg(V8 v) { return __builtin_bit_cast(V8, __builtin_bit_cast(u32x4, v) ^ 0x80008000u); }
    static SPD_DEV floatx16 mma(V8 a, V8 b, floatx16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};
