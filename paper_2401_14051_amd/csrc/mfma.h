// mfma.h -- 16x16 MFMA fragments for gfx950 in float32 and bfloat16 (the
// CNN and the FP32 backbone).
//
// Lane layouts (wave64, lane l, g = l / 16, r = l % 16):
//   A (16 x K):  row r, k = g*KPL + e for element e < KPL
//   B (K x 16):  col r, k = g*KPL + e
//   D (16 x 16): row g*4 + i, col r, for i < 4
// FP32 uses v_mfma_f32_16x16x4_f32 (K = 4, one element per lane), BF16 uses
// v_mfma_f32_16x16x32_bf16 (K = 32, eight elements per lane).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nis {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int PREC> struct Mfma;

template <> struct Mfma<0> {
    static constexpr int KS = 4;    // K per instruction
    static constexpr int KPL = 1;   // K elements per lane
    typedef float elem;             // storage type of operands
    typedef float frag;
    __device__ static __forceinline__ f32x4 mma(frag a, frag b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    template <class Get> __device__ static __forceinline__ frag gather(Get get, int k0)
    {
        return get(k0);
    }
    __device__ static __forceinline__ frag load(const elem* p) { return *p; }
    __device__ static __forceinline__ elem cvt(float x) { return x; }
    __device__ static __forceinline__ elem zero() { return 0.f; }
};

template <> struct Mfma<1> {
    static constexpr int KS = 32;
    static constexpr int KPL = 8;
    typedef __bf16 elem;
    typedef bf16x8 frag;
    __device__ static __forceinline__ f32x4 mma(frag a, frag b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    template <class Get> __device__ static __forceinline__ frag gather(Get get, int k0)
    {
        frag f;
#pragma unroll
        for (int e = 0; e < 8; e++) f[e] = get(k0 + e);
        return f;
    }
    __device__ static __forceinline__ frag load(const elem* p)
    {
        return *reinterpret_cast<const frag*>(p);
    }
    __device__ static __forceinline__ elem cvt(float x) { return (__bf16)x; }
    __device__ static __forceinline__ elem zero() { return (__bf16)0.f; }
};

}  // namespace nis
