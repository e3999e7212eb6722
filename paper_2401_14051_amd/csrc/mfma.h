// mfma.h -- 16x16 MFMA fragments for gfx950 in float32 and bfloat16.
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

// FP8 (OCP E4M3FN): v_mfma_scale_f32_16x16x128_f8f6f4 with unit block scales
// (E8M0 exponent 127), K = 128, 32 one-byte elements per lane.  Elements are
// raw fp8 codes; the caller applies its own per-row and per-column scales.
typedef int i32x8 __attribute__((ext_vector_type(8)));
template <> struct Mfma<2> {
    static constexpr int KS = 128;
    static constexpr int KPL = 32;
    typedef uint8_t elem;
    typedef i32x8 frag;
    __device__ static __forceinline__ f32x4 mma(frag a, frag b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    }
    __device__ static __forceinline__ frag load(const elem* p) { return *reinterpret_cast<const frag*>(p); }
    __device__ static __forceinline__ elem zero() { return 0; }
};

// Largest finite OCP E4M3FN value; the hardware conversion does not saturate.
constexpr float kFp8Max = 448.f;

// Four floats (already scaled) -> four E4M3FN codes packed little-endian.
__device__ __forceinline__ int pack_fp8x4(float a, float b, float c, float d)
{
    a = fminf(fmaxf(a, -kFp8Max), kFp8Max);
    b = fminf(fmaxf(b, -kFp8Max), kFp8Max);
    c = fminf(fmaxf(c, -kFp8Max), kFp8Max);
    d = fminf(fmaxf(d, -kFp8Max), kFp8Max);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}

// As pack_fp8x4 for values already known to lie in [-448, 448] after rounding
// to E4M3 (callers scale to at most 447.5 in magnitude).
__device__ __forceinline__ int pack_fp8x4_inrange(float a, float b, float c, float d)
{
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}

}  // namespace nis
