// Device-side helpers shared by the RkMIPS kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

#define RK_WAVE 64

enum { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2,
       // matrix-core operand form only: FP8 e4m3 codes widened to BF16 (every e4m3 value
       // is a BF16 value), with the per-row FP8 scales applied after the product
       DT_FP8B = 3,
       // matrix-core operand form only: FP32 rows split into BF16 pairs [hi | lo]
       // (hi = RN_bf16(x), lo = RN_bf16(x - hi)); a product takes the three terms
       // hi.hi + lo.hi + hi.lo, each k-step's hi fragment serving two of them
       DT_SPLIT = 4 };

// operand types whose rows carry a per-row scale
template <int DT> constexpr bool dt_scaled = DT == DT_FP8 || DT == DT_FP8B;
// operand types multiplied on the BF16 matrix cores
template <int DT> constexpr bool dt_bf16_mma = DT == DT_BF16 || DT == DT_FP8B;

// ------------------------------------------------------------------ element decoding
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// OCP e4m3fn code -> value (exact in FP32/FP64).  NaN codes are rejected at input
// validation, so they are not special-cased here.
__device__ __forceinline__ float e4m3_to_f32(uint8_t c)
{
    uint32_t e = (c >> 3) & 15u, mnt = c & 7u;
    float v = (e == 0) ? (float)mnt * 0.001953125f                       // m * 2^-9
                       : __uint_as_float(((e + 120u) << 23) | (mnt << 20)); // (1+m/8) 2^(e-7)
    return (c & 0x80u) ? -v : v;
}

template <int DT>
__device__ __forceinline__ float elem_f32(const void* base, int64_t idx)
{
    if constexpr (DT == DT_F32) return ((const float*)base)[idx];
    else if constexpr (DT == DT_BF16 || DT == DT_FP8B) return bf16_to_f32(((const uint16_t*)base)[idx]);
    else return e4m3_to_f32(((const uint8_t*)base)[idx]);
}

template <int DT> struct Elt;
template <> struct Elt<DT_F32> { typedef float T; static constexpr int bytes = 4; };
template <> struct Elt<DT_BF16> { typedef uint16_t T; static constexpr int bytes = 2; };
template <> struct Elt<DT_FP8> { typedef uint8_t T; static constexpr int bytes = 1; };
template <> struct Elt<DT_FP8B> { typedef uint16_t T; static constexpr int bytes = 2; };
template <> struct Elt<DT_SPLIT> { typedef uint16_t T; static constexpr int bytes = 2; };

// Canonical FP64 inner product of two stored rows over the first d elements:
// FP32/BF16 data: ((0 + a0 b0) + a1 b1) + ... in index order (products exact in FP64);
// FP8 data: exact sum of code products, then one rounding by the scale product.
template <int DT>
__device__ __forceinline__ double canon_dot(const void* A, int64_t ra, float sa, const void* B,
                                            int64_t rb, float sb, int d, int ld)
{
    double acc = 0.0;
    const int64_t oa = ra * ld, ob = rb * ld;
    for (int i = 0; i < d; i++)
        acc = __fma_rn((double)elem_f32<DT>(A, oa + i), (double)elem_f32<DT>(B, ob + i), acc);
    if constexpr (DT == DT_FP8) acc = ((double)sa * (double)sb) * acc;
    return acc;
}

// ------------------------------------------------------------------ orderable keys
__device__ __forceinline__ uint32_t f32_ord(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_f32(uint32_t o)
{
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint64_t f64_ord(double f)
{
    uint64_t u = (uint64_t)__double_as_longlong(f);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_f64(uint64_t o)
{
    uint64_t u = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double((long long)u);
}

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o); v = v > w ? v : w; }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o); v = v < w ? v : w; }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_or(T v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}
// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int l = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        int w = __shfl_up(v, o);
        if (l >= o) v += w;
    }
    return v;
}

// 32x32 MFMA accumulator layout (single block): register r of lane l holds
// row 8*(r/4) + 4*(l/32) + (r%4), column l%32.
__device__ __forceinline__ int mfma32_row(int r, int l) { return ((r >> 2) << 3) + ((l >> 5) << 2) + (r & 3); }

// SplitMix64 (Steele, Lea, Flood 2014) finaliser: a counter-based generator.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
