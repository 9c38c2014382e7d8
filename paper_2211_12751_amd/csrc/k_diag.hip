// Hardware diagnostics.  Matrix-core accumulation probe.  The library's fast scores assume that a matrix-core
// product accumulates like FP32 arithmetic (the error model of the fast decisions and of
// the lambda certificate); this probe measures one 32 x 32 block of products of e4m3
// codes on the FP8 matrix cores (codes as they are) and on the BF16 matrix cores (codes
// widened to BF16, which is exact), so that the assumption can be checked against exact
// sums on the host.  It is the measurement behind multiplying FP8 data on the BF16
// matrix cores.
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace rk {

typedef long fp8x8;   // eight e4m3 codes, one matrix-core operand register pair
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
// E8M0 block scale 2^(127 - 127) = 1 for the scaled FP8 matrix-core instruction
constexpr int kUnitScale = 127;

// C[i][j] = sum_k A[i][k] B[j][k] for i, j < 32 over K (a multiple of 16), one wave.
// Lane l supplies row l % 32 of each operand, elements [8 (l / 32), 8 (l / 32) + 8) of
// every 16-wide k step; accumulator element r of lane l is C[mfma32_row(r, l)][l % 32].
__global__ __launch_bounds__(64) void k_mma_probe(const uint8_t* A, const uint8_t* B, int K, int kind, float* C)
{
    const int l = threadIdx.x;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.f;
    if (kind == 2) {
        // 32x32x64 steps: lane l supplies 32 codes of row l % 32, bytes [32 (l / 32), +32)
        // of every 64-wide k step, the same for both operands (any order the instruction
        // gives those bytes applies to both, so the sum covers every k once); unit scales
        for (int k0 = 0; k0 < K; k0 += 64) {
            const uint8_t* ar = A + (int64_t)(l & 31) * K + k0 + 32 * (l >> 5);
            const uint8_t* br = B + (int64_t)(l & 31) * K + k0 + 32 * (l >> 5);
            i32x8 a, b;
            for (int e = 0; e < 8; e++) {
                a[e] = (int)((uint32_t)ar[4 * e] | ((uint32_t)ar[4 * e + 1] << 8) | ((uint32_t)ar[4 * e + 2] << 16) |
                             ((uint32_t)ar[4 * e + 3] << 24));
                b[e] = (int)((uint32_t)br[4 * e] | ((uint32_t)br[4 * e + 1] << 8) | ((uint32_t)br[4 * e + 2] << 16) |
                             ((uint32_t)br[4 * e + 3] << 24));
            }
            acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, kUnitScale, 0, kUnitScale);
        }
#pragma unroll
        for (int r = 0; r < 16; r++) C[mfma32_row(r, l) * 32 + (l & 31)] = acc[r];
        return;
    }
    for (int k0 = 0; k0 < K; k0 += 16) {
        const uint8_t* ar = A + (int64_t)(l & 31) * K + k0 + 8 * (l >> 5);
        const uint8_t* br = B + (int64_t)(l & 31) * K + k0 + 8 * (l >> 5);
        if (kind == 1) {
            fp8x8 a = 0, b = 0;
            for (int e = 0; e < 8; e++) {
                a |= (long)ar[e] << (8 * e);
                b |= (long)br[e] << (8 * e);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, acc, 0, 0, 0);
        } else {
            bf16x8 a, b;
            for (int e = 0; e < 8; e++) {
                a[e] = __builtin_bit_cast(__bf16, (uint16_t)(__float_as_uint(e4m3_to_f32(ar[e])) >> 16));
                b[e] = __builtin_bit_cast(__bf16, (uint16_t)(__float_as_uint(e4m3_to_f32(br[e])) >> 16));
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; r++) C[mfma32_row(r, l) * 32 + (l & 31)] = acc[r];
}

void mma_probe(int kind, const uint8_t* a_host, const uint8_t* b_host, int K, float* c_host)
{
    if (kind < 0 || kind > 2) fail(RKMIPS_EINVAL, "kind must be 0 (BF16), 1 (FP8) or 2 (FP8, K = 64 steps)");
    if (K < 16 || K > 4096 || K % 16 != 0) fail(RKMIPS_EINVAL, "K must be a multiple of 16 in [16, 4096]");
    if (kind == 2 && K % 64 != 0) fail(RKMIPS_EINVAL, "kind 2 needs K a multiple of 64");
    if (!a_host || !b_host || !c_host) fail(RKMIPS_EINVAL, "null pointer");
    for (int i = 0; i < 32 * K; i++)
        if ((a_host[i] & 0x7f) == 0x7f || (b_host[i] & 0x7f) == 0x7f) fail(RKMIPS_EINVAL, "NaN code");
    uint8_t *a = nullptr, *b = nullptr;
    float* c = nullptr;
    const size_t nb = (size_t)32 * K;
    hipError_t e = hipMalloc(&a, nb);
    if (e == hipSuccess) e = hipMalloc(&b, nb);
    if (e == hipSuccess) e = hipMalloc(&c, sizeof(float) * 32 * 32);
    if (e == hipSuccess) e = hipMemcpy(a, a_host, nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b, b_host, nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mma_probe, dim3(1), dim3(64), 0, 0, a, b, K, kind, c);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(c_host, c, sizeof(float) * 32 * 32, hipMemcpyDeviceToHost);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(c);
    HIPC(e);
}

// e4m3 decoding with the hardware conversion (v_cvt_pk_f32_fp8, two codes per instruction):
// word i holds codes 4i .. 4i + 3 in byte order; out[4i + j] = value of code j of word i.
__global__ __launch_bounds__(256) void k_fp8_decode(const uint32_t* w, int64_t nw, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
    const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
    out[4 * i + 0] = lo[0];
    out[4 * i + 1] = lo[1];
    out[4 * i + 2] = hi[0];
    out[4 * i + 3] = hi[1];
}

void fp8_decode(const uint8_t* codes_host, int n, float* out_host)
{
    if (!codes_host || !out_host) fail(RKMIPS_EINVAL, "null pointer");
    if (n < 4 || n > (1 << 20) || n % 4 != 0) fail(RKMIPS_EINVAL, "n must be a multiple of 4 in [4, 2^20]");
    uint32_t* w = nullptr;
    float* out = nullptr;
    hipError_t e = hipMalloc(&w, (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&out, sizeof(float) * (size_t)n);
    if (e == hipSuccess) e = hipMemcpy(w, codes_host, (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int64_t nw = n / 4;
        hipLaunchKernelGGL(k_fp8_decode, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, 0, w, nw, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out_host, out, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(w);
    (void)hipFree(out);
    HIPC(e);
}

}  // namespace rk
