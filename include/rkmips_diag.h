/* Diagnostics of the hardware assumptions behind the RkMIPS library (librkmips.so).
 *
 * The fast scores of the lambda build and of the query verification are products on
 * the matrix cores with FP32 accumulation; their error bound (and so every margin test
 * and the lambda certificate, Definition 1) assumes that the matrix cores accumulate
 * like FP32 arithmetic.  This call measures one instruction sequence so that the
 * assumption can be checked against exact sums. */
#ifndef RKMIPS_DIAG_H
#define RKMIPS_DIAG_H

#include "rkmips.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One 32 x 32 block C[i][j] = sum_k A[i][k] B[j][k] of OCP e4m3 codes over k < K, on
 * the FP8 matrix cores (kind 1: v_mfma_f32_32x32x16_fp8_fp8 on the codes; kind 2:
 * v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales, K a multiple of 64) or on the
 * BF16 matrix cores (kind 0: the codes widened to BF16, which is exact, and
 * v_mfma_f32_32x32x16_bf16), FP32 accumulation in all, K / 16 (K / 64) instructions in
 * index order.  a_codes, b_codes: host uint8 [32 x K] row-major; c_out: host float [32 x 32]
 * row-major (row of A, row of B).  The caller owns every array.  Synchronous on the
 * current device's default stream; allocates and frees its own device buffers.
 * Errors: EINVAL (kind not 0/1/2, K not a multiple of 16 in [16, 4096] (of 64 for kind
 * 2), a NULL pointer, a NaN code), EDEVICE. */
rkmips_status rkmips_diag_mma_probe(int32_t kind, const uint8_t *a_codes, const uint8_t *b_codes, int32_t k,
                                    float *c_out);

/* OCP e4m3 decoding with the hardware conversion instruction (v_cvt_pk_f32_fp8, two codes
 * per instruction), which the canonical FP8 rescoring of the lambda build uses: every e4m3
 * value is exact in FP32, so the conversion must reproduce the format's definition (sign,
 * four exponent bits with bias 7, three mantissa bits, subnormals m 2^-9, codes 0x7f and
 * 0xff NaN).  codes: host uint8 [n]; out: host float [n], out[i] the value of codes[i].
 * n a multiple of 4 in [4, 2^20].  The caller owns both arrays.  Synchronous on the
 * current device's default stream; allocates and frees its own device buffers.
 * Errors: EINVAL (NULL pointer, bad n), EDEVICE. */
rkmips_status rkmips_diag_fp8_decode(const uint8_t *codes, int32_t n, float *out);

#ifdef __cplusplus
}
#endif

#endif /* RKMIPS_DIAG_H */
