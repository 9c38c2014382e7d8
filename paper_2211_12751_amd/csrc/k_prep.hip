// Input preparation: validation + canonical squared norms, the norm order of the
// items (Alg. 4 / Alg. 1: sort by descending norm), row gathers into padded copies,
// unit user directions for the Cone-Tree (Fact 2: only directions matter), and a
// bitonic sort used for the item order and for the per-query result lists.
#include <utility>

#include "common.h"
#include "internal.h"

namespace rk {

// ------------------------------------------------------------------ norms + validation
// Canonical squared norm of every row (index-order FP64 sum of the exact squares; FP8:
// times the squared scale), plus what validation needs: stats[slot] = max n2 (bits of a
// non-negative double order like the value), stats[2] = min positive n2, stats[3] = 1
// on any non-finite value, NaN code or non-finite scale.
// One stored element: adds its exact square to acc in index order, clears ok on a
// non-finite value or NaN code.
template <int DT>
__device__ __forceinline__ void norm_step(uint32_t raw, double& acc, bool& ok)
{
    if constexpr (DT == DT_F32) {
        const float v = __uint_as_float(raw);
        ok &= (raw & 0x7f800000u) != 0x7f800000u;
        acc = __fma_rn((double)v, (double)v, acc);
    } else if constexpr (DT == DT_BF16) {
        ok &= (raw & 0x7f80u) != 0x7f80u;
        const double v = (double)bf16_to_f32((uint16_t)raw);
        acc = __fma_rn(v, v, acc);
    } else {
        ok &= (raw & 0x7fu) != 0x7fu;
        const double v = (double)e4m3_to_f32((uint8_t)raw);
        acc = __fma_rn(v, v, acc);
    }
}

// VEC: rows of a multiple of 16 bytes at a 16-byte aligned base, read 16 bytes at a time
// (the same index-order sum; one load per 16 bytes instead of one per element).
template <int DT, bool VEC>
__global__ __launch_bounds__(256) void k_norm2(const void* X, const float* scales, int64_t rows, int d, int ld, double* n2,
                        unsigned long long* stats, int slot)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int PER = 16 / EB;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = true;
    double acc = 0.0;
    if (r < rows) {
        const int64_t o = r * ld;
        if constexpr (VEC) {
            const i32x4* row = (const i32x4*)((const uint8_t*)X + o * EB);
            for (int c = 0; c * PER < d; c++) {
                const i32x4 v = row[c];
                const int lim = d - c * PER < PER ? d - c * PER : PER;
#pragma unroll
                for (int e = 0; e < PER; e++) {
                    if (e >= lim) break;
                    const uint32_t w = (uint32_t)v[e * EB / 4];
                    norm_step<DT>(EB == 4 ? w : (w >> (8 * ((e * EB) & 3))) & (EB == 2 ? 0xffffu : 0xffu), acc, ok);
                }
            }
        } else {
            for (int i = 0; i < d; i++) {
                uint32_t raw;
                if constexpr (DT == DT_F32) raw = ((const uint32_t*)X)[o + i];
                else if constexpr (DT == DT_BF16) raw = ((const uint16_t*)X)[o + i];
                else raw = ((const uint8_t*)X)[o + i];
                norm_step<DT>(raw, acc, ok);
            }
        }
        if constexpr (DT == DT_FP8) {
            float s = scales[r];
            ok &= (__float_as_uint(s) & 0x7f800000u) != 0x7f800000u;
            acc = ((double)s * (double)s) * acc;
        }
        n2[r] = acc;
    }
    // workgroup reduction, then one atomic per statistic that can still change it
    __shared__ unsigned long long smx[4], smn[4];
    __shared__ int sbad[4];
    const unsigned long long bits = (unsigned long long)__double_as_longlong(acc);
    const unsigned long long mx = wave_max((r < rows && ok) ? bits : 0ull);
    const unsigned long long mn = wave_min((r < rows && ok && acc > 0.0) ? bits : ~0ull);
    const bool any_bad = ballot64(r < rows && !ok) != 0ull;
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        smx[w] = mx;
        smn[w] = mn;
        sbad[w] = any_bad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long bx = 0ull, bn = ~0ull;
        int bad = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); q++) {
            bx = smx[q] > bx ? smx[q] : bx;
            bn = smn[q] < bn ? smn[q] : bn;
            bad |= sbad[q];
        }
        if (bx && bx > __hip_atomic_load(&stats[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&stats[slot], bx);
        if (bn != ~0ull && bn < __hip_atomic_load(&stats[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMin(&stats[2], bn);
        if (bad) atomicOr(&stats[3], 1ull);
    }
}

__global__ void k_norm_stats_init(unsigned long long* stats)
{
    if (threadIdx.x < 4) stats[threadIdx.x] = threadIdx.x == 2 ? ~0ull : 0ull;
}

void launch_norm_stats_init(unsigned long long* stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm_stats_init, dim3(1), dim3(64), 0, s, stats);
    HIPC(hipGetLastError());
}

void launch_norm2(int dtype, const void* X, const float* scales, int64_t rows, int d, int ld,
                  double* n2, unsigned long long* stats, int slot, hipStream_t s)
{
    if (rows <= 0) return;
    dim3 g((unsigned)((rows + 255) / 256)), b(256);
    const int eb = dtype == DT_F32 ? 4 : dtype == DT_BF16 ? 2 : 1;
    const bool vec = ((int64_t)ld * eb) % 16 == 0 && ((uintptr_t)X & 15u) == 0;
    if (vec) {
        if (dtype == DT_F32) hipLaunchKernelGGL((k_norm2<DT_F32, true>), g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
        else if (dtype == DT_BF16) hipLaunchKernelGGL((k_norm2<DT_BF16, true>), g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
        else hipLaunchKernelGGL((k_norm2<DT_FP8, true>), g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
    } else {
        if (dtype == DT_F32) hipLaunchKernelGGL((k_norm2<DT_F32, false>), g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
        else if (dtype == DT_BF16) hipLaunchKernelGGL((k_norm2<DT_BF16, false>), g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
        else hipLaunchKernelGGL((k_norm2<DT_FP8, false>), g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
    }
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ split BF16 operands
// FP32 rows as BF16 pairs: h = RN_bf16(x), l = RN_bf16(x - h) (x - h is exact in FP32).
// The row [h | l | h] of an item against the row [h | h | l] of a user gives
// h.h + l.h + h.l on the BF16 matrix cores, which differs from <x, y> by at most about
// 3 * 2^-18 sum |x_i y_i| (the dropped l.l term and the parts below l).
__device__ __forceinline__ uint16_t f32_to_bf16_rn(float x)
{
    const uint32_t b = __float_as_uint(x);   // finite input
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__global__ void k_split_bf16(const float* src, int64_t rows, int ld, uint16_t* dst, int user_layout)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * ld) return;
    const int64_t r = t / ld;
    const int i = (int)(t - r * ld);
    const float x = src[t];
    const uint16_t hb = f32_to_bf16_rn(x);
    const uint16_t lb = f32_to_bf16_rn(x - bf16_to_f32(hb));
    if (user_layout == 2) {   // pair form [hi | lo]
        uint16_t* row = dst + r * 2 * ld;
        row[i] = hb;
        row[ld + i] = lb;
        return;
    }
    uint16_t* row = dst + r * 3 * ld;
    row[i] = hb;
    row[ld + i] = user_layout ? hb : lb;
    row[2 * ld + i] = user_layout ? lb : hb;
}

void launch_split_bf16(const float* src, int64_t rows, int ld, uint16_t* dst, int user_layout, hipStream_t s)
{
    if (rows <= 0) return;
    const int64_t tot = rows * ld;
    hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, rows, ld, dst,
                       user_layout);
    HIPC(hipGetLastError());
}

// FP8 e4m3 codes [rows x ld] -> BF16 [rows x ld] (exact: every e4m3 value is a BF16
// value), for the BF16 matrix cores; the row scales stay separate.
__global__ void k_widen_fp8(const uint8_t* src, int64_t count, uint16_t* dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = (uint16_t)(__float_as_uint(e4m3_to_f32(src[t])) >> 16);
}

// Eight codes per thread (8-byte load, 16-byte store); count8 = count / 8.
__global__ void k_widen_fp8_x8(const uint2* src, int64_t count8, i32x4* dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count8) return;
    const uint2 c = src[t];
    i32x4 o;
#pragma unroll
    for (int h = 0; h < 4; h++) {
        const uint32_t w = h < 2 ? c.x : c.y;
        const int sh = 16 * (h & 1);
        const uint32_t lo = __float_as_uint(e4m3_to_f32((uint8_t)(w >> sh))) >> 16;
        const uint32_t hi = __float_as_uint(e4m3_to_f32((uint8_t)(w >> (sh + 8)))) >> 16;
        o[h] = (int)(lo | (hi << 16));
    }
    dst[t] = o;
}

void launch_mma_operand(int mma_dtype, int dtype, const void* src, int64_t rows, int ld, uint16_t* dst,
                        int user_layout, hipStream_t s)
{
    if (rows <= 0) return;
    if (dtype == DT_F32 && mma_dtype == DT_SPLIT) {
        launch_split_bf16((const float*)src, rows, ld, dst, 2, s);
    } else if (dtype == DT_F32 && mma_dtype == DT_BF16) {
        launch_split_bf16((const float*)src, rows, ld, dst, user_layout, s);
    } else if (dtype == DT_FP8 && mma_dtype == DT_FP8B) {
        const int64_t cnt = rows * ld;
        if (cnt % 8 == 0 && ((uintptr_t)src & 7u) == 0 && ((uintptr_t)dst & 15u) == 0) {
            const int64_t c8 = cnt / 8;
            hipLaunchKernelGGL(k_widen_fp8_x8, dim3((unsigned)((c8 + 255) / 256)), dim3(256), 0, s, (const uint2*)src,
                               c8, (i32x4*)dst);
        } else {
            hipLaunchKernelGGL(k_widen_fp8, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, (const uint8_t*)src,
                               cnt, dst);
        }
        HIPC(hipGetLastError());
    } else {
        fail(RKMIPS_EINVAL, "internal: no matrix-core operand form for this storage type");
    }
}

// ------------------------------------------------------------------ norm sort keys
__global__ void k_norm_keys(const double* n2, int64_t n, int64_t cap, uint64_t* keys, uint32_t* vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    if (i < n) {
        // n2 >= 0, so its bit pattern is monotone; complement -> ascending = descending norm
        keys[i] = ~(uint64_t)__double_as_longlong(n2[i]);
        vals[i] = (uint32_t)i;
    } else {
        keys[i] = ~0ull;
        vals[i] = 0xffffffffu;
    }
}

void launch_norm_keys(const double* n2, int64_t n, int64_t cap, uint64_t* keys, uint32_t* vals,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_norm_keys, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, n2, n, cap,
                       keys, vals);
    HIPC(hipGetLastError());
}

__global__ void k_permute_f64(const double* src, const uint32_t* perm, int64_t n, double* dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}
void launch_permute_f64(const double* src, const uint32_t* perm, int64_t n, double* dst, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_permute_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, perm, n, dst);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ pair sort
// Ascending by (key, val).  Chunks of up to SORT_CHUNK pairs are sorted in LDS by a
// bitonic network (one compare-exchange per thread per stage); sorted runs are then
// merged pairwise, level by level: a pair's output position is its index in its own run
// plus the number of pairs of the partner run that order before it (binary search; a
// left-run pair counts the partner's strictly smaller pairs, a right-run pair also the
// equal ones, so positions never collide).
static constexpr int SORT_CHUNK = 2048;

__device__ __forceinline__ bool lt_pair(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb)
{
    return ka < kb || (ka == kb && va < vb);
}

__global__ __launch_bounds__(SORT_CHUNK / 2) void k_sort_chunk(uint64_t* keys, uint32_t* vals, int chunk)
{
    __shared__ uint64_t sk[SORT_CHUNK];
    __shared__ uint32_t sv[SORT_CHUNK];
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int t = threadIdx.x;   // chunk / 2 threads
    sk[t] = keys[base + t];
    sv[t] = vals[base + t];
    sk[t + chunk / 2] = keys[base + t + chunk / 2];
    sv[t + chunk / 2] = vals[base + t + chunk / 2];
    __syncthreads();
    for (int k = 2; k <= chunk; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int i = 2 * j * (t / j) + (t % j);
            const int p = i + j;
            const bool asc = (i & k) == 0;   // the last stage (k = chunk) sorts every chunk ascending
            const uint64_t ka = sk[i], kb = sk[p];
            const uint32_t va = sv[i], vb = sv[p];
            if (lt_pair(kb, vb, ka, va) == asc) {
                sk[i] = kb; sk[p] = ka;
                sv[i] = vb; sv[p] = va;
            }
            __syncthreads();
        }
    }
    keys[base + t] = sk[t];
    vals[base + t] = sv[t];
    keys[base + t + chunk / 2] = sk[t + chunk / 2];
    vals[base + t + chunk / 2] = sv[t + chunk / 2];
}

__global__ void k_merge_runs(const uint64_t* ki, const uint32_t* vi, uint64_t* ko, uint32_t* vo, int64_t len,
                             int64_t w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    const int64_t r = t / w, a = t - r * w;
    const int64_t pair0 = (r & ~(int64_t)1) * w;
    const int64_t q0 = (r ^ 1) * w;
    const int64_t q1 = q0 + w < len ? q0 + w : len;
    const uint64_t kt = ki[t];
    const uint32_t vt = vi[t];
    int64_t lo = q0, hi = q0 < len ? q1 : q0;   // a partner run past the end is empty
    const bool left = (r & 1) == 0;
    while (lo < hi) {   // first partner position that orders after this pair
        const int64_t mid = (lo + hi) >> 1;
        const uint64_t km = ki[mid];
        const uint32_t vm = vi[mid];
        const bool before = left ? lt_pair(km, vm, kt, vt) : !lt_pair(kt, vt, km, vm);
        if (before) lo = mid + 1;
        else hi = mid;
    }
    const int64_t pos = pair0 + a + (lo - q0);
    ko[pos] = kt;
    vo[pos] = vt;
}

__global__ void k_fill_pad(uint64_t* keys, uint32_t* vals, int64_t n, int64_t cap)
{
    int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    keys[i] = ~0ull;
    vals[i] = 0xffffffffu;
}

void sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* tmp_keys, uint32_t* tmp_vals, int64_t n, int64_t cap,
                hipStream_t s)
{
    if (n <= 1) return;
    int chunk = 2;
    while (chunk < n && chunk < SORT_CHUNK) chunk <<= 1;
    const int64_t len = (n + chunk - 1) / chunk * chunk;
    if (cap < len) fail(RKMIPS_EINVAL, "internal: sort capacity below the padded size");
    if (len > n)
        hipLaunchKernelGGL(k_fill_pad, dim3((unsigned)((len - n + 255) / 256)), dim3(256), 0, s, keys, vals, n, len);
    hipLaunchKernelGGL(k_sort_chunk, dim3((unsigned)(len / chunk)), dim3(chunk / 2), 0, s, keys, vals, chunk);
    uint64_t *k0 = keys, *k1 = tmp_keys;
    uint32_t *v0 = vals, *v1 = tmp_vals;
    for (int64_t w = chunk; w < len; w <<= 1) {
        hipLaunchKernelGGL(k_merge_runs, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, k0, v0, k1, v1, len, w);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    if (k0 != keys) {
        HIPC(hipMemcpyAsync(keys, k0, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        HIPC(hipMemcpyAsync(vals, v0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ row gather
// One wave per destination row; bytes copied in 4-byte words when the row lengths
// allow it, else byte by byte.  Padding columns are zero.
__global__ void k_gather_rows(const uint8_t* src, int64_t src_row_bytes, const uint32_t* perm,
                              int64_t rows, int64_t copy_bytes, uint8_t* dst, int64_t dst_row_bytes,
                              const float* src_scales, float* dst_scales, int words)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int l = threadIdx.x & 63;
    if (r >= rows) return;
    const int64_t sr = perm ? (int64_t)perm[r] : r;
    const uint8_t* s = src + sr * src_row_bytes;
    uint8_t* t = dst + r * dst_row_bytes;
    if (words) {
        for (int64_t w = l; w < dst_row_bytes / 4; w += 64)
            ((uint32_t*)t)[w] = (w * 4 < copy_bytes) ? ((const uint32_t*)s)[w] : 0u;
    } else {
        for (int64_t b = l; b < dst_row_bytes; b += 64) t[b] = b < copy_bytes ? s[b] : (uint8_t)0;
    }
    if (dst_scales && l == 0) dst_scales[r] = src_scales[sr];
}

void launch_gather_rows(int dtype, const void* src, int ld_src, const float* src_scales,
                        const uint32_t* perm, int64_t rows, int d, void* dst, int ld_dst,
                        float* dst_scales, hipStream_t s)
{
    if (rows <= 0) return;
    const int eb = elt_bytes(dtype);
    const int64_t sb = (int64_t)ld_src * eb, db = (int64_t)ld_dst * eb, cb = (int64_t)d * eb;
    const int words = (sb % 4 == 0) && (db % 4 == 0) && (cb % 4 == 0) &&
                      ((uintptr_t)src % 4 == 0) && ((uintptr_t)dst % 4 == 0);
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s,
                       (const uint8_t*)src, sb, perm, rows, cb, (uint8_t*)dst, db,
                       dtype == DT_FP8 ? src_scales : nullptr, dtype == DT_FP8 ? dst_scales : nullptr, words);
    HIPC(hipGetLastError());
}


}  // namespace rk
