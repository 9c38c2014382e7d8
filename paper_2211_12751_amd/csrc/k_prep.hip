// Input preparation: validation + canonical squared norms, the norm order of the
// items (Alg. 4 / Alg. 1: sort by descending norm), row gathers into padded copies,
// unit user directions for the Cone-Tree (Fact 2: only directions matter), and a
// bitonic sort used for the item order and for the per-query result lists.
#include "common.h"
#include "internal.h"

namespace rk {

// ------------------------------------------------------------------ norms + validation
// Canonical squared norm of every row (index-order FP64 sum of the exact squares; FP8:
// times the squared scale), plus what validation needs: stats[slot] = max n2 (bits of a
// non-negative double order like the value), stats[2] = min positive n2, stats[3] = 1
// on any non-finite value, NaN code or non-finite scale.
template <int DT>
__global__ void k_norm2(const void* X, const float* scales, int64_t rows, int d, int ld, double* n2,
                        unsigned long long* stats, int slot)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = true;
    double acc = 0.0;
    if (r < rows) {
        const int64_t o = r * ld;
        for (int i = 0; i < d; i++) {
            if constexpr (DT == DT_F32) {
                float v = ((const float*)X)[o + i];
                ok &= (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
                acc = __fma_rn((double)v, (double)v, acc);
            } else if constexpr (DT == DT_BF16) {
                uint16_t b = ((const uint16_t*)X)[o + i];
                ok &= (b & 0x7f80u) != 0x7f80u;
                double v = (double)bf16_to_f32(b);
                acc = __fma_rn(v, v, acc);
            } else {
                uint8_t c = ((const uint8_t*)X)[o + i];
                ok &= (c & 0x7fu) != 0x7fu;
                double v = (double)e4m3_to_f32(c);
                acc = __fma_rn(v, v, acc);
            }
        }
        if constexpr (DT == DT_FP8) {
            float s = scales[r];
            ok &= (__float_as_uint(s) & 0x7f800000u) != 0x7f800000u;
            acc = ((double)s * (double)s) * acc;
        }
        n2[r] = acc;
    }
    const unsigned long long bits = (unsigned long long)__double_as_longlong(acc);
    const unsigned long long mx = wave_max((r < rows && ok) ? bits : 0ull);
    const unsigned long long mn = wave_min((r < rows && ok && acc > 0.0) ? bits : ~0ull);
    const bool any_bad = ballot64(r < rows && !ok) != 0ull;
    if (lane_id() == 0) {
        if (mx) atomicMax(&stats[slot], mx);
        if (mn != ~0ull) atomicMin(&stats[2], mn);
        if (any_bad) atomicOr(&stats[3], 1ull);
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
    if (dtype == DT_F32) hipLaunchKernelGGL(k_norm2<DT_F32>, g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_norm2<DT_BF16>, g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
    else hipLaunchKernelGGL(k_norm2<DT_FP8>, g, b, 0, s, X, scales, rows, d, ld, n2, stats, slot);
    HIPC(hipGetLastError());
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

// ------------------------------------------------------------------ bitonic sort
// Ascending by (key, val).  Chunk-local stages run in LDS; longer strides in global.
static constexpr int SORT_THREADS = 256;
static constexpr int SORT_CHUNK = 2048;  // elements per workgroup in the LDS stages

template <bool HV>
__device__ __forceinline__ bool gt_pair(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb)
{
    if constexpr (HV) return ka > kb || (ka == kb && va > vb);
    else return ka > kb;
}

// Stages (k, j) for k in [k_lo, k_hi] (k doubling) and j from min(k/2, chunk/2) to 1,
// all inside one chunk of `chunk` elements.
template <bool HV>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_local(uint64_t* keys, uint32_t* vals,
                                                               int chunk, int64_t k_lo, int64_t k_hi)
{
    __shared__ uint64_t sk[SORT_CHUNK];
    __shared__ uint32_t sv[HV ? SORT_CHUNK : 1];
    const int64_t base = (int64_t)blockIdx.x * chunk;
    for (int i = threadIdx.x; i < chunk; i += SORT_THREADS) {
        sk[i] = keys[base + i];
        if constexpr (HV) sv[i] = vals[base + i];
    }
    __syncthreads();
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (k >> 1) < (chunk >> 1) ? (k >> 1) : (chunk >> 1); j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (chunk >> 1); t += SORT_THREADS) {
                int i = (int)(2 * j * (t / j) + (t % j));
                int p = i + (int)j;
                bool asc = (((base + i) & k) == 0);
                uint64_t ka = sk[i], kb = sk[p];
                uint32_t va = 0, vb = 0;
                if constexpr (HV) { va = sv[i]; vb = sv[p]; }
                bool sw = asc ? gt_pair<HV>(ka, va, kb, vb) : gt_pair<HV>(kb, vb, ka, va);
                if (sw) {
                    sk[i] = kb; sk[p] = ka;
                    if constexpr (HV) { sv[i] = vb; sv[p] = va; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < chunk; i += SORT_THREADS) {
        keys[base + i] = sk[i];
        if constexpr (HV) vals[base + i] = sv[i];
    }
}

template <bool HV>
__global__ void k_sort_global(uint64_t* keys, uint32_t* vals, int64_t npairs, int64_t k, int64_t j)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npairs) return;
    int64_t i = 2 * j * (t / j) + (t % j);
    int64_t p = i + j;
    bool asc = ((i & k) == 0);
    uint64_t ka = keys[i], kb = keys[p];
    uint32_t va = 0, vb = 0;
    if constexpr (HV) { va = vals[i]; vb = vals[p]; }
    bool sw = asc ? gt_pair<HV>(ka, va, kb, vb) : gt_pair<HV>(kb, vb, ka, va);
    if (sw) {
        keys[i] = kb; keys[p] = ka;
        if constexpr (HV) { vals[i] = vb; vals[p] = va; }
    }
}

__global__ void k_fill_pad(uint64_t* keys, uint32_t* vals, int64_t n, int64_t cap)
{
    int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    keys[i] = ~0ull;
    if (vals) vals[i] = 0xffffffffu;
}

static int64_t pow2ceil(int64_t n)
{
    int64_t p = 2;
    while (p < n) p <<= 1;
    return p;
}

template <bool HV>
static void bitonic(uint64_t* keys, uint32_t* vals, int64_t n, int64_t cap, hipStream_t s)
{
    if (n <= 1) return;
    const int64_t P = pow2ceil(n);
    if (cap < P) fail(RKMIPS_EINVAL, "internal: sort capacity below the padded size");
    if (P > n)
        hipLaunchKernelGGL(k_fill_pad, dim3((unsigned)((P - n + 255) / 256)), dim3(256), 0, s, keys,
                           HV ? vals : nullptr, n, P);
    const int chunk = (int)(P < SORT_CHUNK ? P : SORT_CHUNK);
    const unsigned nch = (unsigned)(P / chunk);
    hipLaunchKernelGGL(k_sort_local<HV>, dim3(nch), dim3(SORT_THREADS), 0, s, keys, vals, chunk,
                       (int64_t)2, (int64_t)chunk);
    for (int64_t k = (int64_t)chunk * 2; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j >= chunk; j >>= 1)
            hipLaunchKernelGGL(k_sort_global<HV>, dim3((unsigned)((P / 2 + 255) / 256)), dim3(256), 0, s,
                               keys, vals, P / 2, k, j);
        hipLaunchKernelGGL(k_sort_local<HV>, dim3(nch), dim3(SORT_THREADS), 0, s, keys, vals, chunk, k, k);
    }
    HIPC(hipGetLastError());
}

void sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int64_t cap, hipStream_t s)
{
    bitonic<true>(keys, vals, n, cap, s);
}
void sort_keys(uint64_t* keys, int64_t n, int64_t cap, hipStream_t s) { bitonic<false>(keys, nullptr, n, cap, s); }

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

// ------------------------------------------------------------------ unit rows
template <int DT>
__global__ void k_unit_rows(const void* X, const float* scales, const double* n2, int64_t rows, int d,
                            int ld, float* out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * ld) return;
    int64_t r = t / ld;
    int i = (int)(t - r * ld);
    float v = 0.f;
    if (i < d && n2[r] > 0.0) {
        double x = (double)elem_f32<DT>(X, r * ld + i);
        if constexpr (DT == DT_FP8) x *= (double)scales[r];
        v = (float)(x / sqrt(n2[r]));
    }
    out[t] = v;
}

void launch_unit_rows(int dtype, const void* X, const float* scales, const double* n2, int64_t rows,
                      int d, int ld, float* out, hipStream_t s)
{
    if (rows <= 0) return;
    const int64_t tot = rows * ld;
    dim3 g((unsigned)((tot + 255) / 256)), b(256);
    if (dtype == DT_F32) hipLaunchKernelGGL(k_unit_rows<DT_F32>, g, b, 0, s, X, scales, n2, rows, d, ld, out);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_unit_rows<DT_BF16>, g, b, 0, s, X, scales, n2, rows, d, ld, out);
    else hipLaunchKernelGGL(k_unit_rows<DT_FP8>, g, b, 0, s, X, scales, n2, rows, d, ld, out);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ exclusive scan (int32)
// Three phases: per-block sums, a single-block scan of the sums, then the add-back.
static constexpr int SCAN_B = 1024;

__global__ __launch_bounds__(256) void k_scan_blocks(const int* in, int* out, int64_t n, int* sums)
{
    __shared__ int ws[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B;
    int v[4], loc = 0;
    for (int e = 0; e < 4; e++) {
        int64_t i = base + threadIdx.x * 4 + e;
        v[e] = i < n ? in[i] : 0;
        loc += v[e];
    }
    int inc = wave_incl_scan(loc);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) ws[w] = inc;
    __syncthreads();
    int off = 0;
    for (int q = 0; q < w; q++) off += ws[q];
    int run = off + inc - loc;
    for (int e = 0; e < 4; e++) {
        int64_t i = base + threadIdx.x * 4 + e;
        if (i < n) out[i] = run;
        run += v[e];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = off + inc;
}

__global__ __launch_bounds__(256) void k_scan_sums(int* sums, int64_t nb)
{
    __shared__ int ws[4];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        int64_t i = b0 + threadIdx.x;
        int v = i < nb ? sums[i] : 0;
        int inc = wave_incl_scan(v);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 63) ws[w] = inc;
        __syncthreads();
        int off = carry;
        for (int q = 0; q < w; q++) off += ws[q];
        if (i < nb) sums[i] = off + inc - v;
        __syncthreads();
        if (threadIdx.x == 255) carry = off + inc;
        __syncthreads();
    }
}

__global__ void k_scan_add(int* out, int64_t n, const int* sums)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += sums[i / SCAN_B];
}

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_B - 1) / SCAN_B + 1; }

void exclusive_scan_i32(const int* in, int* out, int64_t n, int* tmp, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, in, out, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, tmp);
    HIPC(hipGetLastError());
}

}  // namespace rk
