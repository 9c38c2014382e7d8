// SA-ALSH index (Alg. 1): norm partitions of the items (sorted by descending norm),
// partition centroids c_j and radii R_j, the shifting-invariant item transform
// I(p, c_j) = [p - c_j ; sqrt(R_j^2 - ||p - c_j||^2)] (Eqn. 6) and K sign-random-
// projection bits per item (Eqn. 1).  User codes use U(u) = [R_j/||u|| u ; 0] (Eqn. 7),
// whose signs do not depend on the partition (positive factor, zero last coordinate),
// so one K-bit code per user serves every partition.
//
// The projection is a dense (rows x (d+1)) . ((d+1) x K) product on the FP32 matrix
// cores; the sign of each output is packed straight from the accumulators with one
// ballot per accumulator register (a 32x32 output block holds 32 hash bits of 32 rows).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "index.h"
#include "internal.h"

namespace rk {

// One wave finds the partition starts with a 64-ary search per partition: partition j
// starts at the first unassigned position s (M_j^2 = n2[s]) and ends at the first
// position whose n2 <= (b*b) M_j^2 (n2 is non-increasing).  A zero M_j closes the list
// with one last partition of the remaining (zero-norm) items.
__global__ void k_partitions(const double* n2, int64_t n0, int64_t n, float b, int64_t* part_start, int* num_parts)
{
    const int l = lane_id();
    const double bb = (double)b * (double)b;
    int64_t start = n0;
    int t = 0;
    while (start < n) {
        if (l == 0) part_start[t] = start;
        t++;
        const double M2 = n2[start];
        if (!(M2 > 0.0)) { start = n; break; }
        const double thr = bb * M2;
        int64_t lo = start + 1, hi = n;
        while (lo < hi) {
            const int64_t step = (hi - lo + 63) / 64;
            const int64_t pos = lo + (int64_t)l * step;
            const bool pred = pos < hi ? (n2[pos] <= thr) : true;
            const uint64_t bal = ballot64(pred);
            if (bal == 0ull) { lo = lo + 63 * step + 1; continue; }
            const int f = __builtin_ctzll(bal);
            if (f == 0) { hi = lo; break; }
            const int64_t nlo = lo + (int64_t)(f - 1) * step + 1;
            const int64_t nhi = lo + (int64_t)f * step;
            lo = nlo;
            hi = nhi < hi ? nhi : hi;
        }
        start = lo;
    }
    if (l == 0) {
        part_start[t] = n;
        *num_parts = t;
    }
}

// Centroid sums.  Each partition is cut into pieces of at most CEN_PIECE items; one
// workgroup per (piece, 64-column chunk) sums its piece with 4 interleaved row groups in
// FP64, combined in a fixed order.  A second pass gives one wave to each (partition,
// column): lane i adds the pieces i, i + 64, ... in order, the wave combines the lanes
// in a fixed shuffle tree, and the sum is divided by |S_j|.  The result does not
// depend on scheduling.
static constexpr int64_t CEN_PIECE = 256;

// Pieces are numbered partition by partition: pp[j] = first piece of partition j,
// pp[t] = number of pieces (one workgroup, scan over the partitions).
__global__ __launch_bounds__(1024) void k_pieces(const int64_t* part_start, const int* num_parts, int64_t* pp)
{
    __shared__ int64_t wtot[16];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    const int t = *num_parts;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int c0 = 0; c0 < t; c0 += 1024) {
        const int j = c0 + tid;
        const int64_t c = j < t ? (part_start[j + 1] - part_start[j] + CEN_PIECE - 1) / CEN_PIECE : 0;
        int64_t incl = c;   // wave inclusive scan (64-bit)
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(incl, o);
            if (l >= o) incl += y;
        }
        if (l == 63) wtot[w] = incl;
        __syncthreads();
        int64_t off = carry_s;
        for (int q = 0; q < w; q++) off += wtot[q];
        if (j < t) pp[j] = off + incl - c;
        __syncthreads();
        if (tid == 0) {
            int64_t s = 0;
            for (int q = 0; q < 16; q++) s += wtot[q];
            carry_s += s;
        }
        __syncthreads();
    }
    if (tid == 0) pp[t] = carry_s;
}

template <int DT>
__global__ __launch_bounds__(256) void k_centroid_piece(const void* X, const float* scales, const int64_t* part_start,
                                                        const int* num_parts, const int64_t* pp, int d, int ld,
                                                        double* psum)
{
    __shared__ double part[4][64];
    const int t = *num_parts;
    const int64_t pc = blockIdx.x;
    if (pc >= pp[t]) return;   // grid sized for the most pieces any partitioning can give
    int lo = 0, hi = t - 1;    // partition of the piece: largest j with pp[j] <= pc
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pp[mid] <= pc) lo = mid;
        else hi = mid - 1;
    }
    const int64_t s0 = part_start[lo] + (pc - pp[lo]) * CEN_PIECE;
    const int64_t s1 = s0 + CEN_PIECE < part_start[lo + 1] ? s0 + CEN_PIECE : part_start[lo + 1];
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    double acc = 0.0;
    if (c < d) {
#pragma unroll 8
        for (int64_t p = s0 + g; p < s1; p += 4) {
            double v = (double)elem_f32<DT>(X, p * ld + c);
            if constexpr (DT == DT_FP8) v *= (double)scales[p];
            acc += v;
        }
    }
    part[g][threadIdx.x & 63] = acc;
    __syncthreads();
    if (g == 0 && c < ld)
        psum[pc * ld + c] = ((part[0][c & 63] + part[1][c & 63]) + part[2][c & 63]) + part[3][c & 63];
}

__global__ __launch_bounds__(256) void k_centroid_final(const double* psum, const int64_t* part_piece,
                                                        const int64_t* part_start, int t, int d, int ld,
                                                        double* cen64, float* cen32)
{
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // (partition, column)
    if (e >= (int64_t)t * ld) return;
    const int l = lane_id();
    const int j = (int)(e / ld), c = (int)(e % ld);
    double v = 0.0;
    if (c < d) {
        for (int64_t pc = part_piece[j] + l; pc < part_piece[j + 1]; pc += 64) v += psum[pc * ld + c];
        v = wave_sum(v);
        v /= (double)(part_start[j + 1] - part_start[j]);
    }
    if (l == 0) {
        cen64[e] = v;
        cen32[e] = (float)v;
    }
}

// r2[p] = ||p - c_j||^2 (FP64) and the partition radius as max (atomicMax on the bits
// of a non-negative double is order-independent).
template <int DT>
__global__ void k_radius(const void* X, const float* scales, const int64_t* part_start, int t, int64_t n, int d,
                         int ld, const double* cen64, double* r2out, unsigned long long* rad2_bits)
{
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p0 < n;
    const int64_t p = in ? p0 : n - 1;   // out-of-range lanes repeat the last item (max is unchanged)
    int lo = 0, hi = t - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (part_start[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    const double* c = cen64 + (int64_t)lo * ld;
    const double sc = DT == DT_FP8 ? (double)scales[p] : 1.0;
    // the lane's row in 16-byte loads (rows are 16-byte aligned: ld >= 32), the terms in
    // index order
    constexpr int VPL = 16 / Elt<DT>::bytes;
    const uint8_t* row = (const uint8_t*)X + p * ld * Elt<DT>::bytes;
    double r2 = 0.0;
    for (int i0 = 0; i0 < d; i0 += VPL) {
        const i32x4 q = *(const i32x4*)(row + i0 * Elt<DT>::bytes);
#pragma unroll
        for (int e = 0; e < VPL; e++) {
            if (i0 + e < d) {
                const double v = (double)elem_f32<DT>(&q, e) * sc - c[i0 + e];
                r2 = __fma_rn(v, v, r2);
            }
        }
    }
    if (p < part_start[0]) r2 = 0.0;   // SAH: P' items belong to no partition
    if (in) r2out[p] = r2;
    // partitions are contiguous ranges: reduce inside the wave, one atomic per partition
    uint64_t rem = ballot64(true);
    while (rem) {
        const int leader = __builtin_ctzll(rem);
        const int j0 = __shfl(lo, leader);
        const bool mine = lo == j0;
        rem &= ~ballot64(mine);
        const double mx = wave_max(mine ? r2 : 0.0);
        if (lane_id() == leader) atomicMax(&rad2_bits[j0], (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void k_radius_final(const unsigned long long* rad2_bits, int t, float* radius, double* rad2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= t) return;
    const double r2 = __longlong_as_double((long long)rad2_bits[j]);
    rad2[j] = r2;
    radius[j] = (float)sqrt(r2);
}

// Projection + sign packing.  MODE 0: item rows with the SAT transform of their
// partition; MODE 1: raw user rows.  A workgroup takes 128 rows (32 per wave) and all K
// hash columns; the transformed rows and the projection matrix pass through LDS in
// chunks of 32 dimensions.
static constexpr int PJ_KC = 32;

template <int DT, int MODE, int KB>
__global__ __launch_bounds__(256) void k_project(const void* X, const float* scales, int64_t rows, int d, int ld,
                                                 const int64_t* part_start, int t, const float* cen32,
                                                 const double* r2, const double* rad2, const float* A, int K,
                                                 uint32_t* codes)
{
    __shared__ float xs[128][PJ_KC + 1];
    __shared__ float as[PJ_KC][KB * 32];
    __shared__ int pj[128];
    const int l = lane_id(), w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 128;
    const int D = MODE == 0 ? d + 1 : d;
    if (MODE == 0 && threadIdx.x < 128) {
        const int64_t p = r0 + threadIdx.x;
        int lo = 0, hi = t - 1;
        if (p < rows)
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (part_start[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
        pj[threadIdx.x] = lo;
    }
    __syncthreads();   // pj is read before the first tile store
    f32x16 acc[KB];
#pragma unroll
    for (int cb = 0; cb < KB; cb++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[cb][r] = 0.f;
    // Chunk k0 + PJ_KC is loaded from global memory while the products of chunk k0 run.
    // Thread map: row rr, the XE consecutive values from column kb of the chunk, read in
    // 16-byte loads where they lie inside the padded row.
    constexpr int XE = 128 * PJ_KC / 256, AE = PJ_KC * KB * 32 / 256;
    static_assert(XE == 16 && PJ_KC == 32, "chunk map: two threads per row");
    const int rr = threadIdx.x >> 1, kb = (threadIdx.x & 1) * XE;
    const int64_t p = r0 + rr;
    i32x4 raw[Elt<DT>::bytes];
    float av[AE];
    auto fetch = [&](int k0) {
        const bool vec = p < rows && k0 + kb + XE <= ld && k0 + kb < d;
#pragma unroll
        for (int j = 0; j < Elt<DT>::bytes; j++) {
            raw[j] = i32x4{0, 0, 0, 0};
            if (vec) raw[j] = *(const i32x4*)((const uint8_t*)X + (p * ld + k0 + kb) * Elt<DT>::bytes + 16 * j);
        }
#pragma unroll
        for (int q = 0; q < AE; q++) {
            const int e = threadIdx.x + 256 * q;
            const int kk = e / (KB * 32), h = e % (KB * 32);
            const int i = k0 + kk;
            av[q] = (i < D && h < K) ? A[(int64_t)i * K + h] : 0.f;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < D; k0 += PJ_KC) {
        float xv[XE];
#pragma unroll
        for (int q = 0; q < XE; q++) {
            const int i = k0 + kb + q;
            float v = 0.f;
            if (p < rows) {
                if (i < d) {
                    float x = elem_f32<DT>(raw, q);
                    if constexpr (DT == DT_FP8) x *= scales[p];
                    if (MODE == 0) x -= cen32[(int64_t)pj[rr] * ld + i];
                    v = x;
                } else if (MODE == 0 && i == d) {
                    const double rest = rad2[pj[rr]] - r2[p];
                    v = rest > 0.0 ? (float)sqrt(rest) : 0.f;
                }
            }
            xv[q] = v;
        }
        __syncthreads();   // the previous chunk's products have read the LDS tiles
#pragma unroll
        for (int q = 0; q < XE; q++) xs[rr][kb + q] = xv[q];
#pragma unroll
        for (int q = 0; q < AE; q++) {
            const int e = threadIdx.x + 256 * q;
            as[e / (KB * 32)][e % (KB * 32)] = av[q];
        }
        __syncthreads();
        if (k0 + PJ_KC < D) fetch(k0 + PJ_KC);
#pragma unroll
        for (int kk = 0; kk < PJ_KC; kk += 2) {
            const float a = xs[w * 32 + (l & 31)][kk + (l >> 5)];
#pragma unroll
            for (int cb = 0; cb < KB; cb++)
                acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, as[kk + (l >> 5)][cb * 32 + (l & 31)], acc[cb], 0, 0, 0);
        }
    }
    const int W = K / 32;
#pragma unroll
    for (int cb = 0; cb < KB; cb++)
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const uint64_t bal = ballot64(acc[cb][r] >= 0.f);
            const int row_lo = w * 32 + mfma32_row(r, 0);   // lanes 0..31
            const int row_hi = w * 32 + mfma32_row(r, 32);  // lanes 32..63
            if (l == 0 && cb < W) {
                if (r0 + row_lo < rows) codes[(r0 + row_lo) * W + cb] = (uint32_t)bal;
                if (r0 + row_hi < rows) codes[(r0 + row_hi) * W + cb] = (uint32_t)(bal >> 32);
            }
        }
}

template <int DT, int MODE>
static void project_dispatch(int K, dim3 g, hipStream_t s, const void* X, const float* sc, int64_t rows, int d,
                             int ld, const int64_t* ps, int t, const float* cen32, const double* r2,
                             const double* rad2, const float* A, uint32_t* codes)
{
    const int kb = K / 32;
    if (kb <= 4) hipLaunchKernelGGL((k_project<DT, MODE, 4>), g, dim3(256), 0, s, X, sc, rows, d, ld, ps, t, cen32, r2, rad2, A, K, codes);
    else hipLaunchKernelGGL((k_project<DT, MODE, 8>), g, dim3(256), 0, s, X, sc, rows, d, ld, ps, t, cen32, r2, rad2, A, K, codes);
}

template <int MODE>
static void project(int dtype, int K, const void* X, const float* sc, int64_t rows, int d, int ld,
                    const int64_t* ps, int t, const float* cen32, const double* r2, const double* rad2,
                    const float* A, uint32_t* codes, hipStream_t s)
{
    if (rows <= 0) return;
    dim3 g((unsigned)((rows + 127) / 128));
    if (dtype == DT_F32) project_dispatch<DT_F32, MODE>(K, g, s, X, sc, rows, d, ld, ps, t, cen32, r2, rad2, A, codes);
    else if (dtype == DT_BF16) project_dispatch<DT_BF16, MODE>(K, g, s, X, sc, rows, d, ld, ps, t, cen32, r2, rad2, A, codes);
    else project_dispatch<DT_FP8, MODE>(K, g, s, X, sc, rows, d, ld, ps, t, cen32, r2, rad2, A, codes);
    HIPC(hipGetLastError());
}

// Counter-based Gaussian entries (Box-Muller over SplitMix64) for a library-drawn
// projection matrix.
__global__ void k_gen_srp(float* A, int64_t count, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t a = splitmix64(seed ^ splitmix64(2 * (uint64_t)i + 0x5A17ull));
    const uint64_t b = splitmix64(seed ^ splitmix64(2 * (uint64_t)i + 0x5A18ull));
    const double u1 = ((double)(a >> 11) + 1.0) * 0x1p-53;   // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1p-53;
    A[i] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

// Partition starts of the norm-sorted items; the partition count reaches the host at the
// build's next synchronisation (h_num_parts).
void start_partitions(Index& x, int* h_num_parts, hipStream_t s)
{
    x.part_start.alloc(sizeof(int64_t) * (x.n + 2));
    x.num_parts.alloc(sizeof(int));
    // exact mode: all of P; SAH mode: P minus P' (the first n_lam positions), Alg. 4
    const int64_t n0 = x.prm.mode != RKMIPS_MODE_EXACT ? x.n_lam : 0;
    hipLaunchKernelGGL(k_partitions, dim3(1), dim3(64), 0, s, x.item_n2.d(), n0, x.n, x.prm.b, x.part_start.i64(),
                       x.num_parts.i());
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(h_num_parts, x.num_parts.p, sizeof(int), hipMemcpyDeviceToHost, s));
}

// The rest of Alg. 1 once x.t is known; stream-ordered, no host synchronisation.
// Random projections of the transformed vectors: the caller's, or drawn from the seed.
void saalsh_projections(Index& x, const float* srp, hipStream_t s)
{
    const int K = x.prm.num_hash;
    x.srp.alloc(sizeof(float) * (size_t)(x.d + 1) * K);
    if (srp) HIPC(hipMemcpyAsync(x.srp.p, srp, sizeof(float) * (size_t)(x.d + 1) * K, hipMemcpyDeviceToDevice, s));
    else {
        const int64_t cnt = (int64_t)(x.d + 1) * K;
        hipLaunchKernelGGL(k_gen_srp, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, x.srp.f(), cnt,
                           x.prm.seed ^ 0x53525031ull);
        HIPC(hipGetLastError());
    }
}

// Item side: partition centroids and radii, then the item codes.
void saalsh_items(Index& x, hipStream_t s)
{
    const int K = x.prm.num_hash, W = K / 32;
    const int64_t n = x.n;
    const int t = x.t;
    // centroids and radii
    DevBuf cen64, r2, rad2bits, rad2;
    cen64.alloc(sizeof(double) * (size_t)t * x.ld);
    x.centroid.alloc(sizeof(float) * (size_t)t * x.ld);
    x.radius.alloc(sizeof(float) * t);
    r2.alloc(sizeof(double) * n);
    rad2bits.alloc(sizeof(unsigned long long) * t);
    rad2.alloc(sizeof(double) * t);
    HIPC(hipMemsetAsync(rad2bits.p, 0, sizeof(unsigned long long) * t, s));
    {
        const int64_t max_pieces = (n + CEN_PIECE - 1) / CEN_PIECE + t;
        DevBuf d_pp, psum;
        d_pp.alloc(sizeof(int64_t) * (t + 1));
        psum.alloc(sizeof(double) * (size_t)max_pieces * x.ld);
        hipLaunchKernelGGL(k_pieces, dim3(1), dim3(1024), 0, s, x.part_start.i64(), (const int*)x.num_parts.i(), d_pp.i64());
        dim3 g((unsigned)max_pieces, (unsigned)((x.ld + 63) / 64));
        const int* npp = x.num_parts.i();
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_centroid_piece<DT_F32>, g, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), npp, d_pp.i64(), x.d, x.ld, psum.d());
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_centroid_piece<DT_BF16>, g, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), npp, d_pp.i64(), x.d, x.ld, psum.d());
        else hipLaunchKernelGGL(k_centroid_piece<DT_FP8>, g, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), npp, d_pp.i64(), x.d, x.ld, psum.d());
        const int64_t tot = (int64_t)t * x.ld;
        hipLaunchKernelGGL(k_centroid_final, dim3((unsigned)((tot + 3) / 4)), dim3(256), 0, s, psum.d(),
                           d_pp.i64(), x.part_start.i64(), t, x.d, x.ld, cen64.d(), x.centroid.f());
        HIPC(hipGetLastError());
        dim3 g2((unsigned)((n + 255) / 256));
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_radius<DT_F32>, g2, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), t, n, x.d, x.ld, cen64.d(), r2.d(), (unsigned long long*)rad2bits.p);
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_radius<DT_BF16>, g2, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), t, n, x.d, x.ld, cen64.d(), r2.d(), (unsigned long long*)rad2bits.p);
        else hipLaunchKernelGGL(k_radius<DT_FP8>, g2, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), t, n, x.d, x.ld, cen64.d(), r2.d(), (unsigned long long*)rad2bits.p);
        hipLaunchKernelGGL(k_radius_final, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s,
                           (const unsigned long long*)rad2bits.p, t, x.radius.f(), rad2.d());
        HIPC(hipGetLastError());
    }
    x.item_codes.alloc(sizeof(uint32_t) * (size_t)n * W);
    project<0>(x.dtype, K, x.items.p, x.item_scales.f(), n, x.d, x.ld, x.part_start.i64(), t, x.centroid.f(), r2.d(),
               rad2.d(), x.srp.f(), x.item_codes.u32(), s);
}

// User codes, users in leaf order.
void saalsh_users(Index& x, hipStream_t s)
{
    const int K = x.prm.num_hash, W = K / 32;
    x.user_codes.alloc(sizeof(uint32_t) * (size_t)x.m * W);
    project<1>(x.dtype, K, x.users.p, x.user_scales.f(), x.m, x.d, x.ld, nullptr, 1, nullptr, nullptr, nullptr,
               x.srp.f(), x.user_codes.u32(), s);
}

}  // namespace rk
