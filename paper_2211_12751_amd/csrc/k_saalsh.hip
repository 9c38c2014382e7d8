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
__global__ void k_partitions(const double* n2, int64_t n, float b, int64_t* part_start, int* num_parts)
{
    const int l = lane_id();
    const double bb = (double)b * (double)b;
    int64_t start = 0;
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
// FP64, combined in a fixed order; a second pass adds the pieces of a partition in
// order and divides by |S_j|.  The result does not depend on scheduling.
static constexpr int64_t CEN_PIECE = 2048;

template <int DT>
__global__ __launch_bounds__(256) void k_centroid_piece(const void* X, const float* scales, const int64_t* pc_begin,
                                                        const int64_t* pc_end, int d, int ld, double* psum)
{
    __shared__ double part[4][64];
    const int pc = blockIdx.x;
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    const int64_t s0 = pc_begin[pc], s1 = pc_end[pc];
    double acc = 0.0;
    if (c < d)
        for (int64_t p = s0 + g; p < s1; p += 4) {
            double v = (double)elem_f32<DT>(X, p * ld + c);
            if constexpr (DT == DT_FP8) v *= (double)scales[p];
            acc += v;
        }
    part[g][threadIdx.x & 63] = acc;
    __syncthreads();
    if (g == 0 && c < ld)
        psum[(int64_t)pc * ld + c] = ((part[0][c & 63] + part[1][c & 63]) + part[2][c & 63]) + part[3][c & 63];
}

__global__ void k_centroid_final(const double* psum, const int64_t* part_piece, const int64_t* part_start, int t,
                                 int d, int ld, double* cen64, float* cen32)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)t * ld) return;
    const int j = (int)(e / ld), c = (int)(e % ld);
    double v = 0.0;
    if (c < d) {
        for (int64_t pc = part_piece[j]; pc < part_piece[j + 1]; pc++) v += psum[pc * ld + c];
        v /= (double)(part_start[j + 1] - part_start[j]);
    }
    cen64[e] = v;
    cen32[e] = (float)v;
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
    double r2 = 0.0;
    for (int i = 0; i < d; i++) {
        const double v = (double)elem_f32<DT>(X, p * ld + i) * sc - c[i];
        r2 = __fma_rn(v, v, r2);
    }
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
    f32x16 acc[KB];
#pragma unroll
    for (int cb = 0; cb < KB; cb++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[cb][r] = 0.f;
    for (int k0 = 0; k0 < D; k0 += PJ_KC) {
        __syncthreads();
        for (int e = threadIdx.x; e < 128 * PJ_KC; e += 256) {
            const int rr = e / PJ_KC, kk = e % PJ_KC;
            const int64_t p = r0 + rr;
            const int i = k0 + kk;
            float v = 0.f;
            if (p < rows) {
                if (i < d) {
                    float x = elem_f32<DT>(X, p * ld + i);
                    if constexpr (DT == DT_FP8) x *= scales[p];
                    if (MODE == 0) x -= cen32[(int64_t)pj[rr] * ld + i];
                    v = x;
                } else if (MODE == 0 && i == d) {
                    const double rest = rad2[pj[rr]] - r2[p];
                    v = rest > 0.0 ? (float)sqrt(rest) : 0.f;
                }
            }
            xs[rr][kk] = v;
        }
        for (int e = threadIdx.x; e < PJ_KC * KB * 32; e += 256) {
            const int kk = e / (KB * 32), h = e % (KB * 32);
            const int i = k0 + kk;
            as[kk][h] = (i < D && h < K) ? A[(int64_t)i * K + h] : 0.f;
        }
        __syncthreads();
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

void build_saalsh(Index& x, const float* srp, hipStream_t s)
{
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    HIPC(hipEventRecord(e0, s));
    const int K = x.prm.num_hash, W = K / 32;
    const int64_t n = x.n;
    x.srp.alloc(sizeof(float) * (size_t)(x.d + 1) * K);
    if (srp) HIPC(hipMemcpyAsync(x.srp.p, srp, sizeof(float) * (size_t)(x.d + 1) * K, hipMemcpyDeviceToDevice, s));
    else {
        const int64_t cnt = (int64_t)(x.d + 1) * K;
        hipLaunchKernelGGL(k_gen_srp, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, x.srp.f(), cnt,
                           x.prm.seed ^ 0x53525031ull);
    }
    // partitions
    DevBuf ps, np;
    ps.alloc(sizeof(int64_t) * (n + 2));
    np.alloc(sizeof(int));
    hipLaunchKernelGGL(k_partitions, dim3(1), dim3(64), 0, s, x.item_n2.d(), n, x.prm.b, ps.i64(), np.i());
    HIPC(hipGetLastError());
    int t = 0;
    HIPC(hipMemcpyAsync(&t, np.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    x.t = t;
    x.part_start_h.resize(t + 1);
    HIPC(hipMemcpy(x.part_start_h.data(), ps.p, sizeof(int64_t) * (t + 1), hipMemcpyDeviceToHost));
    x.part_start.alloc(sizeof(int64_t) * (t + 1));
    HIPC(hipMemcpyAsync(x.part_start.p, x.part_start_h.data(), sizeof(int64_t) * (t + 1), hipMemcpyHostToDevice, s));
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
        // pieces of each partition
        std::vector<int64_t> pb, pe, pp(t + 1, 0);
        for (int j = 0; j < t; j++) {
            pp[j] = (int64_t)pb.size();
            for (int64_t b0 = x.part_start_h[j]; b0 < x.part_start_h[j + 1]; b0 += CEN_PIECE) {
                pb.push_back(b0);
                pe.push_back(std::min(b0 + CEN_PIECE, x.part_start_h[j + 1]));
            }
        }
        pp[t] = (int64_t)pb.size();
        const int64_t np_ = (int64_t)pb.size();
        DevBuf d_pb, d_pe, d_pp, psum;
        d_pb.alloc(sizeof(int64_t) * np_);
        d_pe.alloc(sizeof(int64_t) * np_);
        d_pp.alloc(sizeof(int64_t) * (t + 1));
        psum.alloc(sizeof(double) * (size_t)np_ * x.ld);
        HIPC(hipMemcpyAsync(d_pb.p, pb.data(), sizeof(int64_t) * np_, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(d_pe.p, pe.data(), sizeof(int64_t) * np_, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(d_pp.p, pp.data(), sizeof(int64_t) * (t + 1), hipMemcpyHostToDevice, s));
        dim3 g((unsigned)np_, (unsigned)((x.ld + 63) / 64));
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_centroid_piece<DT_F32>, g, dim3(256), 0, s, x.items.p, x.item_scales.f(), d_pb.i64(), d_pe.i64(), x.d, x.ld, psum.d());
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_centroid_piece<DT_BF16>, g, dim3(256), 0, s, x.items.p, x.item_scales.f(), d_pb.i64(), d_pe.i64(), x.d, x.ld, psum.d());
        else hipLaunchKernelGGL(k_centroid_piece<DT_FP8>, g, dim3(256), 0, s, x.items.p, x.item_scales.f(), d_pb.i64(), d_pe.i64(), x.d, x.ld, psum.d());
        const int64_t tot = (int64_t)t * x.ld;
        hipLaunchKernelGGL(k_centroid_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, psum.d(),
                           d_pp.i64(), x.part_start.i64(), t, x.d, x.ld, cen64.d(), x.centroid.f());
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(s));   // host piece tables go out of scope
        dim3 g2((unsigned)((n + 255) / 256));
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_radius<DT_F32>, g2, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), t, n, x.d, x.ld, cen64.d(), r2.d(), (unsigned long long*)rad2bits.p);
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_radius<DT_BF16>, g2, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), t, n, x.d, x.ld, cen64.d(), r2.d(), (unsigned long long*)rad2bits.p);
        else hipLaunchKernelGGL(k_radius<DT_FP8>, g2, dim3(256), 0, s, x.items.p, x.item_scales.f(), x.part_start.i64(), t, n, x.d, x.ld, cen64.d(), r2.d(), (unsigned long long*)rad2bits.p);
        hipLaunchKernelGGL(k_radius_final, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s,
                           (const unsigned long long*)rad2bits.p, t, x.radius.f(), rad2.d());
        HIPC(hipGetLastError());
    }
    x.item_codes.alloc(sizeof(uint32_t) * (size_t)n * W);
    x.user_codes.alloc(sizeof(uint32_t) * (size_t)x.m * W);
    project<0>(x.dtype, K, x.items.p, x.item_scales.f(), n, x.d, x.ld, x.part_start.i64(), t, x.centroid.f(), r2.d(),
               rad2.d(), x.srp.f(), x.item_codes.u32(), s);
    project<1>(x.dtype, K, x.users.p, x.user_scales.f(), x.m, x.d, x.ld, nullptr, 1, nullptr, nullptr, nullptr,
               x.srp.f(), x.user_codes.u32(), s);
    HIPC(hipEventRecord(e1, s));
    HIPC(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    x.ms_saalsh = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace rk
