// SA-ALSH query (Alg. 2) for explicit (query, user, k) pairs, one workgroup per pair.
//
// Partitions are visited in the order of Alg. 1 (M_j descending).  For partition j:
//   mu_j = M_j ||u|| ; if phi > mu_j the answer is yes (Alg. 2, pruning test);
//   SimHash probe: the ceil(beta |S_j|) items with the most equal code bits
//     K - popcount(code_u XOR code_p) (equal counts: earlier in norm order first --
//     the reading of "K hash tables" as one K-bit code per item and of probed buckets
//     as a fraction beta of the partition), selected with a counting histogram over
//     the K+1 possible counts and an ordered scan for the ties at the cut;
//   phi = the k-th largest canonical FP64 score among all candidates so far (a radix
//     select over the scores, -inf while fewer than k);
//   if <u, q> < phi the answer is no (stop test).
// After the last partition the answer is yes.  Scores are the canonical FP64 inner
// products, so the comparisons are exact.
//
// In exact mode the stage only rejects: a "no" is proved (phi is the k-th largest
// over a subset of the items, hence <= lambda_u^(k)), a "yes" is left to the FP64
// recheck.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "index.h"
#include "internal.h"

namespace rk {

static constexpr int SQ_T = 256;

template <int DT>
__device__ double sq_dot(const void* A, int64_t ra, float sa, const void* B, int64_t rb, float sb, int d, int ld)
{
    double acc = 0.0;
    for (int i = 0; i < d; i++)
        acc = __fma_rn((double)elem_f32<DT>(A, ra * ld + i), (double)elem_f32<DT>(B, rb * ld + i), acc);
    if constexpr (DT == DT_FP8) acc = ((double)sa * (double)sb) * acc;
    return acc;
}

// k-th largest of vals[0..cnt) (orderable 64-bit keys, 8 byte-digits), by one workgroup
__device__ double block_kth(const double* vals, int64_t cnt, int k, int* hist, int* sh)
{
    const int tid = threadIdx.x;
    uint64_t prefix = 0, pmask = 0;
    int need = k;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
        for (int64_t i = tid; i < cnt; i += SQ_T) {
            const uint64_t key = f64_ord(vals[i]);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
        }
        __syncthreads();
        if (tid == 0) {
            int above = 0;
            sh[0] = 0;
            sh[1] = 0;
            for (int b = 255; b >= 0; b--) {
                if (above < need && need <= above + hist[b]) { sh[0] = b; sh[1] = above; break; }
                above += hist[b];
            }
        }
        __syncthreads();
        prefix |= (uint64_t)sh[0] << shift;
        pmask |= 0xffull << shift;
        need -= sh[1];
        __syncthreads();
    }
    return ord_f64(prefix);
}

template <int DT>
__global__ __launch_bounds__(SQ_T) void k_saalsh_query(SaQueryArgs a, double* scratch, int64_t scratch_stride)
{
    __shared__ int hist[SQ_T + 1];
    __shared__ int sh[4];
    __shared__ int wsum[SQ_T / 64];
    __shared__ int ccount;
    const int tid = threadIdx.x;
    const int W = a.K / 32;
    for (int64_t pi = blockIdx.x; pi < a.npairs; pi += gridDim.x) {
        const uint64_t key = a.pairs[pi];
        const int64_t q = (int64_t)(key >> 32), u = (int64_t)(key & 0xffffffffull);
        const int k = a.qk[q];
        double* cand = scratch + (int64_t)blockIdx.x * scratch_stride;
        const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
        const float sq = DT == DT_FP8 ? a.query_scales[q] : 1.f;
        const double suq = sq_dot<DT>(a.users, u, su, a.queries, q, sq, a.d, a.ld);
        const double unorm = sqrt(a.user_n2[u]);
        uint32_t ucode[8];
        for (int w = 0; w < W; w++) ucode[w] = a.user_codes[u * W + w];
        double phi = -__builtin_inf();
        int64_t ncand = 0;
        if (tid == 0) ccount = 0;
        __syncthreads();
        int ans = 1;
        for (int j = 0; j < a.t; j++) {
            const int64_t s0 = a.part_start[j], s1 = a.part_start[j + 1], sz = s1 - s0;
            const double mu = sqrt(a.item_n2[s0]) * unorm;
            if (phi > mu) { ans = 1; break; }
            int64_t take = (int64_t)ceil((double)a.beta * (double)sz);
            if (take > sz) take = sz;
            // histogram of collision counts over the partition
            for (int b = tid; b <= a.K; b += SQ_T) hist[b] = 0;
            __syncthreads();
            for (int64_t p = s0 + tid; p < s1; p += SQ_T) {
                int diff = 0;
                for (int w = 0; w < W; w++) diff += __popc(a.item_codes[p * W + w] ^ ucode[w]);
                atomicAdd(&hist[a.K - diff], 1);
            }
            __syncthreads();
            if (tid == 0) {   // cut count c*: #(count > c*) < take <= #(count >= c*)
                int64_t above = 0;
                int cut = 0;
                int64_t need_eq = 0;
                for (int c = a.K; c >= 0; c--) {
                    if (above + hist[c] >= take) { cut = c; need_eq = take - above; break; }
                    above += hist[c];
                }
                sh[0] = cut;
                sh[1] = (int)need_eq;
            }
            __syncthreads();
            const int cut = sh[0];
            const int need_eq = sh[1];
            // ordered pass: candidates are the items above the cut and the first need_eq at it
            int eq_before = 0;
            for (int64_t base = s0; base < s1; base += SQ_T) {
                const int64_t p = base + tid;
                int c = -1;
                if (p < s1) {
                    int diff = 0;
                    for (int w = 0; w < W; w++) diff += __popc(a.item_codes[p * W + w] ^ ucode[w]);
                    c = a.K - diff;
                }
                const int iseq = (c == cut) ? 1 : 0;
                // block-exclusive prefix of iseq in position order
                const int incl = wave_incl_scan(iseq);
                if ((tid & 63) == 63) wsum[tid >> 6] = incl;
                __syncthreads();
                int off = eq_before;
                for (int w = 0; w < (tid >> 6); w++) off += wsum[w];
                int tot = 0;
                for (int w = 0; w < SQ_T / 64; w++) tot += wsum[w];
                const int rank_eq = off + incl - iseq;
                const bool take_it = c > cut || (iseq && rank_eq < need_eq);
                __syncthreads();
                // append candidate scores (order inside the candidate multiset is irrelevant)
                if (take_it) {
                    const float sp = DT == DT_FP8 ? a.item_scales[p] : 1.f;
                    const double v = sq_dot<DT>(a.users, u, su, a.items, p, sp, a.d, a.ld);
                    cand[atomicAdd(&ccount, 1)] = v;
                }
                eq_before += tot;
            }
            __syncthreads();
            ncand = ccount;
            __syncthreads();
            phi = ncand >= k ? block_kth(cand, ncand, k, hist, sh) : -__builtin_inf();
            if (suq < phi) { ans = 0; break; }
        }
        if (tid == 0) {
            a.phi[pi] = phi;
            a.answer[pi] = ans;
        }
        __syncthreads();
    }
}

void launch_saalsh_query(const SaQueryArgs& a, double* scratch, int64_t scratch_stride, int grid, hipStream_t s)
{
    if (a.npairs <= 0) return;
    if (a.dtype == DT_F32) hipLaunchKernelGGL(k_saalsh_query<DT_F32>, dim3(grid), dim3(SQ_T), 0, s, a, scratch, scratch_stride);
    else if (a.dtype == DT_BF16) hipLaunchKernelGGL(k_saalsh_query<DT_BF16>, dim3(grid), dim3(SQ_T), 0, s, a, scratch, scratch_stride);
    else hipLaunchKernelGGL(k_saalsh_query<DT_FP8>, dim3(grid), dim3(SQ_T), 0, s, a, scratch, scratch_stride);
    HIPC(hipGetLastError());
}

}  // namespace rk
