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
// recheck.  In SAH mode (Alg. 5) the partitions cover P minus P', the candidate set
// starts from u's scores on P' (phi = L_u^k), and the answer is final.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "index.h"
#include "internal.h"

namespace rk {

static constexpr int SQ_T = 256;

// Canonical FP64 inner product of two stored rows (index-order sum of the exact
// products; FP8: exact code sum times the scale product), 16-byte loads.
template <int DT>
__device__ double sq_dot(const void* A, int64_t ra, float sa, const void* B, int64_t rb, float sb, int d, int ld)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int PER = 16 / EB;
    const uint8_t* ar = (const uint8_t*)A + ra * (int64_t)ld * EB;
    const uint8_t* br = (const uint8_t*)B + rb * (int64_t)ld * EB;
    double acc = 0.0;
    for (int c0 = 0; c0 < d; c0 += PER) {
        const i32x4 x4 = *(const i32x4*)(ar + c0 * EB);
        const i32x4 y4 = *(const i32x4*)(br + c0 * EB);
        const int lim = d - c0 < PER ? d - c0 : PER;
#pragma unroll
        for (int e = 0; e < PER; e++) {
            if (e >= lim) break;
            float x, y;
            if constexpr (DT == DT_F32) {
                x = __int_as_float(x4[e]);
                y = __int_as_float(y4[e]);
            } else if constexpr (DT == DT_BF16) {
                x = bf16_to_f32((uint16_t)((uint32_t)x4[e >> 1] >> (16 * (e & 1))));
                y = bf16_to_f32((uint16_t)((uint32_t)y4[e >> 1] >> (16 * (e & 1))));
            } else {
                x = e4m3_to_f32((uint8_t)((uint32_t)x4[e >> 2] >> (8 * (e & 3))));
                y = e4m3_to_f32((uint8_t)((uint32_t)y4[e >> 2] >> (8 * (e & 3))));
            }
            acc = __fma_rn((double)x, (double)y, acc);
        }
    }
    if constexpr (DT == DT_FP8) acc = ((double)sa * (double)sb) * acc;
    return acc;
}

// collision count of item p with the user code
__device__ __forceinline__ int collisions(const uint32_t* codes, int64_t p, const uint32_t* ucode, int W, int K)
{
    int diff = 0;
    for (int w = 0; w < W; w++) diff += __popc(codes[p * W + w] ^ ucode[w]);
    return K - diff;
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
    int64_t npairs = a.npairs;
    if (a.npairs_dev) {
        const int64_t c = (int64_t)*a.npairs_dev;
        npairs = c < npairs ? c : npairs;
    }
    for (int64_t pi = blockIdx.x; pi < npairs; pi += gridDim.x) {
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
        int ninit = 0;
        if (a.lam64) {
            // SAH: the candidate set starts as P'; its k-th largest score is the k-th of
            // u's k best scores on P', i.e. lambda row entries 1..k
            const uint32_t ou = a.perm[u];
            ninit = (int)((int64_t)k < a.n_init ? (int64_t)k : a.n_init);
            for (int i = tid; i < ninit; i += SQ_T) cand[i] = a.lam64[(int64_t)i * a.m + ou];
            if (ninit >= k) phi = a.lam64[(int64_t)(k - 1) * a.m + ou];
        }
        if (tid == 0) ccount = ninit;
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
            for (int64_t p = s0 + tid; p < s1; p += SQ_T) atomicAdd(&hist[collisions(a.item_codes, p, ucode, W, a.K)], 1);
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
            // ordered selection: candidates are the items above the cut and the first
            // need_eq at it (position order).  Each wave owns a contiguous quarter of
            // the partition: it counts its ties, one block-level prefix orders the
            // quarters, then every wave takes its items with wave-local ballots.
            const int wv = tid >> 6, ln = tid & 63;
            const int64_t qlen = (sz + SQ_T / 64 - 1) / (SQ_T / 64);
            const int64_t w0 = s0 + wv * qlen;
            const int64_t w1 = w0 + qlen < s1 ? w0 + qlen : s1;
            int my_eq = 0;
            for (int64_t base = w0; base < w1; base += 64) {
                const int64_t p = base + ln;
                const bool iseq = p < w1 && collisions(a.item_codes, p, ucode, W, a.K) == cut;
                my_eq += __popcll(ballot64(iseq));
            }
            if (ln == 0) wsum[wv] = my_eq;
            __syncthreads();
            int eq_before = 0;
            for (int w = 0; w < wv; w++) eq_before += wsum[w];
            for (int64_t base = w0; base < w1; base += 64) {
                const int64_t p = base + ln;
                const int c = p < w1 ? collisions(a.item_codes, p, ucode, W, a.K) : -1;
                const bool iseq = c == cut;
                const uint64_t eb = ballot64(iseq);
                const int rank_eq = eq_before + __popcll(eb & lanemask_lt());
                eq_before += __popcll(eb);
                const bool take_it = c > cut || (iseq && rank_eq < need_eq);
                // append candidate scores (order inside the candidate multiset is irrelevant)
                if (take_it) {
                    const float sp = DT == DT_FP8 ? a.item_scales[p] : 1.f;
                    const double v = sq_dot<DT>(a.users, u, su, a.items, p, sp, a.d, a.ld);
                    cand[atomicAdd(&ccount, 1)] = v;
                }
            }
            __syncthreads();
            ncand = ccount;
            __syncthreads();
            phi = ncand >= k ? block_kth(cand, ncand, k, hist, sh) : -__builtin_inf();
            if (suq < phi) { ans = 0; break; }
        }
        if (tid == 0) {
            if (a.phi) a.phi[pi] = phi;
            if (a.answer) a.answer[pi] = ans;
            if (a.qorig) {   // SAH: the decision is the answer
                if (ans) {
                    const uint32_t ou = a.perm[u];
                    const uint32_t qo = a.qorig[q];
                    if (a.bitmap) {
                        atomicOr(&a.bitmap[(int64_t)qo * a.bm_words + (ou >> 5)], 1u << (ou & 31u));
                    } else {
                        const unsigned long long pos = atomicAdd(a.pool_count, 1ull);
                        if ((int64_t)pos < a.pool_cap) a.pool[pos] = ((unsigned long long)qo << 32) | ou;
                    }
                } else {
                    atomicAdd(a.rejects, 1ull);
                }
            }
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
