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
// recheck.  In SAH mode (Alg. 5; k_sah_user, k_sah_decide below) the partitions cover
// P minus P', the candidate set starts from u's scores on P' (phi = L_u^k), and the
// answer is final.
#include <algorithm>
#include <cmath>
#include <cstdint>

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

// collision count of item p with the user code (rows of W words; 16-byte loads when
// the rows are 16-byte multiples)
__device__ __forceinline__ int collisions(const uint32_t* codes, int64_t p, const uint32_t* ucode, int W, int K)
{
    int diff = 0;
    const uint32_t* c = codes + p * W;
    if ((W & 3) == 0) {
        for (int w = 0; w < W; w += 4) {
            const uint4 v = *(const uint4*)(c + w);
            diff += __popc(v.x ^ ucode[w]) + __popc(v.y ^ ucode[w + 1]) + __popc(v.z ^ ucode[w + 2]) +
                    __popc(v.w ^ ucode[w + 3]);
        }
    } else {
        for (int w = 0; w < W; w++) diff += __popc(c[w] ^ ucode[w]);
    }
    return K - diff;
}

// Called by one whole wave: the bin that holds the need-th largest key of a histogram
// over bins [0, nbins) (lane l reads bins PER l .. PER l + PER - 1, nbins <= 64 PER),
// and the number of keys in higher bins; every lane receives both (bin -1 when the
// histogram holds fewer than need keys).
template <int PER>
__device__ __forceinline__ int2 wave_select_bin(const int* hist, int nbins, int need)
{
    const int l = lane_id();
    int h[PER], x = 0;
#pragma unroll
    for (int e = 0; e < PER; e++) {
        const int b = PER * l + e;
        h[e] = b < nbins ? hist[b] : 0;
        x += h[e];
    }
    const int incl = wave_incl_scan(x);
    int above = __shfl(incl, 63) - incl;   // keys in higher lanes' bins
    int sel = -1, sel_above = 0;
#pragma unroll
    for (int e = PER - 1; e >= 0; e--) {
        if (sel < 0 && above < need && need <= above + h[e]) {
            sel = PER * l + e;
            sel_above = above;
        }
        above += h[e];
    }
    const uint64_t bal = ballot64(sel >= 0);
    const int src = bal ? __builtin_ctzll(bal) : 0;
    return make_int2(__shfl(sel, src), __shfl(sel_above, src));
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
        if (tid < 64) {
            const int2 r = wave_select_bin<4>(hist, 256, need);
            if (tid == 0) {
                sh[0] = r.x < 0 ? 0 : r.x;
                sh[1] = r.x < 0 ? 0 : r.y;
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

// SimHash probe of partition [s0, s1) for user u (Alg. 2): the ceil(beta sz) items
// with the most equal code bits (equal counts: earlier position first) are scored and
// their scores appended to cand at *ccount.  Called by the whole workgroup; ends with a
// barrier, after which *ccount holds the new count.
// Canonical scores (as sq_dot) of the candidates whose positions fill cand[c_begin,
// c_end), in place.  Each wave takes 64 candidates at a time, one per lane; their rows
// pass through LDS in 64-byte column slices, four lanes loading one row's slice with
// consecutive 16-byte loads (one request per row and slice instead of one per lane and 16
// bytes), after which each lane continues its own index-order sum.  rows: the calling
// wave's 64 x SS_PITCH bytes of LDS.
static constexpr int SS_PITCH = 64 + 16;

template <int DT>
__device__ void score_staged(const SaQueryArgs& a, int64_t u, float su, double* cand, int c_begin, int c_end,
                             int64_t s0, int64_t s1, uint8_t* rows)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int PER = 16 / EB;
    const int l = lane_id(), wv = threadIdx.x >> 6;
    const int64_t RB = (int64_t)a.ld * EB;
    const int nch = (a.d * EB + 15) / 16;   // 16-byte chunks that hold the d elements
    const uint8_t* ur = (const uint8_t*)a.users + u * RB;
    for (int base = c_begin + wv * 64; base < c_end; base += SQ_T) {
        const int idx = base + l;
        const bool in = idx < c_end;
        int p = -1;
        if (in) {
            const int64_t q = (int64_t)__double_as_longlong(cand[idx]);
            if (q >= s0 && q < s1) p = (int)q;   // always: every slot holds a position of the partition
        }
        double acc = 0.0;
        for (int ch0 = 0; ch0 < nch; ch0 += 4) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int k = i * 64 + l, r = k >> 2, c = k & 3;
                const int pr = __shfl(p, r);
                i32x4 v = {0, 0, 0, 0};
                if (pr >= 0 && ch0 + c < nch) v = *(const i32x4*)((const uint8_t*)a.items + (int64_t)pr * RB + (ch0 + c) * 16);
                *(i32x4*)(rows + r * SS_PITCH + c * 16) = v;
            }
            __builtin_amdgcn_wave_barrier();
            if (p >= 0) {
                for (int c = 0; c < 4; c++) {
                    const int ch = ch0 + c;
                    if (ch >= nch) break;
                    const i32x4 y4 = *(const i32x4*)(rows + l * SS_PITCH + c * 16);
                    const i32x4 x4 = *(const i32x4*)(ur + ch * 16);
                    const int lim = a.d - ch * PER < PER ? a.d - ch * PER : PER;
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
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (in) {
            if (p >= 0) {
                if constexpr (DT == DT_FP8) acc = ((double)su * (double)a.item_scales[p]) * acc;
                cand[idx] = acc;
            } else {
                cand[idx] = -__builtin_inf();
            }
        }
    }
}

// whist: [SQ_T / 64][SQ_T + 1] ints, one collision-count histogram per wave.
template <int DT>
__device__ void probe_partition(const SaQueryArgs& a, int64_t u, float su, const uint32_t* ucode, int W,
                                int64_t s0, int64_t s1, double* cand, int (*whist)[SQ_T + 1], int* sh,
                                int* ccount, uint8_t* rows)
{
    const int tid = threadIdx.x;
    const int64_t sz = s1 - s0;
    int64_t take = (int64_t)ceil((double)a.beta * (double)sz);
    if (take > sz) take = sz;
    // read before any wave can append (the callers change *ccount only behind a barrier)
    const int c_begin = *ccount;
    if (take == sz) {   // every item is a candidate: no selection
        for (int64_t p = s0 + tid; p < s1; p += SQ_T) {
            const int64_t slot = c_begin + (p - s0);
            if (slot < a.cand_cap) cand[slot] = __longlong_as_double((long long)p);
        }
        __syncthreads();
        if (tid == 0) {
            *ccount = (int)(c_begin + sz < a.cand_cap ? c_begin + sz : a.cand_cap);
            if (c_begin + sz > a.cand_cap && a.overflow) atomicOr(a.overflow, kSaalshOverflowBit);
        }
    } else {
        // Each wave owns a contiguous quarter of the partition and histograms its collision
        // counts; the sum over the waves gives the cut, and the waves before a wave hold the
        // ties that precede its quarter in position order.
        const int wv = tid >> 6, ln = tid & 63;
        const int64_t qlen = (sz + SQ_T / 64 - 1) / (SQ_T / 64);
        const int64_t w0 = s0 + wv * qlen;
        const int64_t w1 = w0 + qlen < s1 ? w0 + qlen : s1;
        for (int b = ln; b <= a.K; b += 64) whist[wv][b] = 0;
        __syncthreads();
        for (int64_t p = w0 + ln; p < w1; p += 64) atomicAdd(&whist[wv][collisions(a.item_codes, p, ucode, W, a.K)], 1);
        __syncthreads();
        // the waves' sum, then the cut count c*: #(count > c*) < take <= #(count >= c*)
        for (int b = tid; b <= a.K; b += SQ_T) {
            int h = 0;
            for (int w = 0; w < SQ_T / 64; w++) h += whist[w][b];
            sh[4 + b] = h;
        }
        __syncthreads();
        if (tid < 64) {
            const int2 r = wave_select_bin<5>(sh + 4, a.K + 1, (int)take);
            if (tid == 0) {
                sh[0] = r.x;
                sh[1] = (int)take - r.y;
            }
        }
        __syncthreads();
        const int cut = sh[0];
        const int need_eq = sh[1];
        // ordered selection: candidates are the items above the cut and the first need_eq
        // at it (position order), taken by every wave with wave-local ballots
        int eq_before = 0;
        for (int w = 0; w < wv; w++) eq_before += whist[w][cut];
        for (int64_t base = w0; base < w1; base += 64) {
            const int64_t p = base + ln;
            const int c = p < w1 ? collisions(a.item_codes, p, ucode, W, a.K) : -1;
            const bool iseq = c == cut;
            const uint64_t eb = ballot64(iseq);
            const int rank_eq = eq_before + __popcll(eb & lanemask_lt());
            eq_before += __popcll(eb);
            const bool take_it = c > cut || (iseq && rank_eq < need_eq);
            // the candidate's position, in the slot its score will take (the order inside the
            // candidate multiset is irrelevant)
            // exactly take items pass (take - need_eq above the cut, need_eq ties), so the
            // slots stay below c_begin + take <= cand_cap; the test is the backstop
            if (take_it) {
                const int slot = atomicAdd(ccount, 1);
                if (slot < a.cand_cap) cand[slot] = __longlong_as_double((long long)p);
                else if (a.overflow) atomicOr(a.overflow, kSaalshOverflowBit);
            }
        }
    }
    __syncthreads();
    // scores of the new candidates, every lane busy (the selection keeps about one item
    // in 1/beta, so scoring inside its loop would leave most lanes idle)
    const int c_end = *ccount < a.cand_cap ? *ccount : (int)a.cand_cap;
    score_staged<DT>(a, u, su, cand, c_begin, c_end, s0, s1, rows + (tid >> 6) * 64 * SS_PITCH);
    __syncthreads();
}

template <int DT>
__global__ __launch_bounds__(SQ_T) void k_saalsh_query(SaQueryArgs a, double* scratch, int64_t scratch_stride)
{
    __shared__ int whist[SQ_T / 64][SQ_T + 1];
    __shared__ __attribute__((aligned(16))) uint8_t rows[SQ_T / 64][64 * SS_PITCH];
    __shared__ int sh[4 + SQ_T + 1];   // [0, 4): results; [4, 4 + K + 1]: counts
    __shared__ int ccount;
    int* hist = whist[0];
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
        if (tid == 0) ccount = 0;
        __syncthreads();
        int ans = 1;
        for (int j = 0; j < a.t; j++) {
            const int64_t s0 = a.part_start[j], s1 = a.part_start[j + 1];
            const double mu = sqrt(a.item_n2[s0]) * unorm;
            if (phi > mu) { ans = 1; break; }
            probe_partition<DT>(a, u, su, ucode, W, s0, s1, cand, whist, sh, &ccount, &rows[0][0]);
            const int64_t ncand = ccount < a.cand_cap ? ccount : a.cand_cap;
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

// ------------------------------------------------------------------ SAH: Alg. 2 per user
// In Alg. 2 the candidate sets, and so phi after each partition, depend on the user and
// k only; the query enters through s(u,q) in the two tests.  A batch therefore runs the
// probes once per user that has an undecided pair: row j of the user's table holds the
// kstar largest candidate scores after j partitions (row 0: the scores on P', i.e. the
// lambda row), so phi_j = row j entry k - 1 for every k <= kstar.  k_sah_decide then
// walks each pair through the same tests in the same order as the per-pair kernel
// above, with identical results.

// Users with an undecided pair (flag set by the recheck) get consecutive slots.
__global__ void k_sah_slots(const unsigned char* need, int64_t m, int* slot, int* nslots)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = u < m && need[u];
    const uint64_t bal = ballot64(f);
    int base = 0;
    if (lane_id() == 0 && bal) base = atomicAdd(nslots, __popcll(bal));
    base = __shfl(base, 0);
    if (f) slot[u] = base + __popcll(bal & lanemask_lt());
}

__global__ void k_sah_invert(const unsigned char* need, const int* slot, int64_t m, int* user_of_slot)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < m && need[u]) user_of_slot[slot[u]] = (int)u;
}

// Sorted (descending) kstar largest of vals[0, cnt) into top[0, kstar) (-inf past cnt),
// by one workgroup; vals then holds the same kstar values (cnt becomes min(cnt, kstar)).
__device__ void block_top_sorted(double* vals, int64_t cnt, int kstar, double* top, int* hist, int* sh, int* tcount)
{
    const int tid = threadIdx.x;
    int P = 1;
    while (P < kstar) P <<= 1;
    for (int i = tid; i < P; i += SQ_T) top[i] = -__builtin_inf();
    if (tid == 0) *tcount = 0;
    __syncthreads();
    if (cnt <= kstar) {
        for (int64_t i = tid; i < cnt; i += SQ_T) top[i] = vals[i];
    } else {
        const double T = block_kth(vals, cnt, kstar, hist, sh);   // ends with a barrier
        for (int64_t i = tid; i < cnt; i += SQ_T)
            if (vals[i] > T) top[atomicAdd(tcount, 1)] = vals[i];
        __syncthreads();
        const int gt = *tcount;   // < kstar; the rest of the kstar are copies of T
        for (int i = gt + tid; i < kstar; i += SQ_T) top[i] = T;
    }
    __syncthreads();
    // bitonic sort, descending
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += SQ_T) {
                const int o = i ^ j;
                if (o > i) {
                    const bool desc = (i & kk) == 0;
                    const double x = top[i], y = top[o];
                    if (desc ? x < y : x > y) {
                        top[i] = y;
                        top[o] = x;
                    }
                }
            }
            __syncthreads();
        }
    const int keep = (int)(cnt < kstar ? cnt : kstar);
    for (int i = tid; i < keep; i += SQ_T) vals[i] = top[i];
    __syncthreads();
}

// One workgroup per slot in [c0, c0 + chunk): the user's table rows, tab[(slot - c0)
// (t + 1) kstar ...].  The probes stop once row j's kstar-th score exceeds mu_j: every
// pair of the batch (k <= kstar) is then answered yes at partition j at the latest.
template <int DT>
__global__ __launch_bounds__(SQ_T) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_sah_user(SaQueryArgs a, const int* user_of_slot, const int* nslots,
                                                  int64_t c0, int64_t chunk, int kstar, double* tab,
                                                  double* scratch, int64_t scratch_stride, int* jlast)
{
    __shared__ int whist[SQ_T / 64][SQ_T + 1];
    __shared__ __attribute__((aligned(16))) uint8_t rows[SQ_T / 64][64 * SS_PITCH];
    __shared__ int sh[4 + SQ_T + 1];   // [0, 4): results; [4, 4 + K + 1]: counts
    __shared__ int tcount;
    __shared__ int ccount;
    __shared__ double top[256];
    int* hist = whist[0];
    const int tid = threadIdx.x;
    const int W = a.K / 32;
    int64_t hi = (int64_t)*nslots;
    hi = hi < c0 + chunk ? hi : c0 + chunk;
    double* cand = scratch + (int64_t)blockIdx.x * scratch_stride;
    for (int64_t sl = c0 + blockIdx.x; sl < hi; sl += gridDim.x) {
        const int64_t u = user_of_slot[sl];
        const uint32_t ou = a.perm[u];
        const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
        const double unorm = sqrt(a.user_n2[u]);
        uint32_t ucode[8];
        for (int w = 0; w < W; w++) ucode[w] = a.user_codes[u * W + w];
        double* row = tab + (sl - c0) * (int64_t)(a.t + 1) * kstar;
        const int ninit = (int)((int64_t)kstar < a.n_init ? (int64_t)kstar : a.n_init);
        for (int i = tid; i < kstar; i += SQ_T) {
            const double v = i < ninit ? a.lam64[(int64_t)i * a.m + ou] : -__builtin_inf();
            row[i] = v;
            if (i < ninit) cand[i] = v;
        }
        if (tid == 0) ccount = ninit;
        __syncthreads();
        double phi_min = ninit >= kstar ? a.lam64[(int64_t)(kstar - 1) * a.m + ou] : -__builtin_inf();
        int j = 0;
        for (; j < a.t; j++) {
            const int64_t s0 = a.part_start[j], s1 = a.part_start[j + 1];
            const double mu = sqrt(a.item_n2[s0]) * unorm * a.mu_scale;
            if (phi_min > mu) break;
            probe_partition<DT>(a, u, su, ucode, W, s0, s1, cand, whist, sh, &ccount, &rows[0][0]);
            const int64_t ncand = ccount < a.cand_cap ? ccount : a.cand_cap;
            __syncthreads();
            block_top_sorted(cand, ncand, kstar, top, hist, sh, &tcount);
            double* rj = row + (int64_t)(j + 1) * kstar;
            for (int i = tid; i < kstar; i += SQ_T) rj[i] = top[i];
            phi_min = top[kstar - 1];
            if (tid == 0) ccount = (int)(ncand < kstar ? ncand : kstar);
            __syncthreads();
        }
        if (jlast && tid == 0) jlast[sl - c0] = j;   // rows 0..j are written
    }
}

// Each pair whose user has its slot in [c0, c0 + chunk): the tests of Alg. 2 against the
// user's table; a yes goes to the answers, a no counts in *rejects.
__global__ void k_sah_decide(SaQueryArgs a, const double* score, const int* slot, int64_t c0, int64_t chunk,
                             int kstar, const double* tab)
{
    int64_t np = (int64_t)*a.npairs_dev;
    np = np < a.npairs ? np : a.npairs;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = a.pairs[i];
        const int64_t q = (int64_t)(key >> 32), u = (int64_t)(key & 0xffffffffull);
        const int64_t sl = slot[u];
        if (sl < c0 || sl >= c0 + chunk) continue;
        const int k = a.qk[q];
        const double s = score[i];
        const double unorm = sqrt(a.user_n2[u]);
        const double* row = tab + (sl - c0) * (int64_t)(a.t + 1) * kstar;
        double phi = row[k - 1];
        bool ans = true;
        for (int j = 0; j < a.t; j++) {
            const double mu = sqrt(a.item_n2[a.part_start[j]]) * unorm * a.mu_scale;
            if (phi > mu) break;
            phi = row[(int64_t)(j + 1) * kstar + k - 1];
            if (s < phi) { ans = false; break; }
        }
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

// The sizes the probe kernels rely on, checked on the host before each launch:
//   K: whole 32-bit code words, at most 8 of them (ucode[8]); K + 1 histogram bins fit
//      the SQ_T + 1 per wave;
//   the candidate row: per-user kernels (k_sah_user) start from at most kstar scores
//      (the lambda prefix) and add ceil(beta |S_j|) <= ceil(beta n) per partition
//      before cutting back to kstar, so they need kstar + ceil(beta n); the per-pair
//      kernel keeps every partition's candidates, sum_j ceil(beta |S_j|) <= ceil(beta n)
//      + t;
//   kstar <= 256 (the top[] array of block_top_sorted);
//   grid rows of scratch_stride doubles inside the scratch allocation.
static SaQueryArgs checked_args(const SaQueryArgs& a, int64_t kstar, bool per_user, size_t scratch_bytes,
                                int64_t scratch_stride, int grid)
{
    if (a.K < 32 || a.K > 256 || a.K % 32 != 0) fail(RKMIPS_EINVAL, "internal: SA-ALSH code width");
    static_assert(SQ_T + 1 >= 256 + 1, "collision histogram bins");
    if (per_user && (kstar < 1 || kstar > 256)) fail(RKMIPS_EINVAL, "internal: SA-ALSH table width");
    const int64_t picks = (int64_t)std::ceil((double)a.beta * (double)a.n);
    const int64_t need = per_user ? kstar + picks : picks + a.t;
    if (scratch_stride < need) fail(RKMIPS_EINVAL, "internal: SA-ALSH candidate row too short");
    if (scratch_stride > INT32_MAX) fail(RKMIPS_EINVAL, "internal: SA-ALSH candidate row too long");
    if (grid < 1 || (size_t)grid * (size_t)scratch_stride * sizeof(double) > scratch_bytes)
        fail(RKMIPS_EINVAL, "internal: SA-ALSH scratch smaller than grid x row");
    SaQueryArgs b = a;
    b.cand_cap = scratch_stride;
    return b;
}

// LDS of the probe kernels (static): histograms, staged rows, counts, top[256].
static_assert(sizeof(int) * (SQ_T / 64) * (SQ_T + 1) + (SQ_T / 64) * 64 * SS_PITCH + sizeof(int) * (4 + SQ_T + 1) +
                      2 * sizeof(int) + sizeof(double) * 256 <= 65536,
              "probe kernels' LDS");

void launch_sah(const SaQueryArgs& a0, const unsigned char* need, int* slot, int* user_of_slot, int* nslots,
                const double* score, int kstar, double* tab, int64_t chunk, double* scratch, size_t scratch_bytes,
                int64_t scratch_stride, int grid, hipStream_t s)
{
    if (a0.npairs <= 0 || a0.m <= 0) return;
    const SaQueryArgs a = checked_args(a0, kstar, true, scratch_bytes, scratch_stride, grid);
    hipLaunchKernelGGL(k_sah_slots, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, need, a.m, slot, nslots);
    hipLaunchKernelGGL(k_sah_invert, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, need, slot, a.m,
                       user_of_slot);
    for (int64_t c0 = 0; c0 < a.m; c0 += chunk) {
        if (a.dtype == DT_F32) hipLaunchKernelGGL(k_sah_user<DT_F32>, dim3(grid), dim3(SQ_T), 0, s, a, (const int*)user_of_slot, (const int*)nslots, c0, chunk, kstar, tab, scratch, scratch_stride, (int*)nullptr);
        else if (a.dtype == DT_BF16) hipLaunchKernelGGL(k_sah_user<DT_BF16>, dim3(grid), dim3(SQ_T), 0, s, a, (const int*)user_of_slot, (const int*)nslots, c0, chunk, kstar, tab, scratch, scratch_stride, (int*)nullptr);
        else hipLaunchKernelGGL(k_sah_user<DT_FP8>, dim3(grid), dim3(SQ_T), 0, s, a, (const int*)user_of_slot, (const int*)nslots, c0, chunk, kstar, tab, scratch, scratch_stride, (int*)nullptr);
        const unsigned gd = (unsigned)std::min<int64_t>((a.npairs + 255) / 256, 2048);
        hipLaunchKernelGGL(k_sah_decide, dim3(gd), dim3(256), 0, s, a, score, (const int*)slot, c0, chunk, kstar,
                           (const double*)tab);
    }
    HIPC(hipGetLastError());
}

void launch_saalsh_query(const SaQueryArgs& a0, double* scratch, size_t scratch_bytes, int64_t scratch_stride,
                         int grid, hipStream_t s)
{
    if (a0.npairs <= 0) return;
    const SaQueryArgs a = checked_args(a0, 0, false, scratch_bytes, scratch_stride, grid);
    if (a.dtype == DT_F32) hipLaunchKernelGGL(k_saalsh_query<DT_F32>, dim3(grid), dim3(SQ_T), 0, s, a, scratch, scratch_stride);
    else if (a.dtype == DT_BF16) hipLaunchKernelGGL(k_saalsh_query<DT_BF16>, dim3(grid), dim3(SQ_T), 0, s, a, scratch, scratch_stride);
    else hipLaunchKernelGGL(k_saalsh_query<DT_FP8>, dim3(grid), dim3(SQ_T), 0, s, a, scratch, scratch_stride);
    HIPC(hipGetLastError());
}

// SA-ALSH kMIPS (Alg. 2 without a query): for the users user_of_slot[0, nu) (leaf
// positions), the k best scores found by the probes, partitions visited in order until
// the k-th best exceeds mu_j; tab [nu x (t + 1) x k], jlast [nu]: row jlast of a user is
// its answer.
void launch_saalsh_kmips(const SaQueryArgs& a0, const int* user_of_slot, const int* nslots, int64_t nu, int k,
                         double* tab, int* jlast, double* scratch, size_t scratch_bytes, int64_t scratch_stride,
                         int grid, hipStream_t s)
{
    if (nu <= 0) return;
    if (k < 1 || k > 256) fail(RKMIPS_EINVAL, "internal: kMIPS width");
    const SaQueryArgs a = checked_args(a0, k, true, scratch_bytes, scratch_stride, grid);
    if (a.dtype == DT_F32) hipLaunchKernelGGL(k_sah_user<DT_F32>, dim3(grid), dim3(SQ_T), 0, s, a, user_of_slot, nslots, (int64_t)0, nu, k, tab, scratch, scratch_stride, jlast);
    else if (a.dtype == DT_BF16) hipLaunchKernelGGL(k_sah_user<DT_BF16>, dim3(grid), dim3(SQ_T), 0, s, a, user_of_slot, nslots, (int64_t)0, nu, k, tab, scratch, scratch_stride, jlast);
    else hipLaunchKernelGGL(k_sah_user<DT_FP8>, dim3(grid), dim3(SQ_T), 0, s, a, user_of_slot, nslots, (int64_t)0, nu, k, tab, scratch, scratch_stride, jlast);
    HIPC(hipGetLastError());
}

}  // namespace rk
