// lambda build, pass 2 (k_refine): canonical FP64 rescoring of the candidates that the
// fused top-k pass (k_topk.hip) left in the per-user buffers, ranking, and a certificate:
// tau + eps(u) <= lambda64^(k_max) proves that no left-out item can enter the top k_max
// (Definition 1; the lower-bound array of Alg. 4 taken over all of P).  A seed estimate
// that was too high leaves fewer than k_max candidates above tau and fails it; users
// that fail get a full-row FP64 rescoring (k_fallback).
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace rk {

// ------------------------------------------------------------------ wave radix select
// C-th largest of the first c keys held GPL per lane (entry i of lane l is position
// l + 64 i); *need_eq receives how many keys equal to it belong to the C largest.
// Bits that all keys share are settled at once (close scores share their sign, exponent
// and leading mantissa bits, and a histogram over them would put every key in one bin):
// the digits of up to 8 bits start at the highest bit where two keys differ.
template <int GPL>
__device__ __forceinline__ uint32_t wave_kth_key(const uint32_t (&key)[GPL], int c, int C, int* hist, int* need_eq)
{
    const int l = lane_id();
    const uint32_t k0 = __shfl(key[0], 0);   // c > 0: position 0 holds a key
    uint32_t diff = 0u;
#pragma unroll
    for (int i = 0; i < GPL; i++)
        if (l + 64 * i < c) diff |= key[i] ^ k0;
    diff = wave_or(diff);
    int top = diff ? 32 - __builtin_clz(diff) : 0;   // bits [0, top) are still open
    uint32_t pmask = top >= 32 ? 0u : ~((1u << top) - 1u);
    uint32_t prefix = k0 & pmask;
    int need = C;
    while (top > 0) {
        const int wd = top >= 8 ? 8 : top;
        const int shift = top - wd;
        const uint32_t dmask = (1u << wd) - 1u;
        for (int b = l; b < 256; b += 64) hist[b] = 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < GPL; i++) {
            if (64 * i >= c) break;   // wave-uniform: the rest of the slots are empty
            if (l + 64 * i < c && (key[i] & pmask) == prefix) atomicAdd(&hist[(key[i] >> shift) & dmask], 1);
        }
        __builtin_amdgcn_wave_barrier();
        int h[4], x = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) { h[e] = hist[4 * l + e]; x += h[e]; }
        const int incl = wave_incl_scan(x);
        const int total = __shfl(incl, 63);
        int above = total - incl;  // keys whose digit lies in higher lanes' bins
        int sel = -1, sel_above = 0;
#pragma unroll
        for (int e = 3; e >= 0; e--) {
            if (sel < 0 && above < need && need <= above + h[e]) { sel = 4 * l + e; sel_above = above; }
            above += h[e];
        }
        const uint64_t bal = ballot64(sel >= 0);
        const int src = bal ? __builtin_ctzll(bal) : 0;
        const int dsel = __shfl(sel, src);
        const int dabove = __shfl(sel_above, src);
        prefix |= (uint32_t)dsel << shift;
        pmask |= dmask << shift;
        need -= dabove;
        top = shift;
        __builtin_amdgcn_wave_barrier();
    }
    *need_eq = need;
    return prefix;
}

// Output positions (or -1) of the kept entries: keys > T, then keys == T in position
// order until need_eq of them are kept.
template <int GPL>
__device__ __forceinline__ void wave_keep_positions(const uint32_t (&key)[GPL], int c, uint32_t T, int need_eq,
                                                    int (&outpos)[GPL])
{
    const int l = lane_id();
    int eq_before = 0, kept_before = 0;
#pragma unroll
    for (int i = 0; i < GPL; i++) outpos[i] = -1;
#pragma unroll
    for (int i = 0; i < GPL; i++) {
        if (64 * i >= c) break;
        const bool valid = l + 64 * i < c;
        const bool gt = valid && key[i] > T;
        const bool eq = valid && key[i] == T;
        const uint64_t eb = ballot64(eq);
        const int rank_eq = eq_before + __popcll(eb & lanemask_lt());
        eq_before += __popcll(eb);
        const bool keep = gt || (eq && rank_eq < need_eq);
        const uint64_t kb = ballot64(keep);
        outpos[i] = keep ? kept_before + __popcll(kb & lanemask_lt()) : -1;
        kept_before += __popcll(kb);
    }
}

// ------------------------------------------------------------------ FP64 refine + certificate
static constexpr int RF_MAXN = 2048;  // candidates per user across segments
static constexpr int RF_GPL = RF_MAXN / 64;

// One 16-byte chunk of the canonical sum: elements c0 .. c0 + 16 / EB - 1 (those below d)
// of user chunk a4 and item chunk b4, added in index order to acc.
template <int DT>
__device__ __forceinline__ double canon_chunk(const i32x4& a4, const i32x4& b4, int c0, int d, double acc)
{
    constexpr int PER = 16 / Elt<DT>::bytes;
    const int lim = d - c0 < PER ? d - c0 : PER;
#pragma unroll
    for (int e = 0; e < PER; e++) {
        if (e >= lim) break;
        float x, y;
        if constexpr (DT == DT_F32) {
            x = __int_as_float(a4[e]);
            y = __int_as_float(b4[e]);
        } else if constexpr (DT == DT_BF16) {
            x = bf16_to_f32((uint16_t)((uint32_t)a4[e >> 1] >> (16 * (e & 1))));
            y = bf16_to_f32((uint16_t)((uint32_t)b4[e >> 1] >> (16 * (e & 1))));
        } else {
            x = e4m3_to_f32((uint8_t)((uint32_t)a4[e >> 2] >> (8 * (e & 3))));
            y = e4m3_to_f32((uint8_t)((uint32_t)b4[e >> 2] >> (8 * (e & 3))));
        }
        acc = __fma_rn((double)x, (double)y, acc);
    }
    return acc;
}

// FP8 form of canon_chunk: the user's values come decoded from LDS (ux, exact e4m3
// values as floats, shared by the wave), the item's from its codes.  Two e4m3 values
// multiply exactly in FP32 (at most 8 significant bits, magnitudes in [2^-18, 2^18]),
// so acc + (double)(x y) is the canonical step RN(acc + x y), bit for bit.
// The item codes are decoded by the hardware conversion (two codes per instruction; every
// e4m3 value is exact in FP32, and rkmips_diag_fp8_decode checks the conversion against
// the format's definition code by code).
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double canon_chunk_fp8(const float* ux, const i32x4& b4, int c0, int d, double acc)
{
    const int lim = d - c0 < 16 ? d - c0 : 16;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const f32x4 x4 = *(const f32x4*)(ux + c0 + 4 * q);
        const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(b4[q], false);   // bytes 0, 1
        const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8(b4[q], true);    // bytes 2, 3
        const float y[4] = {lo[0], lo[1], hi[0], hi[1]};
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (4 * q + e >= lim) break;
            acc = acc + (double)(x4[e] * y[e]);
        }
    }
    return acc;
}

// The user row's values for canon_chunk_fp8: udec[i] = value of code i (0 past d).
// Called by the whole wave; ends with a wave barrier.
__device__ __forceinline__ void decode_user_fp8(const RefineArgs& a, int64_t u, float* udec)
{
    const uint8_t* ur = (const uint8_t*)a.users + u * (int64_t)a.ld;
    for (int i = lane_id(); i < a.ld; i += 64) udec[i] = i < a.d ? e4m3_to_f32(ur[i]) : 0.f;
    __builtin_amdgcn_wave_barrier();
}

// Canonical scores of user u against the items sid[0, Nk), lane l taking candidate l
// (lanes past Nk, and positions past n, get -inf).  The candidate rows pass through LDS
// in 64-byte column slices: four lanes load one row's slice with consecutive 16-byte
// loads (one request per row and slice instead of one per lane and 16 bytes), then each
// lane continues its own index-order sum over the slice.  (Issuing several slices' loads
// together cost registers and occupancy and ran slower.)
static constexpr int RF_SLICE = 64;
static constexpr int RF_PITCH = RF_SLICE + 16;   // LDS row pitch (bank spread)

// udec (FP8): the user's decoded values (decode_user_fp8).
template <int DT>
__device__ __forceinline__ double canon_dot_staged(const RefineArgs& a, int64_t u, float su, const uint32_t* sid,
                                                   int Nk, uint8_t* rows, const float* udec)
{
    constexpr int EB = Elt<DT>::bytes;
    const int l = lane_id();
    const int RB = a.ld * EB;
    const uint8_t* ur = (const uint8_t*)a.users + u * (int64_t)RB;
    const uint32_t mine = l < Nk ? sid[l] : 0xffffffffu;
    const bool live = l < Nk && (int64_t)mine < a.n;   // positions come from k_topk; the test guards the loads
    double acc = 0.0;
    for (int s0 = 0; s0 < RB; s0 += RF_SLICE) {
        constexpr int CPS = RF_SLICE / 16;   // chunks per row slice
#pragma unroll
        for (int i = 0; i < CPS; i++) {
            const int k = i * 64 + l, r = k / CPS, c = k % CPS;
            const int off = s0 + c * 16;
            i32x4 val = {0, 0, 0, 0};
            if (r < Nk && off < RB) {
                const uint32_t p = sid[r];
                if ((int64_t)p < a.n) val = *(const i32x4*)((const uint8_t*)a.items + (int64_t)p * RB + off);
            }
            *(i32x4*)(rows + r * RF_PITCH + c * 16) = val;
        }
        __builtin_amdgcn_wave_barrier();
        if (live) {
#pragma unroll
            for (int c = 0; c < CPS; c++) {
                const int off = s0 + c * 16;
                if (off >= RB) break;
                const i32x4 b4 = *(const i32x4*)(rows + l * RF_PITCH + c * 16);
                if constexpr (DT == DT_FP8) {
                    acc = canon_chunk_fp8(udec, b4, off, a.d, acc);
                } else {
                    const i32x4 a4 = *(const i32x4*)(ur + off);
                    acc = canon_chunk<DT>(a4, b4, off / EB, a.d, acc);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (!live) return -__builtin_inf();
    if constexpr (DT == DT_FP8) acc = ((double)su * (double)a.item_scales[mine]) * acc;
    return acc;
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long* addr, double v)
{
    // non-negative doubles order like their bit patterns; skip the atomic when it cannot win
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(addr, b);
}

// One wave per user: gather the candidates of all segments, keep the C best by the fast
// score (wave radix select), rescore those in canonical FP64, rank them, write
// lambda64/lambda32 for j <= k_max and test the certificate
//   max(tau_s, cut) + eps(u) <= lambda64^(k_max)
// where every item outside the rescored set scored at most max(tau_s, cut) in the fast
// arithmetic (tau_s: segment thresholds of the streaming pass; cut: the C-th best fast
// score among all candidates when some were dropped here).
// Gathers user u's candidates from every segment's buffer and keeps the C best by the
// fast score (all of them when there are at most C) in skey/sid, in gather order.
// *cut: the C-th best fast score when some were dropped (else -inf); *tau_max: the
// largest segment threshold.  Returns false (and lists u for the wide pass) when the
// candidates do not fit GPL per lane.
template <int GPL>
__device__ bool refine_select(const RefineArgs& a, int64_t u, uint32_t* skey, uint32_t* sid, int* hist, int* nk_out,
                              float* cut_out, float* tau_out)
{
    const int l = lane_id();
    // gather every segment's buffer straight into registers (entry j = lane + 64 i).
    // Part p = 2 s + h is half h of segment s's buffer; there are P = 2 nseg <= 64 parts
    // (nseg G <= RF_MAXN with G >= 128 gives at most 16 segments).  Lane p reads part p's
    // count; the running totals cum[0..P] go to the wave's LDS scratch (hist, which the
    // selection below reuses once the gather is done).
    const int P = 2 * a.nseg;
    int* cum = hist;
    const int c = l < P ? a.cnt[(u * a.nseg + (l >> 1)) * 2 + (l & 1)] : 0;
    const int incl = wave_incl_scan(c);
    if (l < P) cum[l + 1] = incl;
    if (l == 0) cum[0] = 0;
    const int N = __shfl(incl, P - 1);
    const float tau_max = wave_max(l < a.nseg ? a.tau[u * a.nseg + l] : -__builtin_inff());
    __builtin_amdgcn_wave_barrier();
    if (N > GPL * 64) {   // more candidates than this instance holds: the wide pass takes it
        if (l == 0) a.spill[atomicAdd(a.spill_count, 1)] = (int)u;
        return false;
    }
    const int HG = a.G / 2;
    uint32_t key[GPL], id[GPL];
#pragma unroll
    for (int i = 0; i < GPL; i++) {
        key[i] = 0u;
        id[i] = 0u;
    }
#pragma unroll
    for (int i = 0; i < GPL; i++) {
        if (64 * i >= N) break;   // wave-uniform
        const int j = l + 64 * i;
        if (j < N) {
            // part of entry j: the first q in [1, P) with cum[q] > j, minus one (empty
            // parts have cum[q] == cum[q + 1] and are passed over)
            int lo = 1, hi = P;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cum[mid] > j) hi = mid;
                else lo = mid + 1;
            }
            const int p = lo - 1;
            const uint2 e = a.buf[(u * a.nseg + (p >> 1)) * (int64_t)a.G + (p & 1) * HG + (j - cum[p])];
            key[i] = f32_ord(__uint_as_float(e.x));
            id[i] = e.y;
        }
    }
    float cut = -__builtin_inff();
    int Nk = N;
    int outpos[GPL];
    if (N > a.C) {
        int need_eq;
        const uint32_t T = wave_kth_key<GPL>(key, N, a.C, hist, &need_eq);
        wave_keep_positions<GPL>(key, N, T, need_eq, outpos);
        cut = ord_f32(T);
        Nk = a.C;
    } else {
#pragma unroll
        for (int i = 0; i < GPL; i++) outpos[i] = (l + 64 * i < N) ? l + 64 * i : -1;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < GPL; i++) {
        if (64 * i >= N) break;
        if (outpos[i] >= 0) {
            skey[outpos[i]] = key[i];
            sid[outpos[i]] = id[i];
        }
    }
    __builtin_amdgcn_wave_barrier();
    *nk_out = Nk;
    *cut_out = cut;
    *tau_out = tau_max;
    return true;
}

// Canonical FP64 rescoring of the kept candidates skey/sid [0, Nk), their ranks,
// lambda64/lambda32 for j <= k_max and the certificate
//   max(tau_max, cut) + eps(u) <= lambda64^(k_max)
// where every item outside the rescored set scored at most max(tau_max, cut) in the fast
// arithmetic.
// Bitonic sort of 64 * NPL (score, slot) pairs held NPL per lane (element i = 64 s + lane
// in v[s], ix[s]) into descending score order, equal scores by ascending slot; pairs that
// are 64 apart or more meet inside a lane, the others across lanes by shuffles.
template <int NPL>
__device__ __forceinline__ void wave_sort_desc(double (&v)[4], int (&ix)[4])
{
    const int l = lane_id();
#pragma unroll
    for (int kk = 2; kk <= 64 * NPL; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
#pragma unroll
                for (int s = 0; s < NPL; s++) {
                    const int p = s ^ (j >> 6);
                    if (p > s) {
                        const bool desc = ((64 * s + l) & kk) == 0;
                        const bool first = v[s] > v[p] || (v[s] == v[p] && ix[s] < ix[p]);
                        if (first != desc) {
                            const double tv = v[s];
                            v[s] = v[p];
                            v[p] = tv;
                            const int ti = ix[s];
                            ix[s] = ix[p];
                            ix[p] = ti;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < NPL; s++) {
                    const double ov = __shfl_xor(v[s], j);
                    const int oi = __shfl_xor(ix[s], j);
                    const bool lower = (l & j) == 0, desc = ((64 * s + l) & kk) == 0;
                    const bool mine_first = v[s] > ov || (v[s] == ov && ix[s] < oi);
                    if (mine_first != (lower == desc)) {
                        v[s] = ov;
                        ix[s] = oi;
                    }
                }
            }
        }
    }
}

template <int DT, bool FAST>
__device__ void refine_rank(const RefineArgs& a, int64_t u, const uint32_t* skey, const uint32_t* sid, int Nk,
                            float cut, float tau_max, double* s64, double* lam_row, uint8_t* rows, float* udec)
{
    if constexpr (DT == DT_FP8) decode_user_fp8(a, u, udec);
    const int l = lane_id();
    const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
    const double un = sqrt(a.user_n2[u]);
    const double M = sqrt(a.item_n2_sorted[0]);
    double worst_raw = 0.0, worst32 = 0.0;
    double lk = -__builtin_inf();   // lambda64^(k_max) over the candidates (-inf with fewer)
    // build diagnostics, reported to FP32 precision (the hardware reciprocal): the relative
    // error of each rescored candidate's fast score, and of each lambda32 entry
    auto rel = [&](double lv, double x) -> double {
        if (lv == 0.0 || !(lv > -__builtin_inf()) || fabs(lv) < 1e-3 * un * M) return 0.0;
        return (double)((float)fabs(x - lv) * __builtin_amdgcn_rcpf((float)fabs(lv)));
    };
    if (FAST || Nk <= 64) {
        // one candidate per lane; the ranks come from a bitonic sort across the wave
        double v = canon_dot_staged<DT>(a, u, su, sid, Nk, rows, udec);
        if (l < Nk) worst_raw = rel(v, (double)ord_f32(skey[l]));
        int idx = l;
#pragma unroll
        for (int kk = 2; kk <= 64; kk <<= 1)
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const double ov = __shfl_xor(v, j);
                const int oi = __shfl_xor(idx, j);
                const bool lower = (l & j) == 0, desc = (l & kk) == 0;
                const bool mine_first = v > ov || (v == ov && idx < oi);
                if (mine_first != (lower == desc)) {
                    v = ov;
                    idx = oi;
                }
            }
        // lane r: the r-th largest canonical score
        for (int r = l; r < a.k_max; r += 64) {
            const double lv = r == l ? v : -__builtin_inf();
            a.lam64[(int64_t)r * a.m + u] = lv;
            a.lam32[(int64_t)r * a.m + u] = (float)lv;
            if (a.lb_rows) a.lb_rows[(int64_t)a.leaf_of[u] * a.k_max + r] = lv / un;
            if (r == l && l < Nk) worst32 = rel(lv, (double)(float)lv);
        }
        lk = a.k_max <= 64 ? __shfl(v, a.k_max - 1) : -__builtin_inf();
    } else if constexpr (!FAST) {
        // 64 candidates at a time through the staged dot products, then a bitonic sort of
        // the scores (padded with -inf to 128 or 256) across the wave: sorted position r
        // (ties: earlier slot first) holds lambda^(r+1)
        for (int j0 = 0; j0 < Nk; j0 += 64) {
            const double x = canon_dot_staged<DT>(a, u, su, sid + j0, Nk - j0, rows, udec);
            if (j0 + l < Nk) {
                s64[j0 + l] = x;
                worst_raw = fmax(worst_raw, rel(x, (double)ord_f32(skey[j0 + l])));
            }
        }
        __builtin_amdgcn_wave_barrier();
        double v[4];
        int ix[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) {
            ix[s4] = 64 * s4 + l;
            v[s4] = ix[s4] < Nk ? s64[ix[s4]] : -__builtin_inf();
        }
        if (Nk <= 128) wave_sort_desc<2>(v, ix);
        else wave_sort_desc<4>(v, ix);
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) {
            const int r = 64 * s4 + l;
            if (r < a.k_max) {
                a.lam64[(int64_t)r * a.m + u] = v[s4];
                a.lam32[(int64_t)r * a.m + u] = (float)v[s4];
                if (a.lb_rows) a.lb_rows[(int64_t)a.leaf_of[u] * a.k_max + r] = v[s4] / un;
                if (r < Nk) worst32 = fmax(worst32, rel(v[s4], (double)(float)v[s4]));
                if (r == a.k_max - 1) lam_row[0] = v[s4];
            }
        }
        __builtin_amdgcn_wave_barrier();
        lk = Nk >= a.k_max ? lam_row[0] : -__builtin_inf();
    }
    worst_raw = wave_max(worst_raw);
    worst32 = wave_max(worst32);
    if (l == 0) {
        const int slot = blockIdx.x % kErrSlots;
        if (worst_raw > 0.0) atomic_max_pos(a.max_raw_err_bits + slot, worst_raw);
        if (worst32 > 0.0) atomic_max_pos(a.max_raw_err_bits + kErrSlots + slot, worst32);
    }
    bool ok = !a.force_fail;
    const float worst_out = fmaxf(tau_max, cut);
    if (ok && worst_out > -__builtin_inff()) {
        const double bound = (double)worst_out + a.err_rel * un * M + (double)a.d * 0x1p-125 * (un + M + 1.0);
        ok = bound <= lk;
    }
    if (!ok && l == 0) {
        const int pos = atomicAdd(a.fail_count, 1);
        a.fail_list[pos] = (int)u;
    }
}

template <int DT, int GPL, bool FAST>
__device__ void refine_user(const RefineArgs& a, int64_t u, uint32_t* skey, uint32_t* sid, double* s64,
                            double* lam_row, int* hist, uint8_t* rows, float* udec)
{
    int Nk = 0;
    float cut = 0.f, tau_max = 0.f;
    if (!refine_select<GPL>(a, u, skey, sid, hist, &Nk, &cut, &tau_max)) return;
    refine_rank<DT, FAST>(a, u, skey, sid, Nk, cut, tau_max, s64, lam_row, rows, udec);
}


// One wave per user (all users, or the users listed in a.list when it is given).  The
// narrow instance (GPL = 8, C <= 64) keeps its state small for occupancy and hands
// users with more than 512 candidates to the wide instance through a.spill.
// The narrow instance is latency bound (several dependent global round trips per user):
// it trades a few spilled registers for six resident waves per SIMD.
template <int DT, int GPL, bool FAST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FAST ? 6 : 2, 8))) void k_refine(RefineArgs a)
{
    __shared__ uint32_t skey[4][FAST ? 64 : 256];
    __shared__ uint32_t sid[4][FAST ? 64 : 256];
    __shared__ double s64[4][FAST ? 1 : 256];
    __shared__ double lam_row[4][1];
    __shared__ int hist_all[4][256];
    __shared__ __attribute__((aligned(16))) uint8_t rows_all[4][64 * RF_PITCH];
    __shared__ __attribute__((aligned(16))) float udec_all[4][DT == DT_FP8 ? 256 : 4];
    const int w = threadIdx.x >> 6;
    if (!a.list) {
        const int64_t u = (int64_t)blockIdx.x * 4 + w;
        if (u < a.m)
            refine_user<DT, GPL, FAST>(a, u, skey[w], sid[w], s64[w], lam_row[w], hist_all[w],
                                       rows_all[w], udec_all[w]);
    } else {
        const int cnt = *a.list_count;
        for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < cnt; i += (int64_t)gridDim.x * 4)
            refine_user<DT, GPL, FAST>(a, a.list[i], skey[w], sid[w], s64[w], lam_row[w],
                                       hist_all[w], rows_all[w], udec_all[w]);
    }
}

// The narrow pass (C <= 64) in two kernels, so that each runs at the occupancy its own
// registers allow: the selection (gather, radix select) and the rescoring (staged FP64
// dot products, ranks, lambda rows, certificate).  The kept candidates go through
// global memory (8 bytes each).
// GPL = 8 for C <= 64, 16 for C <= 224 (users with more candidates than 64 GPL go to
// the wide pass).
template <int GPL, int CMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GPL == 8 ? 6 : 4, 8))) void k_refine_select(RefineArgs a)
{
    __shared__ uint32_t skey_all[4][CMAX], sid_all[4][CMAX];
    __shared__ int hist_all[4][256];
    const int w = threadIdx.x >> 6, l = lane_id();
    const int64_t u = (int64_t)blockIdx.x * 4 + w;
    if (u >= a.m) return;
    int Nk = 0;
    float cut = 0.f, tau_max = 0.f;
    const bool ok = refine_select<GPL>(a, u, skey_all[w], sid_all[w], hist_all[w], &Nk, &cut, &tau_max);
    if (!ok) Nk = -1;
    if (ok)
        for (int j = l; j < Nk; j += 64) a.sel[u * a.C + j] = make_uint2(skey_all[w][j], sid_all[w][j]);
    if (l == 0) {
        int* mt = a.sel_meta + 4 * u;
        mt[0] = Nk;
        mt[1] = __float_as_int(cut);
        mt[2] = __float_as_int(tau_max);
        mt[3] = 0;
    }
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch); the grid is a multiple of 8 and
// each XCD takes a contiguous range of users, so that the lambda rows' lines (16
// consecutive users per 128 bytes) are completed inside one L2 instead of reaching HBM
// as partial lines from several.
__device__ __forceinline__ int64_t xcd_user(int w)
{
    const int64_t per = gridDim.x / 8;
    return ((int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8) * 4 + w;
}

template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_refine_rank(RefineArgs a)
{
    __shared__ uint32_t skey_all[4][64], sid_all[4][64];
    __shared__ __attribute__((aligned(16))) uint8_t rows_all[4][64 * RF_PITCH];
    __shared__ __attribute__((aligned(16))) float udec_all[4][DT == DT_FP8 ? 256 : 4];
    const int w = threadIdx.x >> 6, l = lane_id();
    const int64_t u = xcd_user(w);
    if (u >= a.m) return;
    const int* mt = a.sel_meta + 4 * u;
    const int Nk = mt[0];
    if (Nk < 0) return;   // the wide pass takes this user
    if (l < Nk) {
        const uint2 e = a.sel[u * a.C + l];
        skey_all[w][l] = e.x;
        sid_all[w][l] = e.y;
    }
    __builtin_amdgcn_wave_barrier();
    refine_rank<DT, true>(a, u, skey_all[w], sid_all[w], Nk, __int_as_float(mt[1]), __int_as_float(mt[2]), nullptr,
                          nullptr, rows_all[w], udec_all[w]);
}

// The rescoring of 64 < C <= 224 kept candidates: staged FP64 dot products 64 at a
// time, ranks by a scan over the wave's scores in LDS.
template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_refine_rank_wide(RefineArgs a)
{
    __shared__ uint32_t skey_all[4][224], sid_all[4][224];
    __shared__ double s64_all[4][224];
    __shared__ double lk_all[4][1];
    __shared__ __attribute__((aligned(16))) uint8_t rows_all[4][64 * RF_PITCH];
    __shared__ __attribute__((aligned(16))) float udec_all[4][DT == DT_FP8 ? 256 : 4];
    const int w = threadIdx.x >> 6, l = lane_id();
    const int64_t u = xcd_user(w);
    if (u >= a.m) return;
    const int* mt = a.sel_meta + 4 * u;
    const int Nk = mt[0];
    if (Nk < 0) return;   // the wide pass takes this user
    for (int j = l; j < Nk; j += 64) {
        const uint2 e = a.sel[u * a.C + j];
        skey_all[w][j] = e.x;
        sid_all[w][j] = e.y;
    }
    __builtin_amdgcn_wave_barrier();
    refine_rank<DT, false>(a, u, skey_all[w], sid_all[w], Nk, __int_as_float(mt[1]), __int_as_float(mt[2]),
                           s64_all[w], lk_all[w], rows_all[w], udec_all[w]);
}

template <int DT>
static void refine_d(const RefineArgs& a, hipStream_t s)
{
    if (a.C <= 64) {
        RefineArgs a0 = a;
        a0.list = nullptr;
        if (a.sel) {
            const unsigned g = (unsigned)((a.m + 3) / 4);
            hipLaunchKernelGGL((k_refine_select<8, 64>), dim3(g), dim3(256), 0, s, a0);
            hipLaunchKernelGGL((k_refine_rank<DT>), dim3((g + 7) / 8 * 8), dim3(256), 0, s, a0);
        } else {
            hipLaunchKernelGGL((k_refine<DT, 8, true>), dim3((unsigned)((a.m + 3) / 4)), dim3(256), 0, s, a0);
        }
        if ((int64_t)a.nseg * a.G <= 8 * 64) return;   // no user can hold more than 512
        RefineArgs a1 = a;
        a1.list = a.spill;
        a1.list_count = a.spill_count;
        a1.spill = nullptr;   // the wide instance never spills
        const unsigned g = (unsigned)std::min<int64_t>((a.m + 3) / 4, 1024);
        hipLaunchKernelGGL((k_refine<DT, RF_GPL, false>), dim3(g), dim3(256), 0, s, a1);
    } else if (a.sel) {
        // select (up to 1024 candidates per user) and rescoring in two kernels; users
        // with more candidates go to the wide instance
        RefineArgs a0 = a;
        a0.list = nullptr;
        const unsigned g = (unsigned)((a.m + 3) / 4);
        hipLaunchKernelGGL((k_refine_select<16, 224>), dim3(g), dim3(256), 0, s, a0);
        hipLaunchKernelGGL((k_refine_rank_wide<DT>), dim3((g + 7) / 8 * 8), dim3(256), 0, s, a0);
        if ((int64_t)a.nseg * a.G <= 16 * 64) return;
        RefineArgs a1 = a;
        a1.list = a.spill;
        a1.list_count = a.spill_count;
        a1.spill = nullptr;
        const unsigned g1 = (unsigned)std::min<int64_t>((a.m + 3) / 4, 1024);
        hipLaunchKernelGGL((k_refine<DT, RF_GPL, false>), dim3(g1), dim3(256), 0, s, a1);
    } else {
        RefineArgs a0 = a;
        a0.list = nullptr;
        hipLaunchKernelGGL((k_refine<DT, RF_GPL, false>), dim3((unsigned)((a.m + 3) / 4)), dim3(256), 0, s, a0);
    }
}

void launch_refine(int dtype, const RefineArgs& a, hipStream_t s)
{
    if (a.m <= 0) return;
    if ((int64_t)a.nseg * a.G > RF_MAXN || a.C > 256 || a.nseg > 32)
        fail(RKMIPS_EINVAL, "internal: too many candidates per user");
    if (dtype == DT_F32) refine_d<DT_F32>(a, s);
    else if (dtype == DT_BF16) refine_d<DT_BF16>(a, s);
    else refine_d<DT_FP8>(a, s);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ full FP64 fallback
// Canonical score of the user whose values sit decoded in ux (LDS, exact as floats) against
// item row p, read 16 bytes at a time: index-order FP64 sum of the exact products (FP8:
// a product of two e4m3 values is exact in FP32), then the scale product for FP8.
template <int DT>
__device__ __forceinline__ double canon_dot_row(const float* ux, const void* P, int64_t p, float su, float sp, int d,
                                                int ld)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int PER = 16 / EB;
    const uint8_t* pr = (const uint8_t*)P + p * (int64_t)ld * EB;
    double acc = 0.0;
    for (int c0 = 0; c0 < d; c0 += PER) {
        const i32x4 b4 = *(const i32x4*)(pr + c0 * EB);
        const int lim = d - c0 < PER ? d - c0 : PER;
#pragma unroll
        for (int e = 0; e < PER; e++) {
            if (e >= lim) break;
            const float x = ux[c0 + e];
            if constexpr (DT == DT_F32) {
                acc = __fma_rn((double)x, (double)__int_as_float(b4[e]), acc);
            } else if constexpr (DT == DT_BF16) {
                const float y = bf16_to_f32((uint16_t)((uint32_t)b4[e >> 1] >> (16 * (e & 1))));
                acc = __fma_rn((double)x, (double)y, acc);
            } else {
                const float y = e4m3_to_f32((uint8_t)((uint32_t)b4[e >> 2] >> (8 * (e & 3))));
                acc = acc + (double)(x * y);
            }
        }
    }
    if constexpr (DT == DT_FP8) acc = ((double)su * (double)sp) * acc;
    return acc;
}

template <int DT>
__global__ __launch_bounds__(256) void k_fallback(RefineArgs a, double* scratch, int64_t scratch_rows)
{
    const int64_t nfail = *a.fail_count;   // written by k_refine earlier on the stream
    __shared__ int hist[256];
    __shared__ int s_sel, s_above;
    __shared__ double top[256];
    __shared__ int ntop;
    __shared__ __attribute__((aligned(16))) float ux[256];   // the user's values (d <= ld <= 256)
    const int tid = threadIdx.x;
    for (int64_t fi = blockIdx.x; fi < nfail; fi += gridDim.x) {
        const int64_t u = a.fail_list[fi];
        double* sc = scratch + (int64_t)(blockIdx.x % scratch_rows) * a.n;
        const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
        for (int i = tid; i < a.ld; i += 256) ux[i] = i < a.d ? elem_f32<DT>(a.users, u * (int64_t)a.ld + i) : 0.f;
        __syncthreads();
        for (int64_t p = tid; p < a.n; p += 256) {
            const float sp = DT == DT_FP8 ? a.item_scales[p] : 1.f;
            sc[p] = canon_dot_row<DT>(ux, a.items, p, su, sp, a.d, a.ld);
        }
        __syncthreads();
        const int want = (int)(a.n < a.k_max ? a.n : a.k_max);
        // radix select of the want-th largest (orderable 64-bit keys, 8 digits)
        uint64_t prefix = 0, pmask = 0;
        int need = want;
        for (int shift = 56; shift >= 0; shift -= 8) {
            hist[tid] = 0;
            __syncthreads();
            for (int64_t p = tid; p < a.n; p += 256) {
                const uint64_t k = f64_ord(sc[p]);
                if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 255], 1);
            }
            __syncthreads();
            if (tid == 0) {
                int above = 0;
                for (int b = 255; b >= 0; b--) {
                    if (above < need && need <= above + hist[b]) { s_sel = b; s_above = above; break; }
                    above += hist[b];
                }
            }
            __syncthreads();
            prefix |= (uint64_t)s_sel << shift;
            pmask |= 0xffull << shift;
            need -= s_above;
            __syncthreads();
        }
        const double T = ord_f64(prefix);
        if (tid == 0) ntop = 0;
        __syncthreads();
        for (int64_t p = tid; p < a.n; p += 256)
            if (sc[p] > T) top[atomicAdd(&ntop, 1)] = sc[p];
        __syncthreads();
        const int ng = ntop;   // < want
        for (int j = tid; j < ng; j += 256) {
            int r = 0;
            for (int i = 0; i < ng; i++) r += (top[i] > top[j]) || (top[i] == top[j] && i < j);
            a.lam64[(int64_t)r * a.m + u] = top[j];
            a.lam32[(int64_t)r * a.m + u] = (float)top[j];
            if (a.lb_rows) a.lb_rows[(int64_t)a.leaf_of[u] * a.k_max + r] = top[j] / sqrt(a.user_n2[u]);
            if (top[j] != 0.0)
                atomic_max_pos(a.max_raw_err_bits + kErrSlots + blockIdx.x % kErrSlots,
                               fabs((double)(float)top[j] - top[j]) / fabs(top[j]));
        }
        for (int r = ng + tid; r < a.k_max; r += 256) {
            const double v = r < want ? T : -__builtin_inf();
            a.lam64[(int64_t)r * a.m + u] = v;
            a.lam32[(int64_t)r * a.m + u] = (float)v;
            if (a.lb_rows) a.lb_rows[(int64_t)a.leaf_of[u] * a.k_max + r] = v / sqrt(a.user_n2[u]);
        }
        __syncthreads();
    }
}

void launch_fallback(int dtype, const RefineArgs& a, double* scratch, int64_t scratch_rows, hipStream_t s)
{
    // one workgroup per scratch row; each takes the failed users in turn (none: no work)
    const unsigned g = (unsigned)scratch_rows;
    if (dtype == DT_F32) hipLaunchKernelGGL(k_fallback<DT_F32>, dim3(g), dim3(256), 0, s, a, scratch, scratch_rows);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_fallback<DT_BF16>, dim3(g), dim3(256), 0, s, a, scratch, scratch_rows);
    else hipLaunchKernelGGL(k_fallback<DT_FP8>, dim3(g), dim3(256), 0, s, a, scratch, scratch_rows);
    HIPC(hipGetLastError());
}

}  // namespace rk
