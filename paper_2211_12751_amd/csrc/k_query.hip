// Query side of Alg. 5 with exact decisions, for a batch of queries at once.
//
// k_verify fuses, per (user tile, query sub-tile of 32):
//   * the node-level bound of Lemma 2 per (block, query): ||q|| cos({phi - omega}_+)
//     against L^k(B) (Alg. 5, block test);
//   * the vector-level bound of Lemma 3 per (user, query): ||q|| ||u|| cos|phi - theta_u|
//     against lambda_u^(k) (Alg. 5, user test);
//   * <u, q> on the matrix cores for the pairs that survive, compared with lambda_u^(k)
//     (Alg. 5, inner-product test): a margin beyond the derived error bound decides in
//     the fast arithmetic, anything closer is queued for the canonical FP64 recheck.
// Users stay resident in registers for the whole query chunk, with the blocks' cone
// data and lower bounds in LDS; the next query tile is fetched into registers while
// the current one is scored.  A 32x32 output block whose pairs are all pruned skips
// its matrix-core work.  Answers are compacted with wave prefix sums and reserved with
// one LDS atomic per wave and one global atomic per workgroup and query tile.
//
// Soundness of the bounds under rounding: phi comes from an FP32 dot product whose cosine
// is known within +-e; the bound functions are 1-Lipschitz in the angle, so the angle
// uncertainty Delta_phi is added to the cosine factor; a relative slack covers the
// FP32 evaluation and the stored cos/sin pairs.  Pruning is only ever a strict "<".
#include <algorithm>
#include <climits>
#include <cmath>
#include <utility>

#include "common.h"
#include "dma.h"
#include "internal.h"

namespace rk {

static constexpr int VF_WAVES = 4;
static constexpr int VF_MAXB = 32;     // blocks with angle data per workgroup
static constexpr int VF_MAXSLOT = 8;   // distinct k values per launch

// <u, q> for the wave's 32 users (register fragments) and the 32 queries of the tile.
template <int DT, int KSTEPS, int LROW>
__device__ __forceinline__ f32x16 verify_block(const uint8_t* qt, const i32x4 (&bfrag)[KSTEPS])
{
    const int l = lane_id(), h = l >> 5;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.f;
    const uint8_t* arow = qt + (l & 31) * LROW + h * 16;
#pragma unroll
    for (int t = 0; t < KSTEPS; t++) {
        const i32x4 af = *(const i32x4*)(arow + t * 32);
        if constexpr (DT == DT_F32) {
            const f32x4 a4 = __builtin_bit_cast(f32x4, af);
            const f32x4 b4 = __builtin_bit_cast(f32x4, bfrag[t]);
#pragma unroll
            for (int e = 0; e < 4; e++) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[e], b4[e], acc, 0, 0, 0);
        } else if constexpr (dt_bf16_mma<DT>) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af),
                                                         __builtin_bit_cast(bf16x8, bfrag[t]), acc, 0, 0, 0);
        } else if constexpr (DT == DT_SPLIT) {
            // pair rows [hi | lo]: k-step t of the hi half meets step t + KSTEPS / 2 of the
            // lo half (same elements); q_h.u_h + q_l.u_h + q_h.u_l
            constexpr int HK = KSTEPS / 2;
            if (t < HK) {
                const i32x4 al = *(const i32x4*)(arow + (t + HK) * 32);
                const bf16x8 ah = __builtin_bit_cast(bf16x8, af), alo = __builtin_bit_cast(bf16x8, al);
                const bf16x8 bh = __builtin_bit_cast(bf16x8, bfrag[t]), bl = __builtin_bit_cast(bf16x8, bfrag[t + HK]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
            }
        } else {
            static_assert(dt_bf16_mma<DT>, "FP8 codes reach the matrix cores widened to BF16");
        }
    }
    return acc;
}

// Node-level bound of Lemma 2 for one (block, query) pair from c = cos(phi) (FP32, known
// within +-err_phi): sin(phi), the angle uncertainty dphi and the bound
// ||q|| (cos({phi - omega}_+) + dphi + slack) on <u, q> / ||u|| over the block's users.
struct NodeBound {
    float s, dphi, ub;
};
__device__ __forceinline__ NodeBound node_bound(float c, float qn, float cw, float sw, float err_phi, float slack)
{
    // each operation rounded on its own (no fused multiply-adds), so that every kernel
    // that evaluates the bound takes the same decision
#pragma clang fp contract(off)
    NodeBound nb;
    nb.s = sqrtf(fmaxf(0.f, 1.f - c * c));
    const float ce = fabsf(c) + err_phi;
    const float rem = 1.f - ce * ce;
    nb.dphi = rem > 4.f * err_phi ? err_phi / sqrtf(rem) : 2.f * sqrtf(2.f * err_phi) + err_phi;
    const float fnode = c >= cw ? 1.f : c * cw + nb.s * sw;
    nb.ub = qn * (fnode + nb.dphi + slack);
    return nb;
}

// Inner-product test of one pair: x against lambda with the fast-path error bound
// (relative to ||u|| ||q||): yes beyond +e, no below -e, otherwise a close call for the
// FP64 recheck.
__device__ __forceinline__ void decide(float x, float lam, float uq, bool force, int r, const QueryArgs& a,
                                       uint32_t& yes, uint32_t& amb)
{
    if (lam == -__builtin_inff()) { yes |= 1u << r; return; }
    const float e = (float)a.err_rel * uq + fabsf(lam) * 0x1p-23f + (float)a.d * 0x1p-120f;
    const float diff = x - lam;
    if (force || !(diff > e || diff < -e)) amb |= 1u << r;
    else if (diff > e) yes |= 1u << r;
}

// Waves per SIMD the register budget is cut for: three, except for long fragments
// (FP32 rows of 256, scaled rows of 256 bytes) that would spill, and four for the pair
// rows of split FP32 data.
template <int DT, int DPT>
constexpr int verify_wpe()
{
    if (DT == DT_SPLIT) return 4;   // pair rows: eight resident fragments
    return (DT == DT_F32 && DPT >= 256) ? 1
                                          : ((DPT * Elt<DT>::bytes >= 384 || (dt_scaled<DT> && DPT * Elt<DT>::bytes >= 256)) ? 2 : 3);
}

template <int DT, int DPT, int UBW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(verify_wpe<DT, DPT>(), 8))) void k_verify(QueryArgs a, int64_t q_begin, int64_t q_end)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int ROWB = DPT * EB;
    constexpr int LROW = ROWB + 16;
    constexpr int KSTEPS = ROWB / 32;
    constexpr int UT = VF_WAVES * UBW * 32;
    constexpr int CH = 32 * (ROWB / 16);      // 16-byte chunks of one query tile
    constexpr int PF = (CH + 255) / 256;
    constexpr bool PREFETCH = PF <= 4;
    __shared__ __attribute__((aligned(16))) uint8_t qt[32 * LROW];
    __shared__ float qn_s[32], qs_s[32];
    __shared__ int qslot_s[32];
    __shared__ f32x4 phi_s[VF_MAXB][32];
    __shared__ float lam_s[VF_MAXSLOT][UT];
    __shared__ float bcw[VF_MAXB], bsw[VF_MAXB];
    __shared__ int bok[VF_MAXB];
    __shared__ float blb[VF_MAXSLOT][VF_MAXB];
    __shared__ unsigned int cnt_s[2];
    __shared__ uint32_t live_q[VF_MAXB];   // per block: queries of the tile not pruned by Lemma 2
    __shared__ unsigned long long base_s[2];
    // "yes" answers are staged here and reserved in the global pool once per stage-full
    // (one contended atomic per workgroup and flush instead of per tile)
    constexpr int YS = 1024;
    __shared__ unsigned long long ystage[YS];
    __shared__ unsigned int ycnt;
    __shared__ unsigned long long st_s[4];

    const int l = lane_id(), w = threadIdx.x >> 6, h = l >> 5;
    const int64_t u0 = (int64_t)blockIdx.x * UT;
    const int64_t ulast = (u0 + UT - 1 < a.m - 1) ? u0 + UT - 1 : a.m - 1;
    const int bfirst = a.user_block[u0];
    const int nb = a.user_block[ulast] - bfirst + 1;
    const int nbb = nb < VF_MAXB ? nb : VF_MAXB;
    const bool use_bounds = !(a.flags & RKMIPS_FLAG_NO_BOUNDS);
    const bool use_vec = use_bounds && !(a.flags & RKMIPS_FLAG_NO_VECTOR_BOUND);
    const bool force = (a.flags & RKMIPS_FLAG_FORCE_RECHECK) != 0;

    // ---- per-workgroup tables: lambda rows of the k slots, the blocks' cone data and
    // lower bounds (the user tile and its blocks are fixed for the whole launch)
    for (int e = threadIdx.x; e < a.nslots * UT; e += 256) {
        const int sl = e / UT, ul = e % UT;
        const int64_t u = u0 + ul;
        lam_s[sl][ul] = u < a.m ? a.lam32[(int64_t)(a.slot_k[sl] - 1) * a.m + a.perm[u]] : 0.f;
    }
    for (int b = threadIdx.x; b < nbb; b += 256) {
        const int bg = bfirst + b;
        bok[b] = use_bounds && a.block_ok[bg];
        bcw[b] = a.cos_w[bg];
        bsw[b] = a.sin_w[bg];
    }
    for (int e = threadIdx.x; e < a.nslots * nbb; e += 256) {
        const int sl = e / nbb, b = e % nbb;
        blb[sl][b] = a.block_lb[(int64_t)(a.slot_k[sl] - 1) * a.nblocks + bfirst + b];
    }

    i32x4 bfrag[UBW][KSTEPS];
    float un[UBW], ct[UBW], st[UBW], su[UBW];
    int bl[UBW], ul_[UBW];
    uint32_t ouid[UBW];
    bool uok[UBW];
#pragma unroll
    for (int cb = 0; cb < UBW; cb++) {
        ul_[cb] = (w * UBW + cb) * 32 + (l & 31);
        const int64_t u = u0 + ul_[cb];
        uok[cb] = u < a.m;
        const int64_t uu = uok[cb] ? u : u0;
        const uint8_t* row = (const uint8_t*)a.mma_users + uu * ROWB;
#pragma unroll
        for (int t = 0; t < KSTEPS; t++) {
            i32x4 z = {0, 0, 0, 0};
            bfrag[cb][t] = uok[cb] ? *(const i32x4*)(row + t * 32 + h * 16) : z;
        }
        un[cb] = a.unorm[uu];
        ct[cb] = a.cos_t[uu];
        st[cb] = a.sin_t[uu];
        su[cb] = dt_scaled<DT> ? a.user_scales[uu] : 1.f;
        bl[cb] = a.user_block[uu] - bfirst;
        ouid[cb] = a.perm[uu];
    }

    // ---- query tiles: registers hold the next tile while the current one is scored
    auto load_chunk = [&](int64_t qb, int c) -> i32x4 {
        const int r = c / (ROWB / 16), c16 = c % (ROWB / 16);
        const int64_t q = qb + r;
        i32x4 v = {0, 0, 0, 0};
        if (c < CH && q < q_end) v = *(const i32x4*)((const uint8_t*)a.mma_queries + q * ROWB + c16 * 16);
        return v;
    };
    i32x4 pf[PREFETCH ? PF : 1];
    float pqn = 0.f, pqs = 1.f;
    int pqsl = 0;
    // cos(phi) of the tile's (block, query) entries threadIdx.x and threadIdx.x + 256, loaded
    // one tile ahead with the query rows (entries past 512 are read when used)
    float pc[2] = {1.f, 1.f};
    auto prefetch = [&](int64_t qb) {
        if constexpr (PREFETCH) {
#pragma unroll
            for (int e = 0; e < PF; e++) pf[e] = load_chunk(qb, threadIdx.x + 256 * e);
        }
        if (threadIdx.x < 32) {
            const int64_t q = qb + threadIdx.x;
            const bool ok = q < q_end;
            pqn = ok ? a.qnorm[q] : 0.f;
            pqs = (ok && dt_scaled<DT>) ? a.query_scales[q] : 1.f;
            pqsl = ok ? a.qslot[q] : 0;
        }
        if (use_bounds) {
#pragma unroll
            for (int i = 0; i < 2; i++) {
                const int e = threadIdx.x + 256 * i;
                if (e < nbb * 32 && qb + (e & 31) < q_end)
                    pc[i] = a.cphi[(int64_t)(bfirst + (e >> 5)) * a.nq + qb + (e & 31)];
            }
        }
    };
    prefetch(q_begin);
    if (threadIdx.x == 0) ycnt = 0u;
    if (threadIdx.x < 4) st_s[threadIdx.x] = 0ull;

    unsigned long long n_node = 0, n_vec = 0, n_scored = 0, n_amb = 0;

    for (int64_t qb = q_begin; qb < q_end; qb += 32) {
        __syncthreads();
        if constexpr (PREFETCH) {
#pragma unroll
            for (int e = 0; e < PF; e++) {
                const int c = threadIdx.x + 256 * e;
                if (c < CH) *(i32x4*)(qt + (c / (ROWB / 16)) * LROW + (c % (ROWB / 16)) * 16) = pf[e];
            }
        } else {
            for (int c = threadIdx.x; c < CH; c += 256)
                *(i32x4*)(qt + (c / (ROWB / 16)) * LROW + (c % (ROWB / 16)) * 16) = load_chunk(qb, c);
        }
        if (threadIdx.x < 32) {
            qn_s[threadIdx.x] = pqn;
            qs_s[threadIdx.x] = pqs;
            qslot_s[threadIdx.x] = pqsl;
        }
        if (threadIdx.x == 0) {
            cnt_s[0] = 0u;
            cnt_s[1] = 0u;
        }
        if (threadIdx.x < VF_MAXB) live_q[threadIdx.x] = 0u;
        __syncthreads();
        const float pc0 = pc[0], pc1 = pc[1];   // this tile's; the prefetch below reloads them
        if (qb + 32 < q_end) prefetch(qb + 32);

        // node-level data per (block, query): cos(phi) from the pre-pass, the rest here
        for (int e = threadIdx.x; e < nbb * 32; e += 256) {
            const int b = e >> 5, qi = e & 31;
            f32x4 out = {1.f, 0.f, 0.f, 2.f};     // w = 2: no angle data, never prune
            if (bok[b] && qb + qi < q_end && qn_s[qi] > 0.f) {
                const float c = e < 256 ? pc0 : e < 512 ? pc1 : a.cphi[(int64_t)(bfirst + b) * a.nq + qb + qi];
                const NodeBound nd = node_bound(c, qn_s[qi], bcw[b], bsw[b], a.err_phi, a.bound_slack);
                out = f32x4{c, nd.s, nd.dphi, nd.ub < blb[qslot_s[qi]][b] ? 1.f : 0.f};
            }
            phi_s[b][qi] = out;
            if (out[3] != 1.f && qb + qi < q_end) atomicOr(&live_q[b], 1u << qi);
        }
        __syncthreads();

        uint32_t yes = 0u, amb = 0u;
        const int ul = ul_[0];
        const int blk = bl[0];
        if constexpr (DT == DT_F32) {
            // FP32: the bounds first, so a 32 x 32 tile whose pairs are all pruned skips its
            // (comparatively costly) matrix-core work
            uint32_t live = 0u;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int qi = mfma32_row(r, l);
                if (!uok[0] || qb + qi >= q_end) continue;
                const f32x4 ph = blk < VF_MAXB ? phi_s[blk][qi] : f32x4{1.f, 0.f, 0.f, 2.f};
                if (ph[3] == 1.f) { n_node++; continue; }
                if (use_vec && ph[3] == 0.f) {
                    const float lam = lam_s[qslot_s[qi]][ul];
                    const float ubv = qn_s[qi] * un[0] * (ph[0] * ct[0] + ph[1] * st[0] + ph[2] + a.bound_slack);
                    if (ubv < lam - fabsf(lam) * 0x1p-22f) { n_vec++; continue; }
                }
                live |= 1u << r;
            }
            if (ballot64(live != 0u)) {
                const f32x16 acc = verify_block<DT, KSTEPS, LROW>(qt, bfrag[0]);
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    if (!(live & (1u << r))) continue;
                    const int qi = mfma32_row(r, l);
                    const float lam = lam_s[qslot_s[qi]][ul];
                    decide(acc[r], lam, un[0] * qn_s[qi], force, r, a, yes, amb);
                }
                n_scored += __popc(live);
                n_amb += __popc(amb);
            }
        } else {
            // narrow types: the matrix cores cost less than any per-pair bound, so every
            // tile with a query the node-level test leaves alive is multiplied and the
            // inner-product test decides each of its pairs directly (for a multiplied pair
            // the vector-level bound of Lemma 3 could only repeat what the product shows).
            const int nvalid = (int)((q_end - qb) < 32 ? (q_end - qb) : 32);
            const uint32_t vmask = nvalid == 32 ? 0xffffffffu : ((1u << nvalid) - 1u);
            const uint32_t hmask = 0x0f0f0f0fu << (4 * h);   // the lane's 16 rows
            const uint32_t qlive = uok[0] ? (blk < VF_MAXB ? live_q[blk] : vmask) : 0u;
            if (uok[0]) n_node += __popc(vmask & hmask & ~qlive);
            if (ballot64(qlive != 0u)) {
                const f32x16 acc = verify_block<DT, KSTEPS, LROW>(qt, bfrag[0]);
                const uint32_t mine = qlive & hmask;
                n_scored += __popc(mine);
                // queries arrive sorted by k: a tile usually has one k slot, whose lambda
                // terms then stay in registers
                const int sl0 = qslot_s[0], sl1 = qslot_s[nvalid - 1];
                // (err_rel widened by 2^-20 so the regrouped FP32 product cannot undercut it)
                const float uerr = (float)(a.err_rel * (1.0 + 0x1p-20)) * un[0];
                // bit r of on16: the lane's row r (query mfma32_row(r, l)) is live
                const uint32_t mh = mine >> (4 * h);
                const uint32_t on16 = (mh & 0xfu) | ((mh >> 4) & 0xf0u) | ((mh >> 8) & 0xf00u) | ((mh >> 12) & 0xf000u);
                if (sl0 == sl1) {
                    // yes beyond +e, a close call within +-e, no below -e; with lambda = -inf
                    // every difference is +inf, so every live query is a yes
                    const float lam = lam_s[sl0][ul];
                    const bool lam_inf = lam == -__builtin_inff();
                    const float elam = (lam_inf ? 0.f : fabsf(lam) * 0x1p-23f) + (float)a.d * 0x1p-120f;
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        const int qi = mfma32_row(r, l);
                        float x = acc[r];
                        if constexpr (dt_scaled<DT>) x = (su[0] * qs_s[qi]) * x;
                        const float e = fmaf(uerr, qn_s[qi], elam);
                        const float diff = x - lam;
                        yes |= (uint32_t)(diff > e) << r;
                        amb |= (uint32_t)(fabsf(diff) <= e) << r;
                    }
                    yes &= on16;
                    amb &= on16;
                    if (force) {
                        yes = lam_inf ? on16 : 0u;
                        amb = lam_inf ? 0u : on16;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        const int qi = mfma32_row(r, l);
                        const float lam = lam_s[qslot_s[qi]][ul];
                        float x = acc[r];
                        if constexpr (dt_scaled<DT>) x = (su[0] * qs_s[qi]) * x;
                        const bool li = lam == -__builtin_inff();
                        const float e = fmaf(uerr, qn_s[qi], (li ? 0.f : fabsf(lam) * 0x1p-23f) + (float)a.d * 0x1p-120f);
                        const float diff = x - lam;
                        yes |= (uint32_t)(li || (!force && diff > e)) << r;
                        amb |= (uint32_t)(!li && (force || fabsf(diff) <= e)) << r;
                    }
                    yes &= on16;
                    amb &= on16;
                }
                n_amb += __popc(amb);
            }
        }

        if (a.sah) {   // SAH: every pair the test does not reject goes on to the recheck
            n_amb += __popc(yes);
            amb |= yes;
            yes = 0u;
        }
        if (a.bitmap) {   // yes answers as bits (workgroup-uniform); the pool takes close calls only
#pragma unroll
            for (int r = 0; r < 16; r++)
                if (yes & (1u << r)) {
                    const int64_t q = qb + mfma32_row(r, l);
                    atomicOr(&a.bitmap[(int64_t)a.qorig[q] * a.bm_words + (ouid[0] >> 5)], 1u << (ouid[0] & 31u));
                }
            yes = 0u;
        }
        // ---- appends: wave prefix sums, one LDS reservation per wave, one global
        // reservation per workgroup and tile
        const int ny = __popc(yes), na = __popc(amb);
        const int iy = wave_incl_scan(ny), ia = wave_incl_scan(na);
        const int ty = __shfl(iy, 63), ta = __shfl(ia, 63);
        unsigned int wy = 0u, wa = 0u;
        if (l == 0) {
            if (ty) wy = atomicAdd(&cnt_s[0], (unsigned int)ty);
            if (ta) wa = atomicAdd(&cnt_s[1], (unsigned int)ta);
        }
        wy = __shfl(wy, 0);
        wa = __shfl(wa, 0);
        __syncthreads();
        const unsigned int T = cnt_s[0];            // yes answers of this tile
        const unsigned int y0 = ycnt;                // staged before it
        const bool direct = T > (unsigned int)YS;    // too many for the stage: reserve now
        const bool flush = !direct && y0 + T > (unsigned int)YS;
        if (threadIdx.x == 0) {
            unsigned long long b = 0ull;
            if (direct) b = atomicAdd(a.pool_count, (unsigned long long)T);
            else if (flush) b = atomicAdd(a.pool_count, (unsigned long long)y0);
            base_s[0] = b;
            base_s[1] = cnt_s[1] ? atomicAdd(a.amb_count, (unsigned long long)cnt_s[1]) : 0ull;
        }
        __syncthreads();
        if (flush) {   // workgroup-uniform
            for (unsigned int i = threadIdx.x; i < y0; i += 256) {
                const unsigned long long pos = base_s[0] + i;
                if ((int64_t)pos < a.pool_cap) a.pool[pos] = ystage[i];
            }
            __syncthreads();
        }
        const unsigned int ybase = flush ? 0u : y0;
        if (ty | ta) {
            int64_t py = direct ? (int64_t)base_s[0] + wy + iy - ny : (int64_t)ybase + wy + iy - ny;
            int64_t pa = (int64_t)base_s[1] + wa + ia - na;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int64_t q = qb + mfma32_row(r, l);
                if (yes & (1u << r)) {
                    const unsigned long long e = ((unsigned long long)a.qorig[q] << 32) | ouid[0];
                    if (direct) {
                        if (py < a.pool_cap) a.pool[py] = e;
                    } else {
                        ystage[py] = e;
                    }
                    py++;
                }
                if (amb & (1u << r)) {
                    if (pa < a.amb_cap) a.amb[pa] = ((unsigned long long)q << 32) | (uint32_t)(u0 + ul_[0]);
                    pa++;
                }
            }
        }
        if (threadIdx.x == 0) ycnt = direct ? y0 : ybase + T;
    }
    // the rest of the stage
    __syncthreads();
    const unsigned int yl = ycnt;
    if (yl) {
        if (threadIdx.x == 0) base_s[0] = atomicAdd(a.pool_count, (unsigned long long)yl);
        __syncthreads();
        for (unsigned int i = threadIdx.x; i < yl; i += 256) {
            const unsigned long long pos = base_s[0] + i;
            if ((int64_t)pos < a.pool_cap) a.pool[pos] = ystage[i];
        }
    }
    n_node = wave_sum(n_node);
    n_vec = wave_sum(n_vec);
    n_scored = wave_sum(n_scored);
    n_amb = wave_sum(n_amb);
    if (l == 0) {
        if (n_node) atomicAdd(&st_s[0], n_node);
        if (n_vec) atomicAdd(&st_s[1], n_vec);
        if (n_scored) atomicAdd(&st_s[2], n_scored);
        if (n_amb) atomicAdd(&st_s[3], n_amb);
    }
    __syncthreads();
    if (threadIdx.x < 4 && st_s[threadIdx.x]) atomicAdd(&a.stats[threadIdx.x], st_s[threadIdx.x]);
}

// ------------------------------------------------------------------ ring form
// BF16 operands (BF16 data, widened FP8 codes) with rows of 256 bytes and more, and the
// BF16 pair rows of split FP32 data with d <= 64 (256 bytes).  A wave
// holds two groups of 32 users in registers, so that every query fragment read from LDS
// feeds two products; a workgroup holds 256 users.  The query tiles (32 rows at the
// absolute positions 32 T .. 32 T + 31; rows outside the launch's range are loaded and
// masked) reach LDS by direct loads into a ring of three padded buffers, two tiles ahead
// of the one being scored, together with the tile's per-query data (norm, scale, k slot,
// caller index) and the Lemma 2 prune words of the workgroup's first 64 blocks (written
// by k_phi; users of later blocks are never pruned).  One barrier per tile.  Each wave
// stages its yes answers in LDS and reserves pool space once per stage-full, and a wave
// with close calls reserves their slots itself, so no step waits for the other waves.
// The products (same operands, same k order) and the inner-product test are those of
// k_verify, so both forms take the same decisions.
static constexpr int VR_UPB = 256;   // users per workgroup
static constexpr int VR_SW = 128;    // yes answers staged per wave
static constexpr int VR_HQ = 320;    // per-tile words: norms, scales, slots, prune words, caller indexes

template <int DT, int KSTEPS, int LROW>
__device__ __forceinline__ void ring_block(const uint8_t* tile, const i32x4 (&bfrag)[2][KSTEPS], f32x16 (&acc)[2])
{
    const int l = lane_id(), h = l >> 5;
#pragma unroll
    for (int g = 0; g < 2; g++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[g][r] = 0.f;
    const uint8_t* arow = tile + (l & 31) * LROW + h * 16;
    if constexpr (DT == DT_SPLIT) {
        // pair rows [hi | lo]: k-step t of the hi half meets step t + KSTEPS / 2 of the lo
        // half; q_h u_h + q_l u_h + q_h u_l in the one-group kernel's order
        constexpr int HK = KSTEPS / 2;
#pragma unroll
        for (int t = 0; t < HK; t++) {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const i32x4*)(arow + t * 32));
            const bf16x8 al = __builtin_bit_cast(bf16x8, *(const i32x4*)(arow + (t + HK) * 32));
#pragma unroll
            for (int g = 0; g < 2; g++) {
                const bf16x8 bh = __builtin_bit_cast(bf16x8, bfrag[g][t]);
                const bf16x8 bl = __builtin_bit_cast(bf16x8, bfrag[g][t + HK]);
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[g], 0, 0, 0);
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[g], 0, 0, 0);
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[g], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < KSTEPS; t++) {
            const bf16x8 af = __builtin_bit_cast(bf16x8, *(const i32x4*)(arow + t * 32));
#pragma unroll
            for (int g = 0; g < 2; g++)
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, __builtin_bit_cast(bf16x8, bfrag[g][t]), acc[g], 0, 0, 0);
        }
        // schedule: the first three fragment reads, then per k-step two products and the
        // read three steps ahead (left alone, the scheduler keeps two reads in flight and
        // each pair of k-steps waits for LDS)
        __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
        for (int t = 0; t < KSTEPS - 3; t++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
    }
}

template <int DT, int DPT>
constexpr int verify_ring_wpe()
{
    return 2;
}

// Grid: (user tile, chunk) pairs, chunk-major; chunk c covers the range's tiles
// [c per, (c + 1) per) (relative to the first).
template <int DT, int DPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(verify_ring_wpe<DT, DPT>(), 8))) void k_verify_ring(QueryArgs a, int64_t q_first, int64_t q_last, int64_t per, int64_t wgs)
{
    static_assert(dt_bf16_mma<DT> || DT == DT_SPLIT, "the ring form takes BF16 operands");
    constexpr int NG = 2;
    constexpr int UPW = 32 * NG;
    constexpr int ROWB = DPT * Elt<DT>::bytes;
    constexpr int LROW = ROWB + 16;               // padded LDS row (bank spread)
    constexpr int CPR = LROW / 16;
    constexpr int KSTEPS = ROWB / 32;
    constexpr int NLD = (32 * LROW + 1023) / 1024;   // 1 KB direct loads per tile
    constexpr int LPW = (NLD + 3) / 4;
    constexpr int TBYTES = NLD * 1024;
    constexpr bool SC = dt_scaled<DT>;
    __shared__ __attribute__((aligned(1024))) uint8_t ring_all[3 * TBYTES];
    // per tile: [0, 64) query norms, [64, 128) scales, [128, 192) k slots, [192, 256) prune
    // words by block (relative to the workgroup's first), [256, 320) caller indexes
    __shared__ __attribute__((aligned(256))) uint32_t hq_all[3 * VR_HQ];
    __shared__ float lam_s[VF_MAXSLOT][VR_UPB];
    // per user of the workgroup: original index, block relative to the first (the loop
    // reads them from here: registers are scarce, and a spill reload would make the
    // compiler wait for the tile loads in flight)
    __shared__ uint32_t ouid_s[VR_UPB];
    __shared__ int br_s[VR_UPB];
    __shared__ unsigned long long ystage_all[4][VR_SW];
    __shared__ unsigned long long st_s[4];
    __shared__ uint32_t doff_all[4][LPW][64];   // each lane's direct-load offsets (fixed)

    const int l = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (SGPR)
    const int h = l >> 5;
    unsigned long long* ystage = ystage_all[w];
    const int64_t chunk = (int64_t)blockIdx.x / wgs;
    const int64_t u0 = ((int64_t)blockIdx.x - chunk * wgs) * VR_UPB;
    const int64_t tb = ((q_first >> 5) + chunk * per) * 32;
    const int64_t q_begin = q_first > tb ? q_first : tb;
    const int64_t q_end = q_last < tb + per * 32 ? q_last : tb + per * 32;
    const bool use_bounds = !(a.flags & RKMIPS_FLAG_NO_BOUNDS) && a.prune != nullptr;
    const bool force = (a.flags & RKMIPS_FLAG_FORCE_RECHECK) != 0;

    // lambda rows of the k slots (fixed for the launch)
    for (int e = threadIdx.x; e < a.nslots * VR_UPB; e += 256) {
        const int sl = e / VR_UPB, ul = e % VR_UPB;
        const int64_t u = u0 + ul;
        lam_s[sl][ul] = u < a.m ? a.lam32[(int64_t)(a.slot_k[sl] - 1) * a.m + a.perm[u]] : 0.f;
    }
    if (threadIdx.x < 4) st_s[threadIdx.x] = 0ull;
    const int bfirst = a.user_block[u0];
    const int nbw = (int)(a.nblocks - bfirst < 64 ? a.nblocks - bfirst : 64);

    // ---- resident user fragments (B operands), one user column per lane and group
    i32x4 bfrag[NG][KSTEPS];
    float su[NG], uerr[NG];
    bool uok[NG];
#pragma unroll
    for (int g = 0; g < NG; g++) {
        const int64_t u = u0 + w * UPW + g * 32 + (l & 31);
        uok[g] = u < a.m;
        const int64_t uu = uok[g] ? u : u0;
        const uint8_t* row = (const uint8_t*)a.mma_users + uu * ROWB;
#pragma unroll
        for (int t = 0; t < KSTEPS; t++) {
            i32x4 z = {0, 0, 0, 0};
            bfrag[g][t] = uok[g] ? *(const i32x4*)(row + t * 32 + h * 16) : z;
        }
        su[g] = SC ? a.user_scales[uu] : 1.f;
        // (err_rel widened by 2^-20 so the regrouped FP32 product cannot undercut it)
        uerr[g] = (float)(a.err_rel * (1.0 + 0x1p-20)) * a.unorm[uu];
        if (h == 0) {
            br_s[w * UPW + g * 32 + (l & 31)] = a.user_block[uu] - bfirst;
            ouid_s[w * UPW + g * 32 + (l & 31)] = a.perm[uu];
        }
    }

    const int64_t T0 = q_begin >> 5;
    const int ntiles = (int)(((q_end + 31) >> 5) - T0);
    const uint32_t pbytes = use_bounds ? (uint32_t)nbw * (uint32_t)a.ntq * 4u : 0u;
    const uint32_t* pbase = use_bounds ? a.prune + (int64_t)bfirst * a.ntq : (const uint32_t*)a.qnorm;

    // ---- direct loads: load j of this wave fills LDS bytes [k * 1024, (k + 1) * 1024) of
    // a slot, k = w * LPW + j; lane l writes 16 bytes at k * 1024 + 16 l, which is chunk
    // (pos % CPR) of padded row pos / CPR (the padding chunk takes a copy of chunk 0).
    // The offsets are the same for every tile: kept in LDS, not in registers.
#pragma unroll
    for (int j = 0; j < LPW; j++) {
        const unsigned pos = (unsigned)(w * LPW * 64 + l) + (unsigned)j * 64u;
        const unsigned c = pos % (unsigned)CPR;
        doff_all[w][j][l] = (pos / (unsigned)CPR) * (unsigned)ROWB + (c < (unsigned)(ROWB / 16) ? c : 0u) * 16u;
    }
    auto issue = [&](uint8_t* ring, uint32_t* hq, int tt) {
        const int64_t T = T0 + tt;
        const int64_t r0 = T * 32;
        const int rows = q_end - r0 < 32 ? (int)(q_end - r0) : 32;
        // rows past the launch's last query read as zeros
        const dma_rsrc rs = dma_buffer((const uint8_t*)a.mma_queries + r0 * ROWB, (uint32_t)(rows * ROWB));
        const uint32_t lb = RK_LDS_ADDR(ring);
        // all offsets read before the first load: the loads' asm blocks order every later
        // LDS read behind them
        uint32_t dv[LPW];
#pragma unroll
        for (int j = 0; j < LPW; j++) dv[j] = doff_all[w][j][l];
#pragma unroll
        for (int j = 0; j < LPW; j++)
            if (w * LPW + j < NLD) dma_load16(rs, lb + (uint32_t)((w * LPW + j) * 1024), dv[j]);
        if (w == 0) {
            const uint32_t hb = RK_LDS_ADDR(hq);
            const uint32_t qb4 = (uint32_t)(rows * 4);
            dma_load4(dma_buffer(a.qnorm + r0, qb4), hb, (uint32_t)(l * 4));
            if constexpr (SC) dma_load4(dma_buffer(a.query_scales + r0, qb4), hb + 256u, (uint32_t)(l * 4));
            dma_load4(dma_buffer(a.qslot + r0, qb4), hb + 512u, (uint32_t)(l * 4));
            // lane i: the word of block bfirst + i (lanes past the staged blocks read 0)
            uint32_t lt = (uint32_t)l;
            asm volatile("" : "+v"(lt));   // recomputed per tile, not kept live
            dma_load4(dma_buffer(pbase, pbytes), hb + 768u, (lt * (uint32_t)a.ntq + (uint32_t)T) * 4u);
            dma_load4(dma_buffer(a.qorig + r0, qb4), hb + 1024u, (uint32_t)(l * 4));
        }
    };
    // Before tile tt is read: this wave's loads of tile tt have landed when no more than
    // its loads of tile tt + 1 (if issued) are in flight; anything issued after those
    // (answer stores) only makes the wait stricter.  Wave 0 also loads the per-query data.
    auto wait_tile = [&](bool next_issued) {
        constexpr int n0 = (NLD < LPW ? NLD : LPW) + (SC ? 5 : 4);
        constexpr int n1 = NLD - LPW <= 0 ? 0 : (NLD - LPW < LPW ? NLD - LPW : LPW);
        constexpr int n2 = NLD - 2 * LPW <= 0 ? 0 : (NLD - 2 * LPW < LPW ? NLD - 2 * LPW : LPW);
        constexpr int n3 = NLD - 3 * LPW <= 0 ? 0 : (NLD - 3 * LPW < LPW ? NLD - 3 * LPW : LPW);
        static_assert(n0 < 64, "wait counts");
        if (!next_issued) RK_WAIT_VMCNT(0);
        else if (w == 0) RK_WAIT_VMCNT(n0);
        else if (w == 1) RK_WAIT_VMCNT(n1);
        else if (w == 2) RK_WAIT_VMCNT(n2);
        else RK_WAIT_VMCNT(n3);
    };

    uint32_t n_node = 0u, n_scored = 0u, n_amb = 0u;
    int ycnt = 0;   // yes answers staged by this wave (wave-uniform)
    auto flush = [&]() {
        if (ycnt == 0) return;
        unsigned long long b = 0ull;
        if (l == 0) b = atomicAdd(a.pool_count, (unsigned long long)ycnt);
        b = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
            __builtin_amdgcn_readfirstlane((uint32_t)b);
        __builtin_amdgcn_wave_barrier();
        for (int i = l; i < ycnt; i += 64)
            if ((int64_t)(b + i) < a.pool_cap) a.pool[b + i] = ystage[i];
        __builtin_amdgcn_wave_barrier();
        ycnt = 0;
    };

    auto tile = [&](const uint8_t* ring, const uint32_t* hq, int tt) {
        const int64_t r0 = (T0 + tt) * 32;
        const int lo = r0 < q_begin ? (int)(q_begin - r0) : 0;
        const int hi = q_end - r0 < 32 ? (int)(q_end - r0) : 32;
        const uint32_t vmask = (hi == 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        // lane terms recomputed per tile (opaque to the compiler): hoisted out of the
        // loop, the row and user indexes of every output would be kept live, and spill
        int h4 = 4 * h, lc = l & 31;
        asm volatile("" : "+v"(h4), "+v"(lc));
        const uint32_t hmask = 0x0f0f0f0fu << h4;   // the lane's 16 rows
        auto row_of = [&](int r) -> int { return ((r >> 2) << 3) + h4 + (r & 3); };
        uint32_t qlive[NG];
#pragma unroll
        for (int g = 0; g < NG; g++) {
            const int br = br_s[w * UPW + g * 32 + lc];
            const uint32_t pw = br < 64 ? hq[192 + br] : 0u;
            qlive[g] = uok[g] ? (vmask & ~pw) : 0u;
            if (uok[g]) n_node += __popc(vmask & hmask & ~qlive[g]);
        }
        uint32_t yes[NG] = {0u, 0u}, amb[NG] = {0u, 0u};
        if (ballot64((qlive[0] | qlive[1]) != 0u)) {
            f32x16 acc[NG];
            ring_block<DT, KSTEPS, LROW>(ring, bfrag, acc);
            const float* hf = (const float*)hq;
            // bit r of on16: the lane's row r (query mfma32_row(r, l)) is live
            uint32_t on16[NG];
#pragma unroll
            for (int g = 0; g < NG; g++) {
                const uint32_t mine = qlive[g] & hmask;
                n_scored += __popc(mine);
                const uint32_t mh = mine >> h4;
                on16[g] = (mh & 0xfu) | ((mh >> 4) & 0xf0u) | ((mh >> 8) & 0xf00u) | ((mh >> 12) & 0xf000u);
            }
            // queries arrive sorted by k: a tile usually has one k slot
            const int sl0 = (int)(hq[128 + lo] & 7u), sl1 = (int)(hq[128 + hi - 1] & 7u);
            if (sl0 == sl1) {
                // yes beyond +e, a close call within +-e, no below -e; with lambda = -inf
                // every difference is +inf, so every live query is a yes
                float lam[NG], elam[NG];
                bool linf[NG];
#pragma unroll
                for (int g = 0; g < NG; g++) {
                    lam[g] = lam_s[sl0][w * UPW + g * 32 + lc];
                    linf[g] = lam[g] == -__builtin_inff();
                    elam[g] = (linf[g] ? 0.f : fabsf(lam[g]) * 0x1p-23f) + (float)a.d * 0x1p-120f;
                }
                // Screen: a pair is a yes or a close call only if x - lambda >= -e.  The
                // screen evaluates x - lambda + 8 e in one rounded step per term; its error
                // (a few units in the last place of |x| + |lambda|) stays below the extra
                // 7 e, as e >= |lambda| 2^-23, so a wave whose pairs all fail it has only
                // "no" answers and skips the test itself (lambda = -inf gives +inf).
                float mx = -__builtin_inff();
                {
                    float u8[NG], c8[NG];
#pragma unroll
                    for (int g = 0; g < NG; g++) {
                        u8[g] = 8.f * uerr[g];
                        c8[g] = 8.f * elam[g] - lam[g];
                    }
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const f32x4 qn4 = *(const f32x4*)(hf + 8 * j + h4);
                        f32x4 qs4 = {1.f, 1.f, 1.f, 1.f};
                        if constexpr (SC) qs4 = *(const f32x4*)(hf + 64 + 8 * j + h4);
#pragma unroll
                        for (int g = 0; g < NG; g++)
#pragma unroll
                            for (int e = 0; e < 4; e++) {
                                const float b = fmaf(u8[g], qn4[e], c8[g]);
                                const float t = SC ? fmaf(acc[g][4 * j + e], su[g] * qs4[e], b) : acc[g][4 * j + e] + b;
                                mx = fmaxf(mx, t);
                            }
                    }
                }
                if (force || ballot64(mx >= 0.f)) {
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const f32x4 qn4 = *(const f32x4*)(hf + 8 * j + h4);
                        f32x4 qs4 = {1.f, 1.f, 1.f, 1.f};
                        if constexpr (SC) qs4 = *(const f32x4*)(hf + 64 + 8 * j + h4);
#pragma unroll
                        for (int g = 0; g < NG; g++)
#pragma unroll
                            for (int e = 0; e < 4; e++) {
                                const int r = 4 * j + e;
                                float x = acc[g][r];
                                if constexpr (SC) x = (su[g] * qs4[e]) * x;
                                const float ef = fmaf(uerr[g], qn4[e], elam[g]);
                                const float diff = x - lam[g];
                                yes[g] |= (uint32_t)(diff > ef) << r;
                                amb[g] |= (uint32_t)(fabsf(diff) <= ef) << r;
                            }
                    }
#pragma unroll
                    for (int g = 0; g < NG; g++) {
                        yes[g] &= on16[g];
                        amb[g] &= on16[g];
                        if (force) {
                            yes[g] = linf[g] ? on16[g] : 0u;
                            amb[g] = linf[g] ? 0u : on16[g];
                        }
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const f32x4 qn4 = *(const f32x4*)(hf + 8 * j + h4);
                    f32x4 qs4 = {1.f, 1.f, 1.f, 1.f};
                    if constexpr (SC) qs4 = *(const f32x4*)(hf + 64 + 8 * j + h4);
                    const i32x4 sl4 = *(const i32x4*)(hq + 128 + 8 * j + h4);
#pragma unroll
                    for (int g = 0; g < NG; g++)
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const int r = 4 * j + e;
                            const float lam = lam_s[sl4[e] & 7][w * UPW + g * 32 + lc];
                            float x = acc[g][r];
                            if constexpr (SC) x = (su[g] * qs4[e]) * x;
                            const bool li = lam == -__builtin_inff();
                            const float ef = fmaf(uerr[g], qn4[e], (li ? 0.f : fabsf(lam) * 0x1p-23f) + (float)a.d * 0x1p-120f);
                            const float diff = x - lam;
                            yes[g] |= (uint32_t)(li || (!force && diff > ef)) << r;
                            amb[g] |= (uint32_t)(!li && (force || fabsf(diff) <= ef)) << r;
                        }
                }
#pragma unroll
                for (int g = 0; g < NG; g++) {
                    yes[g] &= on16[g];
                    amb[g] &= on16[g];
                }
            }
            n_amb += __popc(amb[0]) + __popc(amb[1]);
        }
        if (a.sah) {   // SAH: every pair the test does not reject goes on to the recheck
#pragma unroll
            for (int g = 0; g < NG; g++) {
                n_amb += __popc(yes[g]);
                amb[g] |= yes[g];
                yes[g] = 0u;
            }
        }
        if (a.bitmap) {   // yes answers as bits; the pool takes close calls only
#pragma unroll
            for (int g = 0; g < NG; g++)
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (yes[g] & (1u << r)) {
                        const uint32_t qo = hq[256 + row_of(r)];
                        const uint32_t ou = ouid_s[w * UPW + g * 32 + lc];
                        atomicOr(&a.bitmap[(int64_t)qo * a.bm_words + (ou >> 5)], 1u << (ou & 31u));
                    }
        } else {
            const int ny = __popc(yes[0]) + __popc(yes[1]);
            if (ballot64(ny != 0)) {
                const int iy = wave_incl_scan(ny);
                const int ty = __builtin_amdgcn_readlane(iy, 63);
                if (ycnt + ty > VR_SW) flush();
                const bool direct = ty > VR_SW;   // more than the stage holds: reserve now
                int64_t py = (int64_t)ycnt + iy - ny;
                if (direct) {
                    unsigned long long b = 0ull;
                    if (l == 0) b = atomicAdd(a.pool_count, (unsigned long long)ty);
                    b = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)b);
                    py = (int64_t)b + iy - ny;
                }
#pragma unroll
                for (int g = 0; g < NG; g++)
#pragma unroll
                    for (int r = 0; r < 16; r++)
                        if (yes[g] & (1u << r)) {
                            const unsigned long long e =
                                ((unsigned long long)hq[256 + row_of(r)] << 32) | ouid_s[w * UPW + g * 32 + lc];
                            if (direct) {
                                if (py < a.pool_cap) a.pool[py] = e;
                            } else {
                                ystage[py] = e;
                            }
                            py++;
                        }
                if (!direct) ycnt += ty;
                __builtin_amdgcn_wave_barrier();
            }
        }
        // close calls: one reservation per wave and tile that has any
        const int na = __popc(amb[0]) + __popc(amb[1]);
        if (ballot64(na != 0)) {
            const int ia = wave_incl_scan(na);
            const int ta = __builtin_amdgcn_readlane(ia, 63);
            unsigned long long b = 0ull;
            if (l == 0) b = atomicAdd(a.amb_count, (unsigned long long)ta);
            b = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
                __builtin_amdgcn_readfirstlane((uint32_t)b);
            int64_t pa = (int64_t)b + ia - na;
#pragma unroll
            for (int g = 0; g < NG; g++)
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (amb[g] & (1u << r)) {
                        const int64_t q = r0 + row_of(r);
                        const int64_t u = u0 + w * UPW + g * 32 + lc;
                        if (pa < a.amb_cap) a.amb[pa] = ((unsigned long long)q << 32) | (uint32_t)u;
                        pa++;
                    }
        }
    };

    __syncthreads();   // lambda rows and counters
    // the user data is in registers before the first tile load: the in-loop waits then
    // count the tile loads (and later stores) only
    __builtin_amdgcn_s_waitcnt(0);
    if (ntiles > 0) issue(ring_all, hq_all, 0);
    if (ntiles > 1) issue(ring_all + TBYTES, hq_all + VR_HQ, 1);
    int slot = 0, slot2 = 2;   // ring slots of tiles tt and tt + 2
    for (int tt = 0; tt < ntiles; tt++) {
        wait_tile(tt + 1 < ntiles);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");   // no LDS read moves above the barrier
        if (tt + 2 < ntiles) issue(ring_all + slot2 * TBYTES, hq_all + slot2 * VR_HQ, tt + 2);
        tile(ring_all + slot * TBYTES, hq_all + slot * VR_HQ, tt);
        slot = slot == 2 ? 0 : slot + 1;
        slot2 = slot2 == 2 ? 0 : slot2 + 1;
    }
    flush();
    const unsigned long long s0 = wave_sum((unsigned long long)n_node);
    const unsigned long long s2 = wave_sum((unsigned long long)n_scored);
    const unsigned long long s3 = wave_sum((unsigned long long)n_amb);
    if (l == 0) {
        if (s0) atomicAdd(&st_s[0], s0);
        if (s2) atomicAdd(&st_s[2], s2);
        if (s3) atomicAdd(&st_s[3], s3);
    }
    __syncthreads();
    if (threadIdx.x < 4 && st_s[threadIdx.x]) atomicAdd(&a.stats[threadIdx.x], st_s[threadIdx.x]);
}

// cos(phi) of every (block, query) pair, phi the angle between the query and the block's
// centre (Lemma 2; Alg. 5 block test), on the matrix cores: a dense contraction of the
// centres [nblocks x d] with the queries [nq x d].  A wave computes 32 blocks x 64 queries
// from operand fragments read straight from global memory (the centres are reused by the
// four waves of a workgroup through L1/L2).  Operand forms (MDT, the index's matrix-core
// type): BF16 and widened FP8 queries are exact BF16 rows and meet the centres' BF16 pair
// rows [hi | lo] as q.hi + q.lo; split FP32 queries (pair rows) take q_h c_h + q_l c_h +
// q_h c_l; FP32 matrix cores take the FP32 rows.  The error of each form is err_phi.
// Output cphi[block x nq + query], clamped to [-1, 1].
template <int MDT, int LD>
__global__ __launch_bounds__(256) void k_phi(QueryArgs a, float* cphi, int64_t b_base)
{
    const int l = lane_id(), w = threadIdx.x >> 6, h = l >> 5;
    const int64_t b0 = b_base + (int64_t)blockIdx.y * 32;
    const int64_t q0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    if (q0 >= a.nq) return;   // wave-uniform
    const int64_t brow = b0 + (l & 31) < a.nblocks ? b0 + (l & 31) : a.nblocks - 1;
    int64_t qrow[2];
#pragma unroll
    for (int g = 0; g < 2; g++) qrow[g] = q0 + g * 32 + (l & 31) < a.nq ? q0 + g * 32 + (l & 31) : a.nq - 1;
    f32x16 acc[2];
#pragma unroll
    for (int g = 0; g < 2; g++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[g][r] = 0.f;
    if constexpr (MDT == DT_F32) {
        // 32x32x2 FP32 products: the 16 bytes at t * 32 + h * 16 hold elements 8t + 4h + e
        const uint8_t* crow = (const uint8_t*)(a.center + brow * LD);
        const uint8_t* qr[2] = {(const uint8_t*)a.mma_queries + qrow[0] * LD * 4,
                                (const uint8_t*)a.mma_queries + qrow[1] * LD * 4};
#pragma unroll 4
        for (int t = 0; t < LD / 8; t++) {
            const f32x4 c4 = *(const f32x4*)(crow + t * 32 + h * 16);
#pragma unroll
            for (int g = 0; g < 2; g++) {
                const f32x4 q4 = *(const f32x4*)(qr[g] + t * 32 + h * 16);
#pragma unroll
                for (int e = 0; e < 4; e++) acc[g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c4[e], q4[e], acc[g], 0, 0, 0);
            }
        }
    } else {
        // BF16 pair rows of the centres: hi at [0, LD), lo at [LD, 2 LD)
        const uint8_t* crow = (const uint8_t*)(a.center_mma + brow * 2 * LD);
        constexpr int QLD = MDT == DT_SPLIT ? 2 * LD : LD;   // query operand row (elements)
        const uint8_t* qr[2] = {(const uint8_t*)a.mma_queries + qrow[0] * QLD * 2,
                                (const uint8_t*)a.mma_queries + qrow[1] * QLD * 2};
#pragma unroll 4
        for (int t = 0; t < LD / 16; t++) {
            const bf16x8 ch = __builtin_bit_cast(bf16x8, *(const i32x4*)(crow + t * 32 + h * 16));
            const bf16x8 cl = __builtin_bit_cast(bf16x8, *(const i32x4*)(crow + LD * 2 + t * 32 + h * 16));
#pragma unroll
            for (int g = 0; g < 2; g++) {
                const bf16x8 qh = __builtin_bit_cast(bf16x8, *(const i32x4*)(qr[g] + t * 32 + h * 16));
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, qh, acc[g], 0, 0, 0);
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cl, qh, acc[g], 0, 0, 0);
                if constexpr (MDT == DT_SPLIT) {
                    const bf16x8 ql = __builtin_bit_cast(bf16x8, *(const i32x4*)(qr[g] + LD * 2 + t * 32 + h * 16));
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, ql, acc[g], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < 2; g++) {
        const int64_t q = q0 + g * 32 + (l & 31);
        const bool qok = q < a.nq;
        const int64_t qq = qok ? q : a.nq - 1;
        const float qn = a.qnorm[qq];
        const float qsc = MDT == DT_FP8B ? a.query_scales[qq] : 1.f;
        const int kq = a.qk[qq];
        // prune word of block row i (lanes 0..31) for this 32-query tile
        uint32_t word = 0u;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int64_t blk = b0 + mfma32_row(r, l);
            const bool ok = qok && blk < a.nblocks;
            float dot = acc[g][r];
            if constexpr (MDT == DT_FP8B) dot *= qsc;
            float c = qn > 0.f ? dot / qn : 0.f;
            c = c > 1.f ? 1.f : (c < -1.f ? -1.f : c);
            if (cphi && ok) cphi[blk * a.nq + q] = c;
            if (a.prune) {
                bool pr = false;
                if (ok && qn > 0.f && a.block_ok[blk]) {
                    const NodeBound nd = node_bound(c, qn, a.cos_w[blk], a.sin_w[blk], a.err_phi, a.bound_slack);
                    pr = nd.ub < a.block_lb[(int64_t)(kq - 1) * a.nblocks + blk];
                }
                // bits 0..31: block row 8 (r / 4) + r % 4, bits 32..63: that row + 4
                const uint64_t bal = ballot64(pr);
                const int ra = ((r >> 2) << 3) + (r & 3);
                if (l == ra) word = (uint32_t)bal;
                if (l == ra + 4) word = (uint32_t)(bal >> 32);
            }
        }
        const int64_t T = (q0 + g * 32) >> 5;
        if (a.prune && l < 32 && b0 + l < a.nblocks && T < a.ntq) a.prune[(b0 + l) * a.ntq + T] = word;
    }
}

template <int MDT>
static void phi_d(const QueryArgs& a, float* cphi, hipStream_t s)
{
    const int64_t per_launch = (int64_t)65535 * 32;
    for (int64_t b0 = 0; b0 < a.nblocks; b0 += per_launch) {
        const int64_t nbl = std::min<int64_t>(per_launch, a.nblocks - b0);
        dim3 g((unsigned)((a.nq + 255) / 256), (unsigned)((nbl + 31) / 32));
        switch (a.ld) {
        case 32: hipLaunchKernelGGL((k_phi<MDT, 32>), g, dim3(256), 0, s, a, cphi, b0); break;
        case 64: hipLaunchKernelGGL((k_phi<MDT, 64>), g, dim3(256), 0, s, a, cphi, b0); break;
        case 128: hipLaunchKernelGGL((k_phi<MDT, 128>), g, dim3(256), 0, s, a, cphi, b0); break;
        case 256: hipLaunchKernelGGL((k_phi<MDT, 256>), g, dim3(256), 0, s, a, cphi, b0); break;
        default: fail(RKMIPS_EINVAL, "internal: unsupported padded dimension");
        }
    }
}

void launch_phi(const QueryArgs& a, float* cphi, hipStream_t s)
{
    if (a.nq <= 0 || a.nblocks <= 0) return;
    if (a.mma_dtype != DT_F32 && !a.center_mma) fail(RKMIPS_EINVAL, "internal: centre operand missing");
    if (a.mma_dtype == DT_F32) phi_d<DT_F32>(a, cphi, s);
    else if (a.mma_dtype == DT_BF16) phi_d<DT_BF16>(a, cphi, s);
    else if (a.mma_dtype == DT_FP8B) phi_d<DT_FP8B>(a, cphi, s);
    else if (a.mma_dtype == DT_SPLIT) phi_d<DT_SPLIT>(a, cphi, s);
    else fail(RKMIPS_EINVAL, "internal: no matrix-core path for this operand type");
    HIPC(hipGetLastError());
}

template <int DT, int DPT>
static void verify_g(const QueryArgs& a, int64_t q0, int64_t q1, hipStream_t s)
{
    // one 32-user column block per wave: the register budget goes to occupancy, which
    // hides the per-tile latencies (the matrix-core share of this pass is small)
    constexpr int UBW = 1;
    constexpr int UT = VF_WAVES * UBW * 32;
    const int64_t tiles = (a.m + UT - 1) / UT;
    // split the queries so that the grid covers the chip several times
    const int64_t nq = q1 - q0;
    int64_t nchunk = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, tiles));
    nchunk = std::min<int64_t>(nchunk, (nq + 31) / 32);
    int64_t clen = (nq + nchunk - 1) / nchunk;
    clen = (clen + 31) / 32 * 32;
    nchunk = (nq + clen - 1) / clen;
    for (int64_t c = 0; c < nchunk; c++) {
        const int64_t qb = q0 + c * clen, qe = std::min(q1, qb + clen);
        hipLaunchKernelGGL((k_verify<DT, DPT, UBW>), dim3((unsigned)tiles), dim3(256), 0, s, a, qb, qe);
    }
}

template <int DT>
static void verify_d(const QueryArgs& a, int64_t q0, int64_t q1, hipStream_t s)
{
    if constexpr (DT == DT_SPLIT) {   // pair rows of FP32 data: 2 x 32, 2 x 64
        if (a.mma_ld == 64) verify_g<DT, 64>(a, q0, q1, s);
        else if (a.mma_ld == 128) verify_g<DT, 128>(a, q0, q1, s);
        else fail(RKMIPS_EINVAL, "internal: unsupported split row length");
    } else {
        switch (a.mma_ld) {
        case 32: verify_g<DT, 32>(a, q0, q1, s); break;
        case 64: verify_g<DT, 64>(a, q0, q1, s); break;
        case 128: verify_g<DT, 128>(a, q0, q1, s); break;
        case 256: verify_g<DT, 256>(a, q0, q1, s); break;
        default: fail(RKMIPS_EINVAL, "internal: unsupported padded dimension");
        }
    }
}

bool verify_uses_ring(const QueryArgs& a)
{
    return (((a.mma_dtype == DT_BF16 || a.mma_dtype == DT_FP8B) && (a.mma_ld == 128 || a.mma_ld == 256)) ||
            (a.mma_dtype == DT_SPLIT && a.mma_ld == 128)) &&
           !(a.flags & RKMIPS_FLAG_VERIFY_SIMPLE);
}

template <int DT, int DPT>
static void verify_ring_g(const QueryArgs& a, int64_t q0, int64_t q1, hipStream_t s)
{
    const int64_t wgs = (a.m + VR_UPB - 1) / VR_UPB;
    // the query range in chunks of whole tiles: enough workgroups to fill the chip in
    // nearly whole rounds (two or three per compute unit), and per-lane counters that
    // stay far below 2^32
    constexpr int64_t kSlots = 256 * verify_ring_wpe<DT, DPT>();   // workgroups resident at once
    const int64_t t0 = q0 >> 5, t1 = (q1 + 31) >> 5, nt = t1 - t0;
    int64_t best = 1;
    double best_cost = 1e300;
    for (int64_t c = 1; c <= 4 && c <= nt; c++) {
        // rounds of resident workgroups, each a chunk's tiles plus its prologue (user
        // rows, lambda rows: about three tiles' time)
        const double rounds = std::ceil((double)(wgs * c) / (double)kSlots);
        const double cost = rounds * ((double)nt / (double)c + 3.0);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = c;
        }
    }
    int64_t per = (nt + best - 1) / best;
    per = std::min<int64_t>(per, int64_t(1) << 15);
    const int64_t nchunk = (nt + per - 1) / per;
    if (wgs * nchunk > INT_MAX) fail(RKMIPS_EINVAL, "internal: verify grid too large");
    hipLaunchKernelGGL((k_verify_ring<DT, DPT>), dim3((unsigned)(wgs * nchunk)), dim3(256), 0, s, a, q0, q1, per, wgs);
}

void launch_verify_range(const QueryArgs& a, int64_t q0, int64_t q1, hipStream_t s)
{
    if (q1 <= q0 || a.m <= 0) return;
    if (a.nslots > VF_MAXSLOT) fail(RKMIPS_EINVAL, "internal: too many distinct k in one launch");
    if (verify_uses_ring(a)) {
        if (a.ntq != (a.nq + 31) / 32 || a.ntq >= (int64_t(1) << 24))
            fail(RKMIPS_EINVAL, "internal: prune-word table does not match the batch");
        if (a.mma_dtype == DT_SPLIT) {
            verify_ring_g<DT_SPLIT, 128>(a, q0, q1, s);
        } else if (a.mma_dtype == DT_BF16) {
            if (a.mma_ld == 128) verify_ring_g<DT_BF16, 128>(a, q0, q1, s);
            else verify_ring_g<DT_BF16, 256>(a, q0, q1, s);
        } else {
            if (a.mma_ld == 128) verify_ring_g<DT_FP8B, 128>(a, q0, q1, s);
            else verify_ring_g<DT_FP8B, 256>(a, q0, q1, s);
        }
        HIPC(hipGetLastError());
        return;
    }
    if (a.mma_dtype == DT_F32) verify_d<DT_F32>(a, q0, q1, s);
    else if (a.mma_dtype == DT_BF16) verify_d<DT_BF16>(a, q0, q1, s);
    else if (a.mma_dtype == DT_FP8B) verify_d<DT_FP8B>(a, q0, q1, s);
    else if (a.mma_dtype == DT_SPLIT) verify_d<DT_SPLIT>(a, q0, q1, s);
    else fail(RKMIPS_EINVAL, "internal: no matrix-core path for this operand type");
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ canonical FP64 recheck
template <int DT>
__device__ double canon_dot2(const void* A, int64_t ra, int lda, float sa, const void* B, int64_t rb, int ldb, float sb, int d)
{
    double acc = 0.0;
    for (int i = 0; i < d; i++)
        acc = __fma_rn((double)elem_f32<DT>(A, ra * lda + i), (double)elem_f32<DT>(B, rb * ldb + i), acc);
    if constexpr (DT == DT_FP8) acc = ((double)sa * (double)sb) * acc;
    return acc;
}

// namb_dev (when given): the close-call count on the device, read here (grid-stride).
template <int DT>
__global__ void k_recheck(QueryArgs a, int64_t namb, const unsigned long long* namb_dev, const int* reject)
{
    if (namb_dev) {
        const int64_t c = (int64_t)*namb_dev;
        namb = c < a.amb_cap ? c : a.amb_cap;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namb; i += (int64_t)gridDim.x * blockDim.x) {
        if (reject && reject[i] == 0) {   // Alg. 2 proved s(u,q) < phi <= lambda_u^(k)
            atomicAdd(&a.stats[4], 1ull);
            continue;
        }
        const unsigned long long key = a.amb[i];
        const int64_t q = (int64_t)(key >> 32);
        const int64_t u = (int64_t)(key & 0xffffffffull);
        const int k = a.qk[q];
        const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
        const float sq = DT == DT_FP8 ? a.query_scales[q] : 1.f;
        const double s = canon_dot2<DT>(a.users, u, a.ld, su, a.queries, q, a.ld, sq, a.d);
        if (s >= a.lam64[(int64_t)(k - 1) * a.m + a.perm[u]]) {
            const uint32_t ou = a.perm[u];
            if (a.sah) {
                // Alg. 5: yes when s(u,q) >= ||u|| ||p_k|| (as s >= 0, s^2 >= n2(u) n2(p_k),
                // each product rounded once: fma with a zero addend, never fused with
                // anything else; the lazy mode widens the right side), else Alg. 2 decides
                const double pk2 = k <= a.n_items ? a.item_n2[k - 1] : 0.0;
                const double un = __fma_rn(a.user_n2[u], pk2, 0.0);
                const double thr = a.norm_widen > 0.0 ? __fma_rn(un, a.norm_widen, un) : un;
                if (!(s >= 0.0 && __fma_rn(s, s, 0.0) >= thr)) {
                    const unsigned long long pos = atomicAdd(a.sah_count, 1ull);
                    if ((int64_t)pos < a.amb_cap) {
                        a.sah_pairs[pos] = key;
                        a.sah_score[pos] = s;
                    }
                    a.sah_need[u] = 1;
                    continue;
                }
            }
            if (a.bitmap) {
                atomicOr(&a.bitmap[(int64_t)a.qorig[q] * a.bm_words + (ou >> 5)], 1u << (ou & 31u));
            } else {
                const unsigned long long pos = atomicAdd(a.pool_count, 1ull);
                if ((int64_t)pos < a.pool_cap) a.pool[pos] = ((unsigned long long)a.qorig[q] << 32) | ou;
            }
        }
    }
}

// Item insertion: the canonical scores of the new items (rows [n_new x ld]) merged into
// every user's lambda row (k-major, original user order).  A score above the row's last
// entry enters at its rank (after equal entries) and the last entry drops out, so the row
// stays the k_max largest scores over the grown item set.  One thread per user (leaf
// position u); *changed counts the users whose row changed.
template <int DT>
__global__ void k_insert_lambda(const void* users, const float* user_scales, const uint32_t* perm, int64_t m, int d,
                                int ld, const void* items, const float* item_scales, int64_t n_new, double* lam64,
                                float* lam32, int k_max, unsigned long long* changed)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= m) return;
    const int64_t ou = perm[u];
    const float su = DT == DT_FP8 ? user_scales[u] : 1.f;
    bool ch = false;
    for (int64_t j = 0; j < n_new; j++) {
        const float sp = DT == DT_FP8 ? item_scales[j] : 1.f;
        const double s = canon_dot2<DT>(users, u, ld, su, items, j, ld, sp, d);
        if (!(s > lam64[(int64_t)(k_max - 1) * m + ou])) continue;
        int r = k_max - 1;
        while (r > 0 && lam64[(int64_t)(r - 1) * m + ou] < s) {
            lam64[(int64_t)r * m + ou] = lam64[(int64_t)(r - 1) * m + ou];
            lam32[(int64_t)r * m + ou] = lam32[(int64_t)(r - 1) * m + ou];
            r--;
        }
        lam64[(int64_t)r * m + ou] = s;
        lam32[(int64_t)r * m + ou] = (float)s;
        ch = true;
    }
    if (ch) atomicAdd(changed, 1ull);
}

void launch_insert_lambda(int dtype, const void* users, const float* user_scales, const uint32_t* perm, int64_t m,
                          int d, int ld, const void* items, const float* item_scales, int64_t n_new, double* lam64,
                          float* lam32, int k_max, unsigned long long* changed, hipStream_t s)
{
    if (m <= 0 || n_new <= 0) return;
    dim3 g((unsigned)((m + 255) / 256)), b(256);
    if (dtype == DT_F32) hipLaunchKernelGGL(k_insert_lambda<DT_F32>, g, b, 0, s, users, user_scales, perm, m, d, ld, items, item_scales, n_new, lam64, lam32, k_max, changed);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_insert_lambda<DT_BF16>, g, b, 0, s, users, user_scales, perm, m, d, ld, items, item_scales, n_new, lam64, lam32, k_max, changed);
    else hipLaunchKernelGGL(k_insert_lambda<DT_FP8>, g, b, 0, s, users, user_scales, perm, m, d, ld, items, item_scales, n_new, lam64, lam32, k_max, changed);
    HIPC(hipGetLastError());
}

void launch_recheck(const QueryArgs& a, int64_t namb, const int* reject, hipStream_t s)
{
    if (namb <= 0) return;
    dim3 g((unsigned)((namb + 255) / 256)), b(256);
    if (a.dtype == DT_F32) hipLaunchKernelGGL(k_recheck<DT_F32>, g, b, 0, s, a, namb, nullptr, reject);
    else if (a.dtype == DT_BF16) hipLaunchKernelGGL(k_recheck<DT_BF16>, g, b, 0, s, a, namb, nullptr, reject);
    else hipLaunchKernelGGL(k_recheck<DT_FP8>, g, b, 0, s, a, namb, nullptr, reject);
    HIPC(hipGetLastError());
}

// Close calls counted on the device: pool[cnt, cnt + namb) is cleared (the recheck
// appends there), span = cnt + namb (capped) is kept in ctr[5], then the recheck runs
// over the device count.
__global__ void k_close_init(unsigned long long* ctr, unsigned long long* pool, int64_t pool_cap, int64_t amb_cap)
{
    const int64_t cnt = (int64_t)ctr[0];
    int64_t namb = (int64_t)ctr[1];
    namb = namb < amb_cap ? namb : amb_cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[5] = (unsigned long long)(cnt + namb < pool_cap ? cnt + namb : pool_cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namb; i += (int64_t)gridDim.x * blockDim.x)
        if (cnt + i < pool_cap) pool[cnt + i] = ~0ull;
}

void launch_recheck_device(const QueryArgs& a, hipStream_t s)
{
    unsigned long long* ctr = a.pool_count;   // ctr[0] = pool count, ctr[1] = close calls
    if (!a.bitmap) hipLaunchKernelGGL(k_close_init, dim3(64), dim3(256), 0, s, ctr, a.pool, a.pool_cap, a.amb_cap);
    const unsigned g = (unsigned)std::min<int64_t>((a.amb_cap + 255) / 256, 256);
    if (a.dtype == DT_F32) hipLaunchKernelGGL(k_recheck<DT_F32>, dim3(g), dim3(256), 0, s, a, (int64_t)0, ctr + 1, nullptr);
    else if (a.dtype == DT_BF16) hipLaunchKernelGGL(k_recheck<DT_BF16>, dim3(g), dim3(256), 0, s, a, (int64_t)0, ctr + 1, nullptr);
    else hipLaunchKernelGGL(k_recheck<DT_FP8>, dim3(g), dim3(256), 0, s, a, (int64_t)0, ctr + 1, nullptr);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ query norms
template <int DT>
__global__ void k_qnorm(const void* Q, const float* qs, int64_t nq, int d, int ld, float* qnorm, int* bad)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    double acc = 0.0;
    bool ok = true;
    for (int i = 0; i < d; i++) {
        const float v = elem_f32<DT>(Q, q * ld + i);
        ok &= (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
        acc = __fma_rn((double)v, (double)v, acc);
    }
    if constexpr (DT == DT_FP8) {
        const float s = qs[q];
        ok &= (__float_as_uint(s) & 0x7f800000u) != 0x7f800000u;
        acc *= (double)s * (double)s;
    }
    if constexpr (DT == DT_FP8) {
        // NaN codes decode to finite magnitudes above 448 only through exponent 15 mantissa 7
        for (int i = 0; i < d; i++) ok &= (((const uint8_t*)Q)[q * ld + i] & 0x7fu) != 0x7fu;
    }
    const double nr = sqrt(acc);
    qnorm[q] = (float)nr;
    if (!ok) atomicOr(bad, 1);
    else if (nr > 1e30 || (nr > 0.0 && nr < 1e-30)) atomicOr(bad, 2);
}

void launch_qnorm(int dtype, const void* Q, const float* qs, int64_t nq, int d, int ld, float* qnorm, int* bad,
                  hipStream_t s)
{
    if (nq <= 0) return;
    dim3 g((unsigned)((nq + 255) / 256)), b(256);
    if (dtype == DT_F32) hipLaunchKernelGGL(k_qnorm<DT_F32>, g, b, 0, s, Q, qs, nq, d, ld, qnorm, bad);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_qnorm<DT_BF16>, g, b, 0, s, Q, qs, nq, d, ld, qnorm, bad);
    else hipLaunchKernelGGL(k_qnorm<DT_FP8>, g, b, 0, s, Q, qs, nq, d, ld, qnorm, bad);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ result lists
// keys sorted ascending; offsets[q] = first key >= q << 32; ids = low halves.
// ------------------------------------------------------------------ result lists
// The result keys (caller's query index << 32 | original user id) become per-query
// ascending id lists: a count per query, an exclusive scan into offsets, a scatter by
// query, then one workgroup per query sorts its ids (in LDS up to QS_CHUNK ids; larger
// lists are sorted in chunks and merged level by level afterwards).  Entries whose query
// field is out of range are unused slots and are skipped.
static constexpr int QS_CHUNK = 4096;

// span_dev (when given): the pool span on the device (grid-stride over it).
__global__ void k_qcount(const uint64_t* keys, int64_t span, const unsigned long long* span_dev, int64_t nq, int* cnt)
{
    if (span_dev) span = (int64_t)*span_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t q = keys[i] >> 32;
        if (q < (uint64_t)nq) atomicAdd(&cnt[q], 1);
    }
}

// One workgroup: offsets[0..nq] = exclusive scan of cnt (64-bit), cnt reset to zero (it
// becomes the scatter cursor), stat[0] = largest count.
__global__ __launch_bounds__(1024) void k_qscan(int* cnt, int64_t nq, int64_t* offsets, long long* stat)
{
    __shared__ long long wtot[16];
    __shared__ long long carry_s;
    __shared__ int maxc_s;
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    if (tid == 0) {
        carry_s = 0;
        maxc_s = 0;
    }
    __syncthreads();
    int mymax = 0;
    for (int64_t c0 = 0; c0 < nq; c0 += 1024) {
        const int64_t q = c0 + tid;
        const int c = q < nq ? cnt[q] : 0;
        mymax = c > mymax ? c : mymax;
        // inclusive scan of c within the wave (64-bit)
        long long v = c;
        for (int o = 1; o < 64; o <<= 1) {
            const long long t = __shfl_up(v, o);
            if (l >= o) v += t;
        }
        if (l == 63) wtot[w] = v;
        __syncthreads();
        long long off = carry_s;
        for (int i = 0; i < w; i++) off += wtot[i];
        if (q < nq) {
            offsets[q] = off + v - c;
            cnt[q] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            long long t = 0;
            for (int i = 0; i < 16; i++) t += wtot[i];
            carry_s += t;
        }
        __syncthreads();
    }
    mymax = wave_max(mymax);
    if (l == 0) atomicMax(&maxc_s, mymax);
    __syncthreads();
    if (tid == 0) {
        offsets[nq] = carry_s;
        stat[0] = maxc_s;
    }
}

__global__ void k_qscatter(const uint64_t* keys, int64_t span, const unsigned long long* span_dev, int64_t nq,
                           const int64_t* offsets, int* cursor, int32_t* out)
{
    if (span_dev) span = (int64_t)*span_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[i];
        const uint64_t q = key >> 32;
        if (q >= (uint64_t)nq) continue;
        out[offsets[q] + atomicAdd(&cursor[q], 1)] = (int32_t)(key & 0xffffffffull);
    }
}

// Ascending sort of up to QS_CHUNK ids in LDS (bitonic over the next power of two,
// padded with INT_MAX), written to dst.
__device__ void qs_sort_chunk(const int32_t* src, int32_t* dst, int c, int32_t* sh)
{
    int P = 1;
    while (P < c) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x) sh[i] = i < c ? src[i] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const int32_t x = sh[i], y = sh[p];
                    if ((x > y) == up) {
                        sh[i] = y;
                        sh[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < c; i += blockDim.x) dst[i] = sh[i];
    __syncthreads();
}

// One workgroup per query: its ids from src sorted into dst (lists longer than
// QS_CHUNK as sorted chunks, merged by k_qmerge).
__global__ __launch_bounds__(256) void k_qsort(const int64_t* offsets, const int32_t* src, int32_t* dst)
{
    __shared__ int32_t sh[QS_CHUNK];
    const int64_t q = blockIdx.x;
    const int64_t b = offsets[q], c = offsets[q + 1] - b;
    for (int64_t c0 = 0; c0 < c; c0 += QS_CHUNK) {
        const int len = (int)(c - c0 < QS_CHUNK ? c - c0 : QS_CHUNK);
        qs_sort_chunk(src + b + c0, dst + b + c0, len, sh);
    }
}

// One merge level for the lists longer than `run`: sorted runs of length `run` in src
// become runs of 2 run in dst (a list not longer than 2 run is complete afterwards).
// Each of the 256 threads merges one slice of the output, found by a binary search on
// its diagonal (ids within a list are distinct).
__global__ __launch_bounds__(256) void k_qmerge(const int64_t* offsets, int64_t run, const int32_t* src,
                                                int32_t* dst)
{
    const int64_t q = blockIdx.x;
    const int64_t b = offsets[q], c = offsets[q + 1] - b;
    if (c <= QS_CHUNK) return;   // never chunked: already final in its own buffer
    for (int64_t s0 = 0; s0 < c; s0 += 2 * run) {
        const int64_t la = c - s0 < run ? c - s0 : run;
        const int64_t lb = c - s0 - la < run ? c - s0 - la : run;
        const int32_t* A = src + b + s0;
        const int32_t* B = A + la;
        int32_t* D = dst + b + s0;
        const int64_t T = la + lb;
        const int64_t d0 = T * threadIdx.x / 256, d1 = T * (threadIdx.x + 1) / 256;
        // split of diagonal d0: i from A, d0 - i from B
        int64_t lo = d0 > lb ? d0 - lb : 0, hi = d0 < la ? d0 : la;
        while (lo < hi) {
            const int64_t i = (lo + hi) >> 1;
            if (A[i] < B[d0 - i - 1]) lo = i + 1;
            else hi = i;
        }
        int64_t i = lo, j = d0 - lo;
        for (int64_t o = d0; o < d1; o++) {
            if (j >= lb || (i < la && A[i] < B[j])) D[o] = A[i++];
            else D[o] = B[j++];
        }
    }
}

// Copies the lists longer than QS_CHUNK from src to dst (after an odd number of merges).
__global__ __launch_bounds__(256) void k_qcopy_long(const int64_t* offsets, const int32_t* src, int32_t* dst)
{
    const int64_t q = blockIdx.x;
    const int64_t b = offsets[q], c = offsets[q + 1] - b;
    if (c <= QS_CHUNK) return;
    for (int64_t i = threadIdx.x; i < c; i += 256) dst[b + i] = src[b + i];
}

// ---- lists from answer bits: one wave per query, words in order, so the ids come out
// ascending without a sort
__global__ __launch_bounds__(256) void k_bm_count(const uint32_t* bm, int64_t words, int64_t nq, int* cnt)
{
    const int l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq) return;
    const uint32_t* row = bm + q * words;
    int c = 0;
    for (int64_t i = l; i < words; i += 64) c += __popc(row[i]);
    c = wave_sum(c);
    if (l == 0) cnt[q] = c;
}

__global__ __launch_bounds__(256) void k_bm_emit(const uint32_t* bm, int64_t words, int64_t nq, const int64_t* offsets,
                                                 int32_t* ids, int64_t ids_cap)
{
    const int l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq) return;
    const uint32_t* row = bm + q * words;
    int64_t base = offsets[q];
    for (int64_t i0 = 0; i0 < words; i0 += 64) {
        const int64_t i = i0 + l;
        uint32_t wd = i < words ? row[i] : 0u;
        const int pc = __popc(wd);
        const int incl = wave_incl_scan(pc);
        int64_t pos = base + incl - pc;
        while (wd) {
            const int bit = __builtin_ctz(wd);
            wd &= wd - 1u;
            if (pos < ids_cap) ids[pos] = (int32_t)(i * 32 + bit);
            pos++;
        }
        base += __shfl(incl, 63);
    }
}

void launch_bitmap_lists(const uint32_t* bitmap, int64_t words, int64_t nq, int* cnt, int64_t* offsets,
                         long long* stat, int32_t* ids, int64_t ids_cap, hipStream_t s)
{
    if (nq <= 0) return;
    const unsigned g = (unsigned)((nq + 3) / 4);
    hipLaunchKernelGGL(k_bm_count, dim3(g), dim3(256), 0, s, bitmap, words, nq, cnt);
    hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, s, cnt, nq, offsets, stat);
    hipLaunchKernelGGL(k_bm_emit, dim3(g), dim3(256), 0, s, bitmap, words, nq, (const int64_t*)offsets, ids, ids_cap);
    HIPC(hipGetLastError());
}

void launch_result_lists(const uint64_t* keys, int64_t span, const unsigned long long* span_dev, int64_t nq, int* cnt,
                         int64_t* offsets, long long* stat, int32_t* tmp, int32_t* ids, hipStream_t s)
{
    if (nq <= 0) return;
    HIPC(hipMemsetAsync(cnt, 0, sizeof(int) * nq, s));
    // with a device span, `span` bounds it (the pool capacity) and sizes the grid
    const unsigned g = (unsigned)std::min<int64_t>((span + 255) / 256, span_dev ? 2048 : INT32_MAX);
    if (span > 0) hipLaunchKernelGGL(k_qcount, dim3(g), dim3(256), 0, s, keys, span, span_dev, nq, cnt);
    hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, s, cnt, nq, offsets, stat);
    if (span > 0)
        hipLaunchKernelGGL(k_qscatter, dim3(g), dim3(256), 0, s, keys, span, span_dev, nq, (const int64_t*)offsets,
                           cnt, tmp);
    hipLaunchKernelGGL(k_qsort, dim3((unsigned)nq), dim3(256), 0, s, (const int64_t*)offsets, (const int32_t*)tmp, ids);
    HIPC(hipGetLastError());
}

void launch_result_merges(int64_t nq, int64_t max_count, const int64_t* offsets, int32_t* tmp, int32_t* ids,
                          hipStream_t s)
{
    if (max_count <= QS_CHUNK) return;
    int32_t* src = ids;
    int32_t* dst = tmp;
    for (int64_t run = QS_CHUNK; run < max_count; run *= 2) {
        hipLaunchKernelGGL(k_qmerge, dim3((unsigned)nq), dim3(256), 0, s, offsets, run, (const int32_t*)src, dst);
        std::swap(src, dst);
    }
    if (src != ids) hipLaunchKernelGGL(k_qcopy_long, dim3((unsigned)nq), dim3(256), 0, s, offsets, (const int32_t*)src, ids);
    HIPC(hipGetLastError());
}

}  // namespace rk
