// lambda build: for every user u, lambda_u^(j), j = 1..k_max, the j-th largest inner
// product of u over all items (Definition 1; the lower-bound array of Alg. 4 taken
// over all of P instead of the top-norm subset P').
//
// Pass 0 (k_topk, seed mode): on a stratified sample of the items, the matrix cores
//   score every user and each lane keeps its few largest scores in registers; their
//   order statistic estimates a per-user threshold that a fixed multiple of C items
//   of the whole set exceed.
// Pass 1 (k_topk, main mode): fused U.P^T on the matrix cores with a streaming per-user
//   top-C (C = k_max + slack).  A wave keeps 64 users' operand fragments in registers
//   (32 where the rows are too long for two groups), so that every item fragment read
//   from LDS feeds two products; a workgroup of four waves streams the norm-sorted items
//   through a ring of three padded LDS tiles, filled by direct loads two tiles ahead of
//   the one being scored.  Every MFMA output lane owns one user column per group; a
//   score enters the user's candidate buffer only if it beats the user's register
//   threshold (starting at the seed estimate).  When a buffer fills, the wave compacts
//   it to its C best entries with a wave radix select and raises the threshold to the
//   running C-th best.  The final threshold tau bounds every item left out.
// Pass 2 (canonical FP64 rescoring and the certificate) is in k_refine.hip.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"
#include "internal.h"

namespace rk {

static constexpr int TK_WAVES = 4;
static constexpr int TK_IT_REG = 64;   // items per tile of the register-prefetch kernel (two blocks)

// ------------------------------------------------------------------ fused GEMM + top-k
// Buffer compaction for the streaming pass, with the keys staged in LDS so that it needs
// few registers (it runs rarely; inlined, since a call would make the main loop save its
// resident fragments around it): of the c0 entries at r0 and the c1 entries at r1, keep the C largest
// (ties at the threshold in staging order) in r0[0, C) and return the C-th largest key
// (orderable form; the entries themselves keep the raw score bits).  The kept entries
// move down in place: entry i lands at a position <= i, and r0 is read in full before r1.
__device__ __forceinline__ uint32_t select_user(uint2* r0, int c0, const uint2* r1, int c1, int C, int* hist,
                                             uint32_t* stage)
{
    const int l = lane_id();
    const int c = c0 + c1;
    for (int i = l; i < c; i += 64) {
        const uint2* src = i < c0 ? r0 + i : r1 + (i - c0);
        const uint32_t raw = __hip_atomic_load((const uint32_t*)src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // buffers hold raw score bits; the selection works on orderable keys
        stage[i] = f32_ord(__uint_as_float(raw));
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t prefix = 0u, pmask = 0u;
    int need = C;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = l; b < 256; b += 64) hist[b] = 0;
        __builtin_amdgcn_wave_barrier();
        for (int i = l; i < c; i += 64) {
            const uint32_t k = stage[i];
            if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1);
        }
        __builtin_amdgcn_wave_barrier();
        int h[4], x = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) { h[e] = hist[4 * l + e]; x += h[e]; }
        const int incl = wave_incl_scan(x);
        const int total = __shfl(incl, 63);
        int above = total - incl;
        int sel = -1, sel_above = 0;
#pragma unroll
        for (int e = 3; e >= 0; e--) {
            if (sel < 0 && above < need && need <= above + h[e]) { sel = 4 * l + e; sel_above = above; }
            above += h[e];
        }
        const uint64_t bal = ballot64(sel >= 0);
        const int src = bal ? __builtin_ctzll(bal) : 0;
        prefix |= (uint32_t)__shfl(sel, src) << shift;
        pmask |= 0xffu << shift;
        need -= __shfl(sel_above, src);
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t T = prefix;
    int eq_before = 0, kept_before = 0;
    for (int i0 = 0; i0 < c; i0 += 64) {
        const int i = i0 + l;
        const bool valid = i < c;
        const uint32_t key = valid ? stage[i] : 0u;
        const bool gt = valid && key > T;
        const bool eq = valid && key == T;
        const uint64_t eb = ballot64(eq);
        const int rank_eq = eq_before + __popcll(eb & lanemask_lt());
        eq_before += __popcll(eb);
        const bool keep = gt || (eq && rank_eq < need);
        const uint64_t kb = ballot64(keep);
        // every lane of the chunk reads its entry before any lane writes
        unsigned long long e = 0ull;
        if (keep)
            e = __hip_atomic_load((const unsigned long long*)(i < c0 ? r0 + i : r1 + (i - c0)), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_wave_barrier();
        if (keep) r0[kept_before + __popcll(kb & lanemask_lt())] = make_uint2((uint32_t)e, (uint32_t)(e >> 32));
        kept_before += __popcll(kb);
    }
    __builtin_amdgcn_wave_barrier();
    return T;
}

// Out-of-line form for the register-prefetch kernel, whose main loop keeps its register
// budget for occupancy.
__device__ __noinline__ uint32_t select_user_call(uint2* r0, int c0, const uint2* r1, int c1, int C, int* hist,
                                                  uint32_t* stage)
{
    return select_user(r0, c0, r1, c1, C, hist, stage);
}

// 32 x 32 blocks of scores on the matrix cores, one per user group: rows = the 32 items
// of LDS rows [row0, row0 + 32) of a staged tile, columns = group g's 32 users (register
// fragments).  Every A fragment read from LDS feeds the NG groups' products.
template <int DT, int KSTEPS, int LROW, int NG>
__device__ __forceinline__ void mfma_block(const uint8_t* tile, int row0, const i32x4 (&bfrag)[NG][KSTEPS],
                                           f32x16 (&acc)[NG])
{
    const int l = lane_id(), h = l >> 5;
#pragma unroll
    for (int g = 0; g < NG; g++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[g][r] = 0.f;
    const uint8_t* arow = tile + (row0 + (l & 31)) * LROW + h * 16;
#pragma unroll
    for (int t = 0; t < KSTEPS; t++) {
        if constexpr (DT == DT_F32) {
            const f32x4 a4 = __builtin_bit_cast(f32x4, *(const i32x4*)(arow + t * 32));
#pragma unroll
            for (int e = 0; e < 4; e++)
#pragma unroll
                for (int g = 0; g < NG; g++)
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[e], __builtin_bit_cast(f32x4, bfrag[g][t])[e],
                                                                  acc[g], 0, 0, 0);
        } else if constexpr (dt_bf16_mma<DT>) {
            const bf16x8 af = __builtin_bit_cast(bf16x8, *(const i32x4*)(arow + t * 32));
#pragma unroll
            for (int g = 0; g < NG; g++)
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, __builtin_bit_cast(bf16x8, bfrag[g][t]), acc[g], 0,
                                                                 0, 0);
        } else if constexpr (DT == DT_SPLIT) {
            // rows [hi | lo]: k-step t < KSTEPS / 2 of the hi half pairs with step
            // t + KSTEPS / 2 of the lo half (same elements); three products per pair
            constexpr int HK = KSTEPS / 2;
            if (t < HK) {
                const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const i32x4*)(arow + t * 32));
                const bf16x8 al = __builtin_bit_cast(bf16x8, *(const i32x4*)(arow + (t + HK) * 32));
#pragma unroll
                for (int g = 0; g < NG; g++) {
                    const bf16x8 bh = __builtin_bit_cast(bf16x8, bfrag[g][t]);
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, bfrag[g][t + HK]);
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[g], 0, 0, 0);
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[g], 0, 0, 0);
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[g], 0, 0, 0);
                }
            }
        } else if constexpr (DT == DT_FP8) {
            // e4m3 codes as they are, 64-wide k steps (two 32-byte units t, t + 1): lane
            // half h supplies bytes [64 s + 32 h, + 32) of step s, for both operands, so the
            // instruction pairs every k once whatever order it gives those bytes; unit
            // scales.  Only the seed pass, an estimate, runs here: its sums carry the FP8
            // matrix cores' own rounding, outside the fast-score error model.
            if ((t & 1) == 0) {
                const uint8_t* a8 = tile + (row0 + (l & 31)) * LROW + h * 32 + (t >> 1) * 64;
                const i32x4 a0 = *(const i32x4*)a8, a1 = *(const i32x4*)(a8 + 16);
                const i32x8 av = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
#pragma unroll
                for (int g = 0; g < NG; g++) {
                    const i32x4 b0 = bfrag[g][t], b1 = bfrag[g][t + 1];
                    const i32x8 bv = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
                    acc[g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[g], 0, 0, 0, 127, 0, 127);
                }
            }
        } else {
            static_assert(dt_bf16_mma<DT>, "unsupported matrix-core operand");
        }
    }
    if constexpr (dt_bf16_mma<DT> && NG == 2 && KSTEPS >= 4) {
        // schedule: three fragment reads ahead, then per k-step two products and the read
        // three steps ahead (left alone, the scheduler keeps two reads in flight, and each
        // pair of k-steps waits for LDS)
        __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
        for (int t = 0; t < KSTEPS - 3; t++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
    }
}

// Two modes over the same matrix-core pipeline (see the file comment).  A wave owns NG
// groups of 32 users; every MFMA output lane owns one user column per group.  Item tiles
// reach LDS by direct (DMA) loads into a ring of three padded tile buffers, two tiles
// ahead of the one being scored; one barrier per tile.
// 32 x 32 block of scores on the matrix cores: rows = the 32 items of LDS rows
// [row0, row0 + 32) of a staged tile, columns = the wave's 32 users (register fragments).
template <int DT, int KSTEPS, int LROW>
__device__ __forceinline__ f32x16 mfma_block1(const uint8_t* tile, int row0, const i32x4 (&bfrag)[KSTEPS])
{
    const int l = lane_id(), h = l >> 5;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.f;
    const uint8_t* arow = tile + (row0 + (l & 31)) * LROW + h * 16;
    i32x4 af[KSTEPS];
#pragma unroll
    for (int t = 0; t < KSTEPS; t++) af[t] = *(const i32x4*)(arow + t * 32);
#pragma unroll
    for (int t = 0; t < KSTEPS; t++) {
        if constexpr (DT == DT_F32) {
            const f32x4 a4 = __builtin_bit_cast(f32x4, af[t]);
            const f32x4 b4 = __builtin_bit_cast(f32x4, bfrag[t]);
#pragma unroll
            for (int e = 0; e < 4; e++) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[e], b4[e], acc, 0, 0, 0);
        } else if constexpr (dt_bf16_mma<DT>) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[t]),
                                                         __builtin_bit_cast(bf16x8, bfrag[t]), acc, 0, 0, 0);
        } else if constexpr (DT == DT_SPLIT) {
            // rows [hi | lo]: k-step t < KSTEPS / 2 of the hi half pairs with step
            // t + KSTEPS / 2 of the lo half (same elements); three products per pair
            constexpr int HK = KSTEPS / 2;
            if (t < HK) {
                const bf16x8 ah = __builtin_bit_cast(bf16x8, af[t]), al = __builtin_bit_cast(bf16x8, af[t + HK]);
                const bf16x8 bh = __builtin_bit_cast(bf16x8, bfrag[t]), bl = __builtin_bit_cast(bf16x8, bfrag[t + HK]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
            }
        } else {
            static_assert(dt_bf16_mma<DT>, "FP8 codes reach the matrix cores widened to BF16");
        }
    }
    return acc;
}

// Register-prefetch form, used for rows shorter than 512 bytes (one group of 32 users
// per wave, tiles of 64 items staged through registers).  Two modes over the same
// matrix-core pipeline.
//  TK_MAIN: streaming top-C.  A score enters the user's candidate buffer only if it
//    beats the user's register threshold (seeded per user); a full buffer is compacted to
//    its C best by a wave radix select, which also raises the threshold to the running
//    C-th best.  The final threshold bounds every item left out.
//  TK_SEED: per user, an estimate of the score that about target items of the whole set
//    exceed, from a stratified item sample: each lane keeps the TK_T largest of its half
//    of the sample rows in registers, and the user's estimate is the smaller of its two
//    lanes' TK_T-th largest (at least 2*TK_T sample items reach it).  The estimate is only
//    a starting point: the main pass and the refine certificate never rely on it.
//
// The item stream is cut into 32-item blocks; a wave's MFMA output for one block is
// 32 items x the wave's 32 users (one user column per lane).  Item tiles of TK_IT_REG rows
// are double-buffered in LDS with one barrier per tile; the next tile waits in
// registers meanwhile.  The epilogue of block b (threshold compares and appends, or
// the register top-T of the seed pass) runs before block b + 1 is accumulated: the
// other resident waves keep the matrix cores busy meanwhile.
template <int DT, int DPT, int GPL, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((DT == DT_F32 && DPT >= 256) ? 1 : 2, 8))) void k_topk_reg(TopkArgs a)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int ROWB = DPT * EB;                // bytes of one stored row
    constexpr int LROW = ROWB + 16;               // padded LDS row (bank spread)
    constexpr int KSTEPS = ROWB / 32;             // 16-byte fragments per half row
    constexpr int IT = ROWB >= 512 ? 32 : TK_IT_REG;  // items per tile (LDS: two tiles per workgroup)
    constexpr int BPT = IT / 32;                  // MFMA blocks per tile
    constexpr int CHUNKS = IT * (ROWB / 16);      // 16-byte chunks per tile
    constexpr int PF = (CHUNKS + 255) / 256;      // chunks per thread
    constexpr int SGPL = MODE == TK_MAIN ? GPL : 1;
    __shared__ __attribute__((aligned(16))) uint8_t tile[2][IT * LROW];
    __shared__ float tscale[3][dt_scaled<DT> ? IT : 1];
    __shared__ int hist_all[TK_WAVES][MODE == TK_MAIN ? 256 : 1];
    __shared__ uint32_t stage_all[TK_WAVES][SGPL * 64];

    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int h = l >> 5;
    int* hist = hist_all[w];
    uint32_t* stage = stage_all[w];
    const int segl = blockIdx.y;
    const int seg = a.seg_base + segl;
    const int64_t seg0 = a.v0 + (int64_t)segl * a.seg_len;
    int64_t seg1 = seg0 + a.seg_len;
    if (seg1 > a.v1) seg1 = a.v1;
    const int seg_rows = seg1 > seg0 ? (int)(seg1 - seg0) : 0;   // segment-relative from here on
    const int ntiles = (seg_rows + IT - 1) / IT;
    const int nblk = ntiles * BPT;

    // ---- resident user fragments (the B operand), one user column per lane
    const int64_t ug = (int64_t)blockIdx.x * (TK_WAVES * 32) + (int64_t)w * 32 + (l & 31);
    const bool uok = ug < a.m;
    i32x4 bfrag[KSTEPS];
    {
        const uint8_t* row = (const uint8_t*)a.users + (uok ? ug : 0) * ROWB;
#pragma unroll
        for (int t = 0; t < KSTEPS; t++) {
            i32x4 z = {0, 0, 0, 0};
            bfrag[t] = uok ? *(const i32x4*)(row + t * 32 + h * 16) : z;
        }
    }
    float theta = -__builtin_inff();
    if (MODE == TK_MAIN && uok && a.theta_init) theta = a.theta_init[ug * a.theta_stride];
    if (!uok) theta = __builtin_inff();   // +inf: nothing enters
    const float su = (dt_scaled<DT> && uok) ? a.user_scales[ug] : 1.0f;
    const int HG = a.G / 2;
    // the workgroup's users' buffers start at wbuf; this lane's half at wbuf + loff
    // (a lane past the last user never appends: its threshold is +inf)
    // (buffer stores: an offset outside the workgroup's records is dropped)
    const int64_t wusers = std::min<int64_t>(TK_WAVES * 32, a.m - (int64_t)blockIdx.x * (TK_WAVES * 32));
    const __amdgpu_buffer_rsrc_t wrsrc = __builtin_amdgcn_make_buffer_rsrc(
        a.buf + (int64_t)blockIdx.x * (TK_WAVES * 32) * a.nseg_total * a.G, (short)0,
        (int)(wusers * a.nseg_total * a.G * (int64_t)sizeof(uint2)), 0x00020000);
    const uint32_t loff8 = 8u * (uint32_t)(((w * 32 + (l & 31)) * a.nseg_total + seg) * a.G + h * HG);
    uint32_t off = loff8;                                   // byte offset of this lane's next entry
    const uint32_t off_full = loff8 + 8u * (uint32_t)(HG - 16);   // past it a block may overflow the half
    float top[MODE == TK_SEED ? TK_T : 1];
#pragma unroll
    for (int i = 0; i < (MODE == TK_SEED ? TK_T : 1); i++) top[i] = -__builtin_inff();

    // ---- item tiles: registers hold tile T + 1 while tile T is scored
    auto load_chunk = [&](int tt, int c) -> i32x4 {
        const int r = c / (ROWB / 16), c16 = c % (ROWB / 16);
        const int64_t v = seg0 + tt * IT + r;
        i32x4 val = {0, 0, 0, 0};
        if (c < CHUNKS && v < seg1)
            val = *(const i32x4*)((const uint8_t*)a.items + v * ROWB + c16 * 16);
        return val;
    };
    i32x4 pf[PF];
    auto prefetch = [&](int tt) {
        if constexpr (MODE == TK_MAIN) {
            // the segment's rows are contiguous: chunk c of the tile lies c * 16 bytes past
            // its first row, and the descriptor ends with the tile's last row (chunks past
            // it, in the segment's last tile, read zeros)
            const int r0 = tt * IT;
            const int rows = seg_rows - r0 < IT ? seg_rows - r0 : IT;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)((const uint8_t*)a.items + (seg0 + r0) * ROWB), (short)0, rows * ROWB, 0x00020000);
#pragma unroll
            for (int e = 0; e < PF; e++)
                pf[e] = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                      rs, (int)(threadIdx.x + 256 * e) * 16, 0, 0));
        } else {
#pragma unroll
            for (int e = 0; e < PF; e++) pf[e] = load_chunk(tt, threadIdx.x + 256 * e);
        }
    };
    auto stage_tile = [&](int tt) {   // registers -> LDS buffer of tile tt
        uint8_t* dst = tile[tt & 1];
#pragma unroll
        for (int e = 0; e < PF; e++) {
            const int c = threadIdx.x + 256 * e;
            if (c < CHUNKS) *(i32x4*)(dst + (c / (ROWB / 16)) * LROW + (c % (ROWB / 16)) * 16) = pf[e];
        }
        if (dt_scaled<DT> && threadIdx.x < IT) {
            const int64_t v = seg0 + tt * IT + threadIdx.x;
            tscale[tt % 3][threadIdx.x] = v < seg1 ? a.item_scales[v] : 0.f;
        }
    };

    // scores of block b as they enter the epilogue, in place (FP8 scaled, rows past the
    // end -inf)
    auto scores = [&](f32x16& v, int b) {
        const int tt = b / BPT;
        const int rb = b % BPT;
        const int base = tt * IT + rb * 32;
        if constexpr (dt_scaled<DT>) {
#pragma unroll
            for (int r = 0; r < 16; r++) v[r] = (su * tscale[tt % 3][rb * 32 + mfma32_row(r, l)]) * v[r];
        }
        if (base + 32 > seg_rows) {   // wave-uniform: the segment's last block
            const int rem = seg_rows - base;
#pragma unroll
            for (int r = 0; r < 16; r++)
                if (mfma32_row(r, l) >= rem) v[r] = -__builtin_inff();
        }
    };
    // the register top-T of the seed pass: a row enters only if it beats the list's last
    // entry (quads and rows that no lane passes are skipped)
    auto early = [&](const f32x16& v) -> uint32_t {
        uint32_t pm = 0u;
        if constexpr (MODE == TK_SEED) {
            float q4[4];
#pragma unroll
            for (int jq = 0; jq < 4; jq++)
                q4[jq] = fmaxf(fmaxf(v[4 * jq], v[4 * jq + 1]), fmaxf(v[4 * jq + 2], v[4 * jq + 3]));
            if (fmaxf(fmaxf(q4[0], q4[1]), fmaxf(q4[2], q4[3])) > top[TK_T - 1]) {
#pragma unroll
                for (int jq = 0; jq < 4; jq++) {
                    if (q4[jq] > top[TK_T - 1]) {
#pragma unroll
                        for (int e4 = 0; e4 < 4; e4++) {
                            float x = v[4 * jq + e4];
                            if (x > top[TK_T - 1]) {
#pragma unroll
                                for (int i = 0; i < TK_T; i++) {
                                    const float hi = fmaxf(top[i], x);
                                    x = fminf(top[i], x);
                                    top[i] = hi;
                                }
                            }
                        }
                    }
                }
            }
        }
        return pm;
    };
    // appends of block b (main pass)
    auto late = [&](const f32x16& v, uint32_t, int b) {
        if constexpr (MODE == TK_MAIN) {
            // compaction of the users whose half-buffer could overflow in this block (a lane
            // appends at most 16 entries per block)
            const uint64_t need = ballot64(off > off_full);
            if (need) {
                const int cnt = (int)((off - loff8) >> 3);
                uint32_t um = (uint32_t)need | (uint32_t)(need >> 32);
                while (um) {
                    const int ul = __builtin_ctz(um);
                    um &= um - 1;
                    const int c0 = __shfl(cnt, ul), c1 = __shfl(cnt, ul + 32);
                    const int64_t ugl = __shfl(ug, ul);
                    uint2* rg = a.buf + (ugl * a.nseg_total + seg) * (int64_t)a.G;
                    const uint32_t T = select_user_call(rg, c0, rg + HG, c1, a.C, hist, stage);
                    if ((l & 31) == ul) {
                        theta = ord_f32(T);
                        off = loff8 + (h ? 0u : 8u * (uint32_t)a.C);
                    }
                }
            }
            // each lane owns its half of the user's buffer: no cross-lane counts; a row
            // that no lane passes costs one compare and one branch.  Entries are the raw
            // score bits and the item position, at 32-bit offsets from the workgroup's
            // buffer base.
            const uint32_t pbase = (uint32_t)seg0 + (uint32_t)(b * 32) + 4u * (uint32_t)h;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                if (v[r] > theta) {
                    const u32x2 e = {__float_as_uint(v[r]), pbase + (uint32_t)(8 * (r / 4) + (r % 4))};
                    __builtin_amdgcn_raw_buffer_store_b64(e, wrsrc, (int)off, 0, 0);
                    off += 8u;
                }
            }
        }
    };

    if (nblk > 0) {
        prefetch(0);
        stage_tile(0);
        __syncthreads();
        if (ntiles > 1) prefetch(1);
        f32x16 acc = mfma_block1<DT, KSTEPS, LROW>(tile[0], 0, bfrag);
        for (int b = 0; b < nblk; b++) {
            scores(acc, b);
            late(acc, early(acc), b);
            if (b + 1 < nblk) {
                const int tn = (b + 1) / BPT;
                if ((b + 1) % BPT == 0) {      // block b + 1 opens tile tn
                    stage_tile(tn);
                    __syncthreads();
                    if (tn + 1 < ntiles) prefetch(tn + 1);
                }
                acc = mfma_block1<DT, KSTEPS, LROW>(tile[tn & 1], ((b + 1) % BPT) * 32, bfrag);
            }
        }
    }

    if constexpr (MODE == TK_SEED) {
        const float mine = top[TK_T - 1];
        const float other = __shfl_xor(mine, 32);
        if (l < 32 && uok) a.theta_out[ug] = fminf(mine, other);
    } else {
        // the buffer halves may hold up to G entries together; the refine pass selects
        if (uok) {
            a.cnt[(ug * a.nseg_total + seg) * 2 + h] = (int)((off - loff8) >> 3);
            if (h == 0) a.tau[ug * a.nseg_total + seg] = theta;
        }
    }
}

template <int DT, int DPT>
constexpr int topk_ng()
{
    // Two groups where a block's k-loop is long (rows of 512 bytes and more), so that the
    // LDS reads per product halve; the two groups' resident fragments (KSTEPS i32x4 each)
    // must fit in 128 VGPRs.  Shorter rows keep one group and twice the workgroups.
    constexpr int rowb = DPT * Elt<DT>::bytes;
    return (rowb >= 512 || DT == DT_FP8) && (rowb / 32) * 4 * 2 <= 128 ? 2 : 1;
}

// Direct (DMA) load of 16 (or 4) bytes per lane into LDS at lds + 16 * lane (4 * lane),
// through a buffer descriptor: bytes past num_records read as zero.  Written as one asm
// block with no register outputs, so that the compiler does not order every later LDS
// read behind it; the kernel waits for these loads itself (vmcnt, then a barrier).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 tk_rsrc(const void* base, uint32_t bytes)
{
    const uint64_t b = (uint64_t)base;
    u32x4 r;
    r.x = (uint32_t)b;
    r.y = (uint32_t)(b >> 32) & 0xffffu;   // stride 0
    r.z = bytes;
    r.w = 0x00020000u;
    return r;
}
__device__ __forceinline__ void tk_dma16(u32x4 rsrc, uint32_t lds, uint32_t voff)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                 :
                 : "s"(lds), "v"(voff), "s"(rsrc)
                 : "memory", "m0");
}
__device__ __forceinline__ void tk_dma4(u32x4 rsrc, uint32_t lds, uint32_t voff)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dword %1, %2, 0 offen lds"
                 :
                 : "s"(lds), "v"(voff), "s"(rsrc)
                 : "memory", "m0");
}

#define TK_LDS(p) ((__attribute__((address_space(3))) void*)(p))
#define TK_GLB(p) ((__attribute__((address_space(1))) void*)(p))

template <int DT, int DPT, int GPL, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_topk_ring(TopkArgs a)
{
    constexpr int NG = topk_ng<DT, DPT>();
    constexpr int UPW = 32 * NG;                  // users per wave
    constexpr int UPB = TK_WAVES * UPW;           // users per workgroup
    constexpr int EB = Elt<DT>::bytes;
    constexpr int ROWB = DPT * EB;
    constexpr int LROW = ROWB + 16;               // padded LDS row (bank spread)
    constexpr int CPR = LROW / 16;                // 16-byte chunks per padded row
    constexpr int KSTEPS = ROWB / 32;
    constexpr int IT = 32;                        // items per tile: one MFMA block
    constexpr int BPT = IT / 32;
    constexpr int NLD = (IT * LROW + 1023) / 1024;   // 1 KB DMA loads per tile
    constexpr int LPW = (NLD + TK_WAVES - 1) / TK_WAVES;
    constexpr int TBYTES = NLD * 1024;
    constexpr int SGPL = MODE == TK_MAIN ? GPL : 1;
    // scaled rows: the user's scale stays out of the per-score work (see below)
    constexpr bool FOLD = dt_scaled<DT>;
    __shared__ __attribute__((aligned(1024))) uint8_t ring0[TBYTES];
    __shared__ __attribute__((aligned(1024))) uint8_t ring1[TBYTES];
    __shared__ __attribute__((aligned(1024))) uint8_t ring2[TBYTES];
    __shared__ __attribute__((aligned(256))) float sc0[dt_scaled<DT> ? 64 : 1];
    __shared__ __attribute__((aligned(256))) float sc1[dt_scaled<DT> ? 64 : 1];
    __shared__ __attribute__((aligned(256))) float sc2[dt_scaled<DT> ? 64 : 1];
    __shared__ int hist_all[TK_WAVES][MODE == TK_MAIN ? 256 : 1];
    __shared__ uint32_t stage_all[TK_WAVES][SGPL * 64];
    __shared__ uint32_t doff_all[TK_WAVES][LPW][64];   // each lane's direct-load offsets

    const int l = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (SGPR)
    const int h = l >> 5;
    int* hist = hist_all[w];
    uint32_t* stage = stage_all[w];
    const int segl = blockIdx.y;
    const int seg = a.seg_base + segl;
    const int64_t seg0 = a.v0 + (int64_t)segl * a.seg_len;
    int64_t seg1 = seg0 + a.seg_len;
    if (seg1 > a.v1) seg1 = a.v1;
    const int seg_rows = seg1 > seg0 ? (int)(seg1 - seg0) : 0;
    const int ntiles = (seg_rows + IT - 1) / IT;

    // ---- resident user fragments (B operands), one user column per lane and group
    // user of group g for this lane (recomputed where needed: registers are scarce)
    auto user_of = [&](int g) -> int64_t {
        int lw = (l & 31) + w * UPW + g * 32;
        asm volatile("" : "+v"(lw));
        return (int64_t)blockIdx.x * UPB + lw;
    };
    i32x4 bfrag[NG][KSTEPS];
    float theta[NG], su[NG];
#pragma unroll
    for (int g = 0; g < NG; g++) {
        const int64_t ug = user_of(g);
        const bool uok = ug < a.m;
        const uint8_t* row = (const uint8_t*)a.users + (uok ? ug : 0) * ROWB;
#pragma unroll
        for (int t = 0; t < KSTEPS; t++) {
            i32x4 z = {0, 0, 0, 0};
            // BF16 forms: unit t is bytes [32 t + 16 h, + 16); FP8 codes: units t, t + 1 (t
            // even) are the 32 bytes [64 (t / 2) + 32 h, + 32) of a 64-wide k step
            const int fo = DT == DT_FP8 ? (t >> 1) * 64 + h * 32 + (t & 1) * 16 : t * 32 + h * 16;
            bfrag[g][t] = uok ? *(const i32x4*)(row + fo) : z;
        }
        theta[g] = -__builtin_inff();
        if (MODE == TK_MAIN && uok && a.theta_init) theta[g] = a.theta_init[ug * a.theta_stride];
        if (!uok) theta[g] = __builtin_inff();
        su[g] = (dt_scaled<DT> && uok) ? a.user_scales[ug] : 1.0f;
        if constexpr (FOLD) {
            // a negative scale moves into the operand (negating BF16 values is exact)
            if (su[g] < 0.f) {
                su[g] = -su[g];
#pragma unroll
                for (int t = 0; t < KSTEPS; t++) bfrag[g][t] ^= (int)(DT == DT_FP8 ? 0x80808080u : 0x80008000u);
            }
        }
    }
    // FP8: the user's scale is folded into its threshold.  The main pass compares
    // w = s_p raw against ths = RD(theta / s_u): an item left out has w <= ths, so its
    // fast score RN(s_u w) <= s_u ths <= theta.  Appended entries carry RN(s_u w).  The
    // seed pass keeps its lists in w (the order is the same for s_u > 0).
    float ths[NG];
    auto fold = [&](float t, float s) -> float {
        if (!(s > 0.f)) return 0.f > t ? -__builtin_inff() : __builtin_inff();
        // one step below the rounded quotient: at most t / s (the rounding error is at
        // most half a step), infinities stay
        const float q = __fdiv_rn(t, s);
        if (!(fabsf(q) < __builtin_inff())) return q;
        const uint32_t b = __float_as_uint(q);
        return __uint_as_float(q > 0.f ? b - 1u : (q == 0.f ? 0x80000001u : b + 1u));
    };
#pragma unroll
    for (int g = 0; g < NG; g++) ths[g] = FOLD ? fold(theta[g], su[g]) : theta[g];
    const int HG = a.G / 2;
    const int64_t wusers = std::min<int64_t>(UPB, a.m - (int64_t)blockIdx.x * UPB);
    const __amdgpu_buffer_rsrc_t wrsrc = __builtin_amdgcn_make_buffer_rsrc(
        a.buf + (int64_t)blockIdx.x * UPB * a.nseg_total * a.G, (short)0,
        (int)(wusers * a.nseg_total * a.G * (int64_t)sizeof(uint2)), 0x00020000);
    uint32_t loff8[NG], off[NG];
#pragma unroll
    for (int g = 0; g < NG; g++) {
        loff8[g] = 8u * (uint32_t)(((w * UPW + g * 32 + (l & 31)) * a.nseg_total + seg) * a.G + h * HG);
        off[g] = loff8[g];
    }
    // Compaction trigger per half-buffer.  A half must keep room for one block's 16
    // appends; below that, compacting once about C new entries have arrived raises the
    // threshold to the running C-th best early (the items come in descending norm
    // order), which cuts the later appends.  After a compaction the C survivors sit in
    // the first half, so that half triggers at 2C and the second at C.
    const uint32_t full_rel = 8u * (uint32_t)std::min(HG - 16, h ? a.C : 2 * a.C);
    float top[NG][MODE == TK_SEED ? TK_T : 1];
#pragma unroll
    for (int g = 0; g < NG; g++)
#pragma unroll
        for (int i = 0; i < (MODE == TK_SEED ? TK_T : 1); i++) top[g][i] = -__builtin_inff();

    // ---- DMA map: load j of this wave fills LDS bytes [k * 1024, (k + 1) * 1024) of a
    // slot, k = w * LPW + j; lane l writes 16 bytes at k * 1024 + 16 l, which is chunk
    // (pos % CPR) of padded row pos / CPR (the padding chunk takes a dummy copy of chunk 0).
    // The byte offsets of a lane's loads within the tile's rows are the same for every
    // tile: computed once into LDS (in registers they would cost five VGPRs, recomputed
    // per tile about forty vector instructions; unsigned: the division by the constant
    // CPR is a multiply-high and a shift)
#pragma unroll
    for (int j = 0; j < LPW; j++) {
        const unsigned pos = (unsigned)(w * LPW * 64 + l) + (unsigned)j * 64u;
        const unsigned c = pos % (unsigned)CPR;
        doff_all[w][j][l] = (pos / (unsigned)CPR) * (unsigned)ROWB + (c < (unsigned)(ROWB / 16) ? c : 0u) * 16u;
    }
    auto issue = [&](uint8_t* ring, float* sc, int tt) {
        const int r0 = tt * IT;
        const int rows = seg_rows - r0 < IT ? seg_rows - r0 : IT;
        {
            // the tile's rows are contiguous (the seed pass reads the gathered sample);
            // loads past its last row read zeros
            const u32x4 rs = tk_rsrc((const uint8_t*)a.items + (seg0 + r0) * ROWB, (uint32_t)(rows * ROWB));
            const uint32_t lbase = (uint32_t)(uintptr_t)TK_LDS(ring);
            // all offsets read before the first load: the loads' asm blocks order every
            // later LDS read behind them
            uint32_t dv[LPW];
#pragma unroll
            for (int j = 0; j < LPW; j++) dv[j] = doff_all[w][j][l];
#pragma unroll
            for (int j = 0; j < LPW; j++) {
                if (w * LPW + j < NLD) tk_dma16(rs, lbase + (uint32_t)((w * LPW + j) * 1024), dv[j]);
            }
            if constexpr (dt_scaled<DT>) {
                if (w == 0) {
                    const u32x4 rsc = tk_rsrc(a.item_scales + seg0 + r0, (uint32_t)(rows * 4));
                    tk_dma4(rsc, (uint32_t)(uintptr_t)TK_LDS(sc), (uint32_t)(l * 4));
                }
            }
        }
    };
    // Before tile tt is read: this wave's loads of tile tt have landed when no more than
    // its loads of tile tt + 1 (if issued; VMEM operations complete in order) are in
    // flight.  The counts are per wave: NLD loads are spread LPW to a wave, the last
    // waves may take fewer, and wave 0 also loads the scales.
    auto wait_tile = [&](bool next_issued) {
#define TK_WAITV(n) __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))
        constexpr int n0 = (NLD < LPW ? NLD : LPW) + (dt_scaled<DT> ? 1 : 0);
        constexpr int n1 = NLD - LPW <= 0 ? 0 : (NLD - LPW < LPW ? NLD - LPW : LPW);
        constexpr int n2 = NLD - 2 * LPW <= 0 ? 0 : (NLD - 2 * LPW < LPW ? NLD - 2 * LPW : LPW);
        constexpr int n3 = NLD - 3 * LPW <= 0 ? 0 : (NLD - 3 * LPW < LPW ? NLD - 3 * LPW : LPW);
        static_assert(TK_WAVES == 4 && n0 < 64, "wait counts assume four waves");
        if (!next_issued) TK_WAITV(0);
        else if (w == 0) TK_WAITV(n0);
        else if (w == 1) TK_WAITV(n1);
        else if (w == 2) TK_WAITV(n2);
        else TK_WAITV(n3);
#undef TK_WAITV
    };

    // scores of block b in place (FP8 scaled, rows past the end -inf)
    auto scores = [&](f32x16 (&v)[NG], const float* sc, int tt, int rb) {
        const int base = tt * IT + rb * 32;
        if constexpr (dt_scaled<DT>) {
            const float* ts = sc + rb * 32 + 4 * h;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const f32x4 s4 = *(const f32x4*)(ts + 8 * j);
#pragma unroll
                for (int g = 0; g < NG; g++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        if constexpr (FOLD) v[g][4 * j + e] = s4[e] * v[g][4 * j + e];
                        else v[g][4 * j + e] = (su[g] * s4[e]) * v[g][4 * j + e];
                    }
            }
        }
        if (base + 32 > seg_rows) {
            const int rem = seg_rows - base;
#pragma unroll
            for (int g = 0; g < NG; g++)
#pragma unroll
                for (int r = 0; r < 16; r++)
                    if (mfma32_row(r, l) >= rem) v[g][r] = -__builtin_inff();
        }
    };
    auto seed_top = [&](const f32x16 (&v)[NG]) {
        if constexpr (MODE == TK_SEED) {
#pragma unroll
            for (int g = 0; g < NG; g++) {
                // a row enters the lane's sorted list only if it beats the list's last
                // entry; quads and rows that no lane of the wave passes are skipped
                float q4[4];
#pragma unroll
                for (int jq = 0; jq < 4; jq++)
                    q4[jq] = fmaxf(fmaxf(v[g][4 * jq], v[g][4 * jq + 1]), fmaxf(v[g][4 * jq + 2], v[g][4 * jq + 3]));
                const float mx = fmaxf(fmaxf(q4[0], q4[1]), fmaxf(q4[2], q4[3]));
                if (mx > top[g][TK_T - 1]) {
#pragma unroll
                    for (int jq = 0; jq < 4; jq++) {
                        if (q4[jq] > top[g][TK_T - 1]) {
#pragma unroll
                            for (int e4 = 0; e4 < 4; e4++) {
                                const float x = v[g][4 * jq + e4];
                                if (x > top[g][TK_T - 1]) {
                                    // sorted insertion, the last entry dropped: entry i becomes
                                    // max(t_i, min(x, t_(i-1))), the median of the three
#pragma unroll
                                    for (int i = TK_T - 1; i > 0; i--)
                                        top[g][i] = __builtin_amdgcn_fmed3f(top[g][i - 1], top[g][i], x);
                                    top[g][0] = fmaxf(top[g][0], x);
                                }
                            }
                        }
                    }
                }
            }
        }
    };
    auto appends = [&](const f32x16 (&v)[NG], int b) {
        if constexpr (MODE == TK_MAIN) {
#pragma unroll
            for (int g = 0; g < NG; g++) {
                const uint64_t need = ballot64(off[g] - loff8[g] > full_rel);
                if (need) {
                    const int cnt = (int)((off[g] - loff8[g]) >> 3);
                    uint32_t um = (uint32_t)need | (uint32_t)(need >> 32);
                    while (um) {
                        const int ul = __builtin_ctz(um);
                        um &= um - 1;
                        const int c0 = __shfl(cnt, ul), c1 = __shfl(cnt, ul + 32);
                        const int64_t ugl = (int64_t)blockIdx.x * UPB + w * UPW + g * 32 + ul;
                        uint2* rg = a.buf + (ugl * a.nseg_total + seg) * (int64_t)a.G;
                        const uint32_t T = select_user(rg, c0, rg + HG, c1, a.C, hist, stage);
                        if ((l & 31) == ul) {
                            theta[g] = ord_f32(T);
                            ths[g] = FOLD ? fold(theta[g], su[g]) : theta[g];
                            off[g] = loff8[g] + (h ? 0u : 8u * (uint32_t)a.C);
                        }
                    }
                    // nothing of the compaction's own loads stays in flight: the waits of
                    // the tile loop then count the tile loads only
                    __builtin_amdgcn_s_waitcnt(0);
                }
                // maxima of the lane's four row quads (rows 8 j + 4 h + e, e < 4): a quad that
                // no lane of the wave passes is skipped with one scalar branch
                float q4[4];
#pragma unroll
                for (int j = 0; j < 4; j++)
                    q4[j] = fmaxf(fmaxf(v[g][4 * j], v[g][4 * j + 1]), fmaxf(v[g][4 * j + 2], v[g][4 * j + 3]));
                const float mx = fmaxf(fmaxf(q4[0], q4[1]), fmaxf(q4[2], q4[3]));
                if (mx > ths[g]) {
                    const uint32_t pbase = (uint32_t)seg0 + (uint32_t)(b * 32) + 4u * (uint32_t)h;
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        if (q4[j] > ths[g]) {
#pragma unroll
                            for (int e4 = 0; e4 < 4; e4++) {
                                const int r = 4 * j + e4;
                                if (v[g][r] > ths[g]) {
                                    const float fs = FOLD ? su[g] * v[g][r] : v[g][r];
                                    const u32x2 e = {__float_as_uint(fs), pbase + (uint32_t)(8 * j + e4)};
                                    __builtin_amdgcn_raw_buffer_store_b64(e, wrsrc, (int)off[g], 0, 0);
                                    off[g] += 8u;
                                }
                            }
                        }
                    }
                }
            }
        }
    };
    // one tile from its ring slot (static per call site, so that the compiler tells the
    // slots' DMA writes apart)
    auto tile = [&](uint8_t* ring, float* sc, uint8_t* ring_next2, float* sc_next2, int tt) {
        wait_tile(tt + 1 < ntiles);
        __builtin_amdgcn_s_barrier();
        if (tt + 2 < ntiles) issue(ring_next2, sc_next2, tt + 2);
#pragma unroll
        for (int rb = 0; rb < BPT; rb++) {
            f32x16 acc[NG];
            mfma_block<DT, KSTEPS, LROW, NG>(ring, rb * 32, bfrag, acc);
            scores(acc, sc, tt, rb);
            seed_top(acc);
            appends(acc, tt * BPT + rb);
        }
    };

    // the user fragments and thresholds are in registers before the first tile load: the
    // in-loop waits then count the tile loads only
    __builtin_amdgcn_s_waitcnt(0);
    if (ntiles > 0) {
        issue(ring0, sc0, 0);
        if (ntiles > 1) issue(ring1, sc1, 1);
        for (int tt = 0; tt < ntiles; tt += 3) {
            tile(ring0, sc0, ring2, sc2, tt);
            if (tt + 1 < ntiles) tile(ring1, sc1, ring0, sc0, tt + 1);
            if (tt + 2 < ntiles) tile(ring2, sc2, ring1, sc1, tt + 2);
        }
    }

#pragma unroll
    for (int g = 0; g < NG; g++) {
        const int64_t ug = user_of(g);
        const bool uok = ug < a.m;
        if constexpr (MODE == TK_SEED) {
            const float mine = top[g][TK_T - 1];
            const float other = __shfl_xor(mine, 32);
            // with the scale folded out the lists hold s_p raw; the estimate is s_u times
            // its threshold (an estimate only: the certificate does not depend on it)
            const float t = fminf(mine, other);
            if (l < 32 && uok) a.theta_out[ug] = (FOLD && su[g] > 0.f) ? su[g] * t : t;
        } else {
            if (uok) {
                a.cnt[(ug * a.nseg_total + seg) * 2 + h] = (int)((off[g] - loff8[g]) >> 3);
                if (h == 0) a.tau[ug * a.nseg_total + seg] = theta[g];
            }
        }
    }
}

// The kernel of one instance: the DMA-ring form for rows of 512 bytes and more, the
// register-prefetch form for shorter rows.
template <int DT, int DPT>
constexpr bool topk_ring()
{
    return DPT * Elt<DT>::bytes >= 512 || DT == DT_FP8;
}
template <int DT, int DPT, int GPL, int MODE>
static void (*topk_kernel())(TopkArgs)
{
    if constexpr (topk_ring<DT, DPT>()) return &k_topk_ring<DT, DPT, GPL, MODE>;
    else return &k_topk_reg<DT, DPT, GPL, MODE>;
}
template <int DT, int DPT>
constexpr int topk_upb()
{
    return topk_ring<DT, DPT>() ? TK_WAVES * 32 * topk_ng<DT, DPT>() : TK_WAVES * 32;
}

template <int DT, int DPT, int MODE>
static void topk_dispatch_g(const TopkArgs& a, hipStream_t s)
{
    constexpr int UPB = topk_upb<DT, DPT>();
    dim3 grid((unsigned)((a.m + UPB - 1) / UPB), (unsigned)a.nseg);
    if constexpr (MODE == TK_SEED) {
        hipLaunchKernelGGL((topk_kernel<DT, DPT, 1, TK_SEED>()), grid, dim3(256), 0, s, a);
    } else {
        const int gpl = a.G / 64;
        if (gpl == 2) hipLaunchKernelGGL((topk_kernel<DT, DPT, 2, TK_MAIN>()), grid, dim3(256), 0, s, a);
        else if (gpl == 4) hipLaunchKernelGGL((topk_kernel<DT, DPT, 4, TK_MAIN>()), grid, dim3(256), 0, s, a);
        else if (gpl == 8) hipLaunchKernelGGL((topk_kernel<DT, DPT, 8, TK_MAIN>()), grid, dim3(256), 0, s, a);
        else if (gpl == 16) hipLaunchKernelGGL((topk_kernel<DT, DPT, 16, TK_MAIN>()), grid, dim3(256), 0, s, a);
        else fail(RKMIPS_EINVAL, "internal: unsupported candidate buffer size");
    }
}

template <int DT>
static int upb_d(int ld)
{
    if constexpr (DT == DT_SPLIT) return ld == 64 ? topk_upb<DT, 64>() : topk_upb<DT, 128>();
    else {
        switch (ld) {
        case 32: return topk_upb<DT, 32>();
        case 64: return topk_upb<DT, 64>();
        case 128: return topk_upb<DT, 128>();
        default: return topk_upb<DT, 256>();
        }
    }
}

int topk_users_per_block(int dtype, int ld)
{
    if (dtype == DT_F32) return upb_d<DT_F32>(ld);
    if (dtype == DT_BF16) return upb_d<DT_BF16>(ld);
    if (dtype == DT_FP8B) return upb_d<DT_FP8B>(ld);
    return upb_d<DT_SPLIT>(ld);
}

// Workgroups of the main pass that one compute unit holds at once (registers and LDS).
template <int DT, int DPT>
static int resident_g(int G)
{
    int nb = 0;
    hipError_t e = hipSuccess;
    const int gpl = G / 64;
    if (gpl == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, topk_kernel<DT, DPT, 2, TK_MAIN>(), 256, 0);
    else if (gpl == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, topk_kernel<DT, DPT, 4, TK_MAIN>(), 256, 0);
    else if (gpl == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, topk_kernel<DT, DPT, 8, TK_MAIN>(), 256, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, topk_kernel<DT, DPT, 16, TK_MAIN>(), 256, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

template <int DT>
static int resident_d(int ld, int G)
{
    if constexpr (DT == DT_SPLIT) {   // pair rows of FP32 data: 2 x 32, 2 x 64
        return ld == 64 ? resident_g<DT, 64>(G) : resident_g<DT, 128>(G);
    } else {
        switch (ld) {
        case 32: return resident_g<DT, 32>(G);
        case 64: return resident_g<DT, 64>(G);
        case 128: return resident_g<DT, 128>(G);
        default: return resident_g<DT, 256>(G);
        }
    }
}

// Cached per (device, dtype, ld, G): the occupancy query costs tens of microseconds.
int topk_resident_blocks(int dtype, int ld, int G)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, dtype, ld, G);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int nb;
    if (dtype == DT_F32) nb = resident_d<DT_F32>(ld, G);
    else if (dtype == DT_BF16) nb = resident_d<DT_BF16>(ld, G);
    else if (dtype == DT_FP8B) nb = resident_d<DT_FP8B>(ld, G);
    else if (dtype == DT_SPLIT) nb = resident_d<DT_SPLIT>(ld, G);
    else fail(RKMIPS_EINVAL, "internal: no matrix-core path for this operand type");
    std::lock_guard<std::mutex> g(mu);
    cache[key] = nb;
    return nb;
}

template <int DT, int MODE>
static void topk_dispatch(const TopkArgs& a, hipStream_t s)
{
    if constexpr (DT == DT_SPLIT) {   // pair rows of FP32 data: 2 x 32, 2 x 64
        if (a.ld == 64) topk_dispatch_g<DT, 64, MODE>(a, s);
        else if (a.ld == 128) topk_dispatch_g<DT, 128, MODE>(a, s);
        else fail(RKMIPS_EINVAL, "internal: unsupported split row length");
    } else {
        switch (a.ld) {
        case 32: topk_dispatch_g<DT, 32, MODE>(a, s); break;
        case 64: topk_dispatch_g<DT, 64, MODE>(a, s); break;
        case 128: topk_dispatch_g<DT, 128, MODE>(a, s); break;
        case 256: topk_dispatch_g<DT, 256, MODE>(a, s); break;
        default: fail(RKMIPS_EINVAL, "internal: unsupported padded dimension");
        }
    }
}

// The stratified sample of the seed pass as contiguous rows: row v of dst is item
// ((2 v + 1) n) / (2 ns) of the norm-sorted operand rows (the middle of slice v of ns
// equal slices), with its scale.
__global__ void k_gather_sample(const i32x4* src, const float* scales, int64_t n, int64_t ns, int chunks,
                                i32x4* dst, float* dscales)
{
    const int64_t total = ns * chunks;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / chunks;
        const int c = (int)(t - v * chunks);
        const int64_t it = ((2 * v + 1) * n) / (2 * ns);
        dst[v * chunks + c] = src[it * chunks + c];
        if (c == 0 && scales) dscales[v] = scales[it];
    }
}

int topk_row_bytes(int dtype, int ld) { return ld * (dtype == DT_F32 ? 4 : dtype == DT_FP8 ? 1 : 2); }

void launch_gather_sample(int dtype, const void* items, const float* scales, int64_t n, int64_t ns, int ld,
                          void* dst, float* dscales, hipStream_t s)
{
    if (ns <= 0) return;
    const int rowb = topk_row_bytes(dtype, ld);
    if (rowb % 16 != 0 || ns > n) fail(RKMIPS_EINVAL, "internal: seed sample shape");
    const int chunks = rowb / 16;
    const int64_t total = ns * chunks;
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gather_sample, dim3(g), dim3(256), 0, s, (const i32x4*)items, scales, n, ns, chunks,
                       (i32x4*)dst, dscales);
    HIPC(hipGetLastError());
}

void launch_topk(int dtype, const TopkArgs& a, hipStream_t s)
{
    if (a.m <= 0 || a.v1 <= a.v0) return;
    if (dtype == DT_F32) topk_dispatch<DT_F32, TK_MAIN>(a, s);
    else if (dtype == DT_BF16) topk_dispatch<DT_BF16, TK_MAIN>(a, s);
    else if (dtype == DT_FP8B) topk_dispatch<DT_FP8B, TK_MAIN>(a, s);
    else if (dtype == DT_SPLIT) topk_dispatch<DT_SPLIT, TK_MAIN>(a, s);
    else fail(RKMIPS_EINVAL, "internal: no matrix-core path for this operand type");
    HIPC(hipGetLastError());
}

void launch_topk_seed(int dtype, const TopkArgs& a, hipStream_t s)
{
    if (a.m <= 0 || a.v1 <= a.v0) return;
    if (a.v1 - a.v0 > a.ns || a.ns > a.n || !a.theta_out) fail(RKMIPS_EINVAL, "internal: bad seed sample");
    if (dtype == DT_F32) topk_dispatch<DT_F32, TK_SEED>(a, s);
    else if (dtype == DT_BF16) topk_dispatch<DT_BF16, TK_SEED>(a, s);
    else if (dtype == DT_FP8B) topk_dispatch<DT_FP8B, TK_SEED>(a, s);
    else if (dtype == DT_FP8 && a.ld == 256) topk_dispatch_g<DT_FP8, 256, TK_SEED>(a, s);
    else if (dtype == DT_SPLIT) topk_dispatch<DT_SPLIT, TK_SEED>(a, s);
    else fail(RKMIPS_EINVAL, "internal: no matrix-core path for this operand type");
    HIPC(hipGetLastError());
}

}  // namespace rk
