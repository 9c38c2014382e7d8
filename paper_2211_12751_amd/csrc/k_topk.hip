// lambda build: for every user u, lambda_u^(j), j = 1..k_max, the j-th largest inner
// product of u over all items (Definition 1; the lower-bound array of Alg. 4 taken
// over all of P instead of the top-norm subset P').
//
// Pass 0 (k_topk, seed mode): on a stratified sample of the items, the matrix cores
//   score every user and each lane keeps its few largest scores in registers; their
//   order statistic estimates a per-user threshold that a fixed multiple of C items
//   of the whole set exceed.
// Pass 1 (k_topk, main mode): fused U.P^T on the matrix cores with a streaming per-user
//   top-C (C = k_max + slack).  A workgroup keeps 128-256 users' operand fragments in
//   registers and streams 64-item tiles of the norm-sorted items through LDS.  Every
//   MFMA output lane owns one user column; a score enters the user's candidate buffer
//   only if it beats the user's register threshold (starting at the seed estimate).
//   When a buffer fills, the wave compacts it to its C best entries with a wave radix
//   select and raises the threshold to the running C-th best.  The final threshold tau
//   bounds every item left out.
// Pass 2 (canonical FP64 rescoring and the certificate) is in k_refine.hip.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"
#include "internal.h"

namespace rk {

static constexpr int TK_WAVES = 4;
static constexpr int TK_IT = 64;  // items per LDS tile (two 32-row MFMA blocks)

// ------------------------------------------------------------------ fused GEMM + top-k
// Buffer compaction for the streaming pass, with the keys staged in LDS so that it needs
// few registers (it runs rarely, and the main loop keeps its register budget for
// occupancy): of the c0 entries at r0 and the c1 entries at r1, keep the C largest
// (ties at the threshold in staging order) in r0[0, C) and return the C-th largest key
// (orderable form; the entries themselves keep the raw score bits).  The kept entries
// move down in place: entry i lands at a position <= i, and r0 is read in full before r1.
__device__ __noinline__ uint32_t select_user(uint2* r0, int c0, const uint2* r1, int c1, int C, int* hist,
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

// Item at virtual position v of a launch: the norm-sorted array itself (main pass), or
// the stratified sample of `ns` items, one from the middle of each of ns equal slices of
// the norm-sorted order (seed pass).
template <int MODE>
__device__ __forceinline__ int64_t item_at(int64_t v, int64_t n, int64_t ns)
{
    if constexpr (MODE == TK_SEED) return ((2 * v + 1) * n) / (2 * ns);
    else return v;
}

// 32 x 32 block of scores on the matrix cores: rows = the 32 items of LDS rows
// [row0, row0 + 32) of a staged tile, columns = the wave's 32 users (register fragments).
template <int DT, int KSTEPS, int LROW>
__device__ __forceinline__ f32x16 mfma_block(const uint8_t* tile, int row0, const i32x4 (&bfrag)[KSTEPS])
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

// Two modes over the same matrix-core pipeline.
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
// 32 items x the wave's 32 users (one user column per lane).  Item tiles of TK_IT rows
// are double-buffered in LDS with one barrier per tile; the next tile waits in
// registers meanwhile.  The epilogue of block b (threshold compares and appends, or
// the register top-T of the seed pass) runs before block b + 1 is accumulated: the
// other resident waves keep the matrix cores busy meanwhile.
template <int DT, int DPT, int GPL, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((DT == DT_F32 && DPT >= 256) ? 1 : 2, 8))) void k_topk(TopkArgs a)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int ROWB = DPT * EB;                // bytes of one stored row
    constexpr int LROW = ROWB + 16;               // padded LDS row (bank spread)
    constexpr int KSTEPS = ROWB / 32;             // 16-byte fragments per half row
    constexpr int IT = ROWB >= 512 ? 32 : TK_IT;  // items per tile (LDS: two tiles per workgroup)
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
            val = *(const i32x4*)((const uint8_t*)a.items + item_at<MODE>(v, a.n, a.ns) * ROWB + c16 * 16);
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
            tscale[tt % 3][threadIdx.x] = v < seg1 ? a.item_scales[item_at<MODE>(v, a.n, a.ns)] : 0.f;
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
    // branch-free part of the epilogue: the register top-T of the seed pass
    auto early = [&](const f32x16& v) -> uint32_t {
        uint32_t pm = 0u;
        if constexpr (MODE == TK_SEED) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                float x = v[r];
#pragma unroll
                for (int i = 0; i < TK_T; i++) {
                    const float hi = fmaxf(top[i], x);
                    x = fminf(top[i], x);
                    top[i] = hi;
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
                    const uint32_t T = select_user(rg, c0, rg + HG, c1, a.C, hist, stage);
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
        f32x16 acc = mfma_block<DT, KSTEPS, LROW>(tile[0], 0, bfrag);
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
                acc = mfma_block<DT, KSTEPS, LROW>(tile[tn & 1], ((b + 1) % BPT) * 32, bfrag);
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

template <int DT, int DPT, int MODE>
static void topk_dispatch_g(const TopkArgs& a, hipStream_t s)
{
    dim3 grid((unsigned)((a.m + TK_WAVES * 32 - 1) / (TK_WAVES * 32)), (unsigned)a.nseg);
    if constexpr (MODE == TK_SEED) {
        hipLaunchKernelGGL((k_topk<DT, DPT, 1, TK_SEED>), grid, dim3(256), 0, s, a);
    } else {
        const int gpl = a.G / 64;
        if (gpl == 2) hipLaunchKernelGGL((k_topk<DT, DPT, 2, TK_MAIN>), grid, dim3(256), 0, s, a);
        else if (gpl == 4) hipLaunchKernelGGL((k_topk<DT, DPT, 4, TK_MAIN>), grid, dim3(256), 0, s, a);
        else if (gpl == 8) hipLaunchKernelGGL((k_topk<DT, DPT, 8, TK_MAIN>), grid, dim3(256), 0, s, a);
        else if (gpl == 16) hipLaunchKernelGGL((k_topk<DT, DPT, 16, TK_MAIN>), grid, dim3(256), 0, s, a);
        else fail(RKMIPS_EINVAL, "internal: unsupported candidate buffer size");
    }
}

int topk_users_per_block(int, int) { return TK_WAVES * 32; }

// Workgroups of the main pass that one compute unit holds at once (registers and LDS).
template <int DT, int DPT>
static int resident_g(int G)
{
    int nb = 0;
    hipError_t e = hipSuccess;
    const int gpl = G / 64;
    if (gpl == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_topk<DT, DPT, 2, TK_MAIN>, 256, 0);
    else if (gpl == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_topk<DT, DPT, 4, TK_MAIN>, 256, 0);
    else if (gpl == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_topk<DT, DPT, 8, TK_MAIN>, 256, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_topk<DT, DPT, 16, TK_MAIN>, 256, 0);
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
    else if (dtype == DT_SPLIT) topk_dispatch<DT_SPLIT, TK_SEED>(a, s);
    else fail(RKMIPS_EINVAL, "internal: no matrix-core path for this operand type");
    HIPC(hipGetLastError());
}

}  // namespace rk
