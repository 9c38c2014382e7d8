// Cone-Tree blocking of the users (Alg. 3), built level-synchronously on the GPU, and
// the per-block / per-user quantities of the node-level (Lemma 2) and vector-level
// (Lemma 3) upper bounds, plus the block lower bounds L^j(B) of Alg. 4.
//
// All splits of one tree level run together: every position of the current user
// permutation knows its segment (node); per node the random point v (a counter-based
// draw), u_l = argmin <u, v> and u_r = argmin <u, u_l> are found with 64-bit atomicMin
// on (orderable dot, position) keys -- ties take the lowest position -- and the node is
// split stably by cos(u, u_l) >= cos(u, u_r) (ties go left).  A split that leaves one
// side empty splits the node in index halves.  Nodes of at most N0 users are leaves.
// Users are unit-normalised first (Fact 2: the norm of u does not change its MIPS
// result), so inner products are cosines.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "index.h"
#include "internal.h"
#include "query.h"

namespace rk {

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

// Segment s of the current level is split (active) when it holds more than N0 users;
// its random point v is the user at a counter-based draw inside the segment.
__device__ __forceinline__ int64_t cone_pivot(const ConeLevelArgs& a, int64_t st, int64_t sz)
{
    const uint64_t r = splitmix64(a.seed ^ splitmix64(((uint64_t)a.level << 40) ^ (uint64_t)st));
    return st + (int64_t)(r % (uint64_t)sz);
}

// <a, b> of two BF16 unit rows, one lane per row (16-byte loads of 8 values; the rows of
// a wave are independent, so their loads overlap).  The split geometry only shapes the
// tree (which never changes a result), so BF16 directions suffice and halve the bytes.
// Rows of 256 bytes and more: each step loads one 128-byte line of both rows before it uses
// any of it, so that requests for a line arrive together and the line is fetched once
// (loads spread over the whole loop find it evicted again when many waves gather rows from
// HBM at once).  Shorter rows keep one load pair per step, which needs fewer registers.
__device__ __forceinline__ float row_dot(const uint16_t* a, const uint16_t* b, int ld)
{
    float acc = 0.f;
    if (ld < 128) {
        for (int c = 0; c < ld; c += 8) {
            const i32x4 x = *(const i32x4*)(a + c), y = *(const i32x4*)(b + c);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t xu = (uint32_t)x[e], yu = (uint32_t)y[e];
                acc = fmaf(__uint_as_float(xu << 16), __uint_as_float(yu << 16), acc);
                acc = fmaf(__uint_as_float(xu & 0xffff0000u), __uint_as_float(yu & 0xffff0000u), acc);
            }
        }
        return acc;
    }
    for (int c0 = 0; c0 < ld; c0 += 64) {
        const int nv = ld - c0 < 64 ? (ld - c0) / 8 : 8;   // ld: 32, 64, 128 or 256
        i32x4 x[8], y[8];
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (j < nv) {
                x[j] = *(const i32x4*)(a + c0 + 8 * j);
                y[j] = *(const i32x4*)(b + c0 + 8 * j);
            }
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (j < nv) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t xu = (uint32_t)x[j][e], yu = (uint32_t)y[j][e];
                    acc = fmaf(__uint_as_float(xu << 16), __uint_as_float(yu << 16), acc);
                    acc = fmaf(__uint_as_float(xu & 0xffff0000u), __uint_as_float(yu & 0xffff0000u), acc);
                }
            }
    }
    return acc;
}

typedef float cone_f32x2 __attribute__((ext_vector_type(2)));

// <a, b> of two rows of FP8 codes (ld of 32, 64, 128 or 256 bytes) in FP32: the code
// products are exact, their sum rounds.  One 128-byte line of both rows per step, as above.
__device__ __forceinline__ float row_dot_fp8(const uint8_t* a, const uint8_t* b, int ld)
{
    float acc = 0.f;
    for (int c0 = 0; c0 < ld; c0 += 128) {
        const int nv = ld - c0 < 128 ? (ld - c0) / 16 : 8;
        i32x4 x[8], y[8];
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (j < nv) {
                x[j] = *(const i32x4*)(a + c0 + 16 * j);
                y[j] = *(const i32x4*)(b + c0 + 16 * j);
            }
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (j < nv) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const cone_f32x2 xl = __builtin_amdgcn_cvt_pk_f32_fp8(x[j][e], false);
                    const cone_f32x2 xh = __builtin_amdgcn_cvt_pk_f32_fp8(x[j][e], true);
                    const cone_f32x2 yl = __builtin_amdgcn_cvt_pk_f32_fp8(y[j][e], false);
                    const cone_f32x2 yh = __builtin_amdgcn_cvt_pk_f32_fp8(y[j][e], true);
                    acc = fmaf(xl[0], yl[0], acc);
                    acc = fmaf(xl[1], yl[1], acc);
                    acc = fmaf(xh[0], yh[0], acc);
                    acc = fmaf(xh[1], yh[1], acc);
                }
            }
    }
    return acc;
}

// cos(u_a, u_b) of two users (original indices) from the level's row form
template <bool F8>
__device__ __forceinline__ float cone_dot(const ConeLevelArgs& a, int64_t ua, int64_t ub)
{
    if constexpr (F8) return (a.fac[ua] * a.fac[ub]) * row_dot_fp8(a.codes + ua * a.ld, a.codes + ub * a.ld, a.ld);
    else return row_dot(a.unit + ua * a.ld, a.unit + ub * a.ld, a.ld);
}

// Argmin keys of an active segment are spread over KEY_WAYS slots (chosen by the
// workgroup) so that the waves of a large segment do not all meet on one address;
// readers take the minimum over the slots.
static constexpr int KEY_WAYS = 8;

__device__ __forceinline__ unsigned long long key_min(const unsigned long long* k, int ai)
{
    unsigned long long v = ~0ull;
#pragma unroll
    for (int q = 0; q < KEY_WAYS; q++) {
        const unsigned long long x = k[(int64_t)ai * KEY_WAYS + q];
        v = x < v ? x : v;
    }
    return v;
}

// One lane per position, 256 consecutive positions per workgroup.  Positions of one
// segment are contiguous, so a wave meets few segments: the per-segment reduction runs
// inside the wave and only one atomic per (wave, segment) reaches memory.
// phase 0: argmin <u, v> -> key1;  phase 1: dot_l and argmin <u, u_l> -> key2;
// phase 2: side flags, their ranks inside the workgroup's block of positions and the
// block's count (the left count of a segment is a difference of two global ranks).
template <bool F8>
__global__ __launch_bounds__(256) void k_cone_phase(ConeLevelArgs a, int phase)
{
    if (a.ctl[2] == 0) return;   // no active segment at this level (workgroup-uniform)
    __shared__ int wt[4];
    const int l = lane_id(), w = threadIdx.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = p < a.m;
    int ai = -1;   // active index of the position's segment (-1: leaf)
    unsigned long long key = ~0ull;
    int lf = 0;
    if (in) {
        const int s = a.seg[p];
        ai = a.act[s];
        if (ai >= 0) {
            const int64_t up = a.perm[p];
            if (phase == 0) {
                const int64_t st = a.seg_start[s], sz = a.seg_start[s + 1] - st;
                const float dv = cone_dot<F8>(a, up, a.perm[cone_pivot(a, st, sz)]);
                key = ((unsigned long long)f32_ord(dv) << 32) | (unsigned long long)p;
            } else if (phase == 1) {
                const int64_t pl = (int64_t)(key_min(a.key1, ai) & 0xffffffffull);
                const float dl = cone_dot<F8>(a, up, a.perm[pl]);
                a.dot_l[p] = dl;
                key = ((unsigned long long)f32_ord(dl) << 32) | (unsigned long long)p;
            } else {
                const int64_t pr = (int64_t)(key_min(a.key2, ai) & 0xffffffffull);
                const float dr = cone_dot<F8>(a, up, a.perm[pr]);
                lf = a.dot_l[p] >= dr ? 1 : 0;
            }
        }
    }
    if (phase == 2) {   // uniform over the workgroup
        const uint64_t bl = ballot64(lf != 0);
        if (l == 0) wt[w] = __popcll(bl);
        __syncthreads();
        int off = 0;
        for (int q = 0; q < w; q++) off += wt[q];
        if (in) {
            a.left[p] = lf;
            a.lrank[p] = off + __popcll(bl & ((1ull << l) - 1ull));
        }
        if (threadIdx.x == 0) a.blk_cnt[blockIdx.x] = wt[0] + wt[1] + wt[2] + wt[3];
        return;
    }
    unsigned long long* keys = phase == 0 ? a.key1 : a.key2;
    uint64_t rem = ballot64(ai >= 0);
    while (rem) {
        const int leader = __builtin_ctzll(rem);
        const int a0 = __shfl(ai, leader);
        const bool mine = ai == a0;
        rem &= ~ballot64(mine);
        const unsigned long long mn = wave_min_u64(mine ? key : ~0ull);
        if (l == leader) atomicMin(&keys[(int64_t)a0 * KEY_WAYS + (blockIdx.x & (KEY_WAYS - 1))], mn);
    }
}

// Level 0: one segment [0, m) (active when m > N0), identity permutation, all positions
// in segment 0, fresh argmin slots.
__global__ void k_cone_init(ConeLevelArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.m) {
        a.perm_init[i] = (uint32_t)i;
        a.seg_init[i] = 0;
    }
    if (i < KEY_WAYS) {
        a.key1[i] = ~0ull;
        a.key2[i] = ~0ull;
    }
    if (i == 0) {
        const bool act = a.m > a.leaf;
        a.ctl[0] = 1;
        a.ctl[1] = 0;
        a.ctl[2] = act ? 1 : 0;
        a.ctl[3] = 0;
        a.seg_start_init[0] = 0;
        a.seg_start_init[1] = a.m;
        a.act_init[0] = act ? 0 : -1;
    }
}

// Threads of the single k_cone_next workgroup: four waves, so that it finds room on a
// compute unit beside the matrix-core kernels of the other stream.
static constexpr int CN_THREADS = 256;

// The next level's segments, by one workgroup: an active segment becomes its left and
// right parts (index halves when one side is empty), an inactive one stays.  Also
// numbers the next level's active segments and resets their argmin slots.
__global__ __launch_bounds__(CN_THREADS) void k_cone_next(ConeLevelArgs a)
{
    __shared__ int64_t wtot[CN_THREADS / 64], wact[CN_THREADS / 64];
    __shared__ int64_t carry_s, active_s, total_left;
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    const int64_t nseg = a.ctl[a.ctl_cur];
    // exclusive prefix of the per-block left counts: global left rank of a position =
    // blk_cnt[p >> 8] + lrank[p]
    const int64_t nblk = (a.m + 255) / 256;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nblk; c0 += CN_THREADS) {
        const int64_t i = c0 + tid;
        const int v = i < nblk ? a.blk_cnt[i] : 0;
        const int incl = wave_incl_scan(v);
        if (l == 63) wtot[w] = incl;
        __syncthreads();
        int64_t off = carry_s;
        for (int q = 0; q < w; q++) off += wtot[q];
        if (i < nblk) a.blk_cnt[i] = (int)(off + incl - v);
        __syncthreads();
        if (tid == 0) {
            int64_t t = 0;
            for (int q = 0; q < CN_THREADS / 64; q++) t += wtot[q];
            carry_s += t;
        }
        __syncthreads();
    }
    if (tid == 0) {
        total_left = carry_s;
        carry_s = 0;
        active_s = 0;
    }
    __syncthreads();
    const int64_t tl = total_left;
    auto lrank_at = [&](int64_t x) -> int64_t { return x < a.m ? (int64_t)a.blk_cnt[x >> 8] + a.lrank[x] : tl; };
    for (int64_t c0 = 0; c0 < nseg; c0 += CN_THREADS) {
        const int64_t s = c0 + tid;
        int64_t st = 0, sz = 0, nl = 0;
        int kids = 0, k0 = 0, k1 = 0;
        bool act = false, dg = false;
        if (s < nseg) {
            st = a.seg_start[s];
            sz = a.seg_start[s + 1] - st;
            act = a.act[s] >= 0;
            kids = act ? 2 : 1;
            if (act) {
                nl = lrank_at(st + sz) - lrank_at(st);
                a.nleft[s] = (int)nl;
                dg = nl == 0 || nl == sz;
                if (dg) nl = sz / 2;
                k0 = nl > a.leaf;
                k1 = sz - nl > a.leaf;
            }
            a.degen[s] = dg ? 1 : 0;
        }
        // block-exclusive prefixes of the kids and of the active kids
        const int incl = wave_incl_scan(kids);
        const int iact = wave_incl_scan(k0 + k1);
        if (l == 63) {
            wtot[w] = incl;
            wact[w] = iact;
        }
        __syncthreads();
        int64_t off = carry_s, aoff = active_s;
        for (int q = 0; q < w; q++) {
            off += wtot[q];
            aoff += wact[q];
        }
        off += incl - kids;
        aoff += iact - (k0 + k1);
        if (s < nseg) {
            a.next_start[off] = st;
            a.next_index[s] = (int)off;
            if (act) {
                a.next_start[off + 1] = st + nl;
                a.next_act[off] = k0 ? (int)aoff : -1;
                a.next_act[off + 1] = k1 ? (int)(aoff + k0) : -1;
            } else {
                a.next_act[off] = -1;
            }
        }
        __syncthreads();
        if (tid == 0) {
            int64_t t = 0, ta = 0;
            for (int q = 0; q < CN_THREADS / 64; q++) {
                t += wtot[q];
                ta += wact[q];
            }
            carry_s += t;
            active_s += ta;
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.next_start[carry_s] = a.m;
        a.ctl[1 - a.ctl_cur] = carry_s;
        a.ctl[2] = active_s;
    }
    // the next level's argmin slots start from their identity
    for (int64_t i = tid; i < active_s * KEY_WAYS; i += CN_THREADS) {
        a.next_key1[i] = ~0ull;
        a.next_key2[i] = ~0ull;
    }
}

// Stable split of every active segment (left side first) and the next level's segment
// of every position.  The left rank of a position inside its segment is the difference
// of two global left ranks (block prefix + rank inside the block).
__global__ void k_cone_scatter(ConeLevelArgs a, uint32_t* new_perm)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.m) return;
    const int s = a.seg[p];
    const int64_t st = a.seg_start[s], sz = a.seg_start[s + 1] - st;
    int64_t np = p;
    int ns = a.next_index[s];
    if (sz > a.leaf) {
        if (!a.degen[s]) {
            const int64_t lb = ((int64_t)a.blk_cnt[p >> 8] + a.lrank[p]) - ((int64_t)a.blk_cnt[st >> 8] + a.lrank[st]);
            if (a.left[p]) {
                np = st + lb;
            } else {
                np = st + a.nleft[s] + (p - st - lb);
                ns += 1;
            }
        } else if (p - st >= sz / 2) {
            ns += 1;   // index halves
        }
    }
    new_perm[np] = a.perm[p];
    a.next_seg[np] = ns;
}


// ------------------------------------------------------------------ local completion
// Below a few hundred users per segment, a grid-wide level costs more in launches and
// barriers than in work: one workgroup per segment of the current level then completes
// its subtree on its own, depth first, with the same split rule (random point drawn from
// (seed, level, segment start), u_l = argmin <u, v>, u_r = argmin <u, u_l>, stable split
// by cos(u, u_l) >= cos(u, u_r), index halves when one side is empty).  Leaf starts are
// flagged per position (is_start); the block table is assembled from the flags.
static constexpr int CL_STACK = 64;
static constexpr int CL_TARGET = 512;   // users per segment where the local completion takes over

__device__ __forceinline__ unsigned long long wg_min_u64(unsigned long long v, unsigned long long* red)
{
    v = wave_min_u64(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    unsigned long long r = red[0];
    for (int i = 1; i < 4; i++) r = red[i] < r ? red[i] : r;
    __syncthreads();
    return r;
}

template <bool F8>
__global__ __launch_bounds__(256) void k_cone_local(ConeLevelArgs a, uint32_t* tmp_perm, int* is_start)
{
    __shared__ int64_t stk_st[CL_STACK];
    __shared__ int stk_sz[CL_STACK], stk_lv[CL_STACK];
    __shared__ int top_s;
    __shared__ unsigned long long red[4];
    __shared__ int wcnt[4];
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    const int64_t nseg = a.ctl[a.ctl_cur];
    if ((int64_t)blockIdx.x >= nseg) return;   // the grid is an upper bound (workgroup-uniform)
    if (tid == 0) {
        const int64_t st0 = a.seg_start[blockIdx.x];
        stk_st[0] = st0;
        stk_sz[0] = (int)(a.seg_start[blockIdx.x + 1] - st0);
        stk_lv[0] = a.level;
        top_s = 1;
    }
    __syncthreads();
    uint32_t* perm = (uint32_t*)a.perm;   // this workgroup owns its segment's positions
    for (;;) {
        const int t = top_s;
        if (t == 0) break;
        const int64_t st = stk_st[t - 1];
        const int sz = stk_sz[t - 1], lv = stk_lv[t - 1];
        __syncthreads();
        if (tid == 0) top_s = t - 1;
        if (sz <= a.leaf) {
            if (tid == 0) is_start[st] = 1;
            __syncthreads();
            continue;
        }
        // random point v, u_l, u_r
        const uint64_t rr = splitmix64(a.seed ^ splitmix64(((uint64_t)lv << 40) ^ (uint64_t)st));
        const int64_t pv = st + (int64_t)(rr % (uint64_t)sz);
        const int64_t vrow = perm[pv];
        unsigned long long k = ~0ull;
        for (int i = tid; i < sz; i += 256) {
            const int64_t p = st + i;
            const float dv = cone_dot<F8>(a, perm[p], vrow);
            const unsigned long long key = ((unsigned long long)f32_ord(dv) << 32) | (unsigned long long)p;
            k = key < k ? key : k;
        }
        const int64_t pl = (int64_t)(wg_min_u64(k, red) & 0xffffffffull);
        const int64_t lrow = perm[pl];
        k = ~0ull;
        for (int i = tid; i < sz; i += 256) {
            const int64_t p = st + i;
            const float dl = cone_dot<F8>(a, perm[p], lrow);
            a.dot_l[p] = dl;
            const unsigned long long key = ((unsigned long long)f32_ord(dl) << 32) | (unsigned long long)p;
            k = key < k ? key : k;
        }
        const int64_t pr = (int64_t)(wg_min_u64(k, red) & 0xffffffffull);
        const int64_t rrow = perm[pr];
        int nl_mine = 0;
        for (int i = tid; i < sz; i += 256) {
            const int64_t p = st + i;
            const float dr = cone_dot<F8>(a, perm[p], rrow);
            const int lf = a.dot_l[p] >= dr ? 1 : 0;
            a.left[p] = lf;
            nl_mine += lf;
        }
        nl_mine = wave_sum(nl_mine);
        if (l == 0) wcnt[w] = nl_mine;
        __syncthreads();
        int nl = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        const bool dg = nl == 0 || nl == sz;
        if (dg) {
            nl = sz / 2;   // index halves: the order stays
        } else {
            // stable partition, chunk by chunk in position order: lefts first
            int lb = 0, rb = 0;   // lefts / rights placed by earlier chunks
            for (int c0 = 0; c0 < sz; c0 += 256) {
                __syncthreads();   // wcnt reuse
                const int i = c0 + tid;
                const bool in = i < sz;
                const int lf = in ? a.left[st + i] : 0;
                const uint64_t bl = ballot64(in && lf), br = ballot64(in && !lf);
                if (l == 0) wcnt[w] = __popcll(bl);
                __syncthreads();
                int wl = 0;
                for (int q = 0; q < w; q++) wl += wcnt[q];
                const int cl = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
                const int clen = sz - c0 < 256 ? sz - c0 : 256;
                if (in) {
                    const int rl = __popcll(bl & lanemask_lt());
                    const int rw = (w * 64 - wl) + __popcll(br & lanemask_lt());   // rights before, inside the chunk
                    const int np = lf ? lb + wl + rl : nl + rb + rw;
                    tmp_perm[st + np] = perm[st + i];
                }
                lb += cl;
                rb += clen - cl;
            }
            __syncthreads();
            for (int i = tid; i < sz; i += 256) perm[st + i] = tmp_perm[st + i];
        }
        __syncthreads();
        if (tid == 0) {
            // the larger part first, so that the smaller one is split next (stack depth
            // stays below log2 of the segment size)
            const int64_t s0 = st, s1 = st + nl;
            const int z0 = nl, z1 = sz - nl;
            const int tt = top_s;
            if (tt + 2 > CL_STACK) {
                // unreachable (the smaller part is split first, so the stack holds fewer
                // than log2(size) + 2 entries); kept in bounds regardless
                is_start[s0] = 1;
                is_start[s1] = 1;
            } else if (z0 >= z1) {
                stk_st[tt] = s0; stk_sz[tt] = z0; stk_lv[tt] = lv + 1;
                stk_st[tt + 1] = s1; stk_sz[tt + 1] = z1; stk_lv[tt + 1] = lv + 1;
            } else {
                stk_st[tt] = s1; stk_sz[tt] = z1; stk_lv[tt] = lv + 1;
                stk_st[tt + 1] = s0; stk_sz[tt + 1] = z0; stk_lv[tt + 1] = lv + 1;
            }
            if (tt + 2 <= CL_STACK) top_s = tt + 2;
        }
        __syncthreads();
    }
}

// Block table from the leaf-start flags: counts per 1024 positions, one workgroup's scan
// of those counts (nblocks into *nblocks), then the starts in position order and m last.
__global__ __launch_bounds__(256) void k_flag_count(const int* is_start, int64_t m, int* bcnt)
{
    __shared__ int wc[4];
    const int64_t b = blockIdx.x;
    int c = 0;
    for (int i = threadIdx.x; i < 1024; i += 256) {
        const int64_t p = b * 1024 + i;
        if (p < m) c += is_start[p];
    }
    c = wave_sum(c);
    if (lane_id() == 0) wc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bcnt[b] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(1024) void k_flag_scan(int* bcnt, int64_t nb, int64_t* nblocks)
{
    __shared__ int64_t wtot[16];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t i = c0 + tid;
        const int v = i < nb ? bcnt[i] : 0;
        const int incl = wave_incl_scan(v);
        if (l == 63) wtot[w] = incl;
        __syncthreads();
        int64_t off = carry_s;
        for (int q = 0; q < w; q++) off += wtot[q];
        if (i < nb) bcnt[i] = (int)(off + incl - v);
        __syncthreads();
        if (tid == 0) {
            int64_t t = 0;
            for (int q = 0; q < 16; q++) t += wtot[q];
            carry_s += t;
        }
        __syncthreads();
    }
    if (tid == 0) *nblocks = carry_s;
}

__global__ __launch_bounds__(256) void k_flag_emit(const int* is_start, int64_t m, const int* boff,
                                                   const int64_t* nblocks, int64_t* block_start)
{
    __shared__ int wc[4];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    int64_t base = boff[b];
    for (int c0 = 0; c0 < 1024; c0 += 256) {
        const int64_t p = b * 1024 + c0 + tid;
        const bool f = p < m && is_start[p];
        const uint64_t bal = ballot64(f);
        if (l == 0) wc[w] = __popcll(bal);
        __syncthreads();
        int off = 0;
        for (int q = 0; q < w; q++) off += wc[q];
        if (f) block_start[base + off + __popcll(bal & lanemask_lt())] = p;
        base += wc[0] + wc[1] + wc[2] + wc[3];
        __syncthreads();
    }
    if (b == 0 && tid == 0) block_start[*nblocks] = m;
}

// BF16 unit rows (original order) for the split phases: eight values of one row per
// thread (ld is a power of two, at least 32), one 16-byte store.
template <int DT>
__global__ void k_unit(const void* X, const float* scales, const double* n2, int64_t rows, int d, int ld,
                       uint16_t* out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sh = __builtin_ctz((unsigned)ld >> 3);   // log2 of the 8-value groups per row
    if (t >= (rows * ld) >> 3) return;
    const int64_t r = t >> sh;
    const int i0 = (int)(t - (r << sh)) * 8;
    const double nn = n2[r];
    const double un = nn > 0.0 ? sqrt(nn) : 1.0;
    const double sc = DT == DT_FP8 ? (double)scales[r] : 1.0;
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int i = i0 + e;
        float v = 0.f;
        if (i < d && nn > 0.0) {
            double x = (double)elem_f32<DT>(X, r * d + i);
            if constexpr (DT == DT_FP8) x *= sc;
            v = (float)(x / un);
        }
        const uint32_t b = __float_as_uint(v);
        const uint32_t h = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;   // round to nearest even
        if (e & 1) o[e >> 1] |= h << 16;
        else o[e >> 1] = h;
    }
    *(i32x4*)(out + t * 8) = i32x4{(int)o[0], (int)o[1], (int)o[2], (int)o[3]};
}

// scale / ||u|| per user (0 for a zero user), the factor of its FP8 code row
__global__ void k_unit_fac(const float* scales, const double* n2, int64_t rows, float* fac)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const double nn = n2[r];
    fac[r] = nn > 0.0 ? (float)((double)scales[r] / sqrt(nn)) : 0.f;
}

// Per block (one wave, one user per lane): unit centre (FP64 mean of the unit user
// rows, normalised), per-user cos/sin of the angle theta_u between u and the centre
// (FP64 from the stored values), and cos/sin of a cone angle omega >= max theta_u.
template <int DT>
__global__ __launch_bounds__(256) void k_leaf_stats(LeafArgs a)
{
    __shared__ float cen[4][256];
    __shared__ double fac[4][64];
    const int l = lane_id(), w = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * 4 + w;
    if (b >= a.nblocks) return;
    const int64_t st = a.block_start[b], en = a.block_start[b + 1];
    const int sz = (int)(en - st);
    const bool mine = l < sz;
    const int64_t p = st + l;
    // FP64 unit vector of each user, from the stored row (leaf order): the block's rows are
    // contiguous, so lane l sums dimensions l, l + 64, ... over the users in order (64
    // consecutive elements per load), each user's factors taken from LDS
    const double un_l = mine ? sqrt(a.user_n2[p]) : 0.0;
    const double inv = un_l > 0.0 ? 1.0 / un_l : 0.0;
    fac[w][l] = inv;
    __builtin_amdgcn_wave_barrier();
    double cs[4] = {0.0, 0.0, 0.0, 0.0};   // dimensions l + 64 c (d <= 256)
    for (int q = 0; q < sz; q++) {
        const double iq = fac[w][q];
        const double sq = DT == DT_FP8 ? (double)a.user_scales[st + q] : 1.0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int i = l + 64 * c;
            if (i < a.d) cs[c] += (double)elem_f32<DT>(a.users, (st + q) * a.ld + i) * sq * iq;
        }
    }
    double cn2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int i = l + 64 * c;
        if (i < a.d) {
            const double v = cs[c] / (double)sz;
            cn2 += v * v;
            cen[w][i] = (float)v;
        }
    }
    cn2 = wave_sum(cn2);
    __builtin_amdgcn_wave_barrier();
    const double cnorm = sqrt(cn2);
    bool ok = cnorm > 1e-6;
    for (int i = l; i < a.ld; i += 64) {
        const float c = (i < a.d && ok) ? (float)((double)cen[w][i] / cnorm) : 0.f;
        cen[w][i] = c;
        a.center[b * a.ld + i] = c;
    }
    __builtin_amdgcn_wave_barrier();
    double ct = 1.0;
    bool zero_user = false;
    if (mine) {
        const double un2 = a.user_n2[p];
        zero_user = !(un2 > 0.0);
        const float su = DT == DT_FP8 ? a.user_scales[p] : 1.f;
        // the lane's row in 16-byte loads (rows are 16-byte aligned), the terms in index order
        constexpr int VPL = 16 / Elt<DT>::bytes;
        const uint8_t* row = (const uint8_t*)a.users + p * a.ld * Elt<DT>::bytes;
        double acc = 0.0;
        for (int i0 = 0; i0 < a.d; i0 += VPL) {
            const i32x4 q = *(const i32x4*)(row + i0 * Elt<DT>::bytes);
#pragma unroll
            for (int e = 0; e < VPL; e++)
                if (i0 + e < a.d) acc = __fma_rn((double)elem_f32<DT>(&q, e), (double)cen[w][i0 + e], acc);
        }
        if constexpr (DT == DT_FP8) acc *= (double)su;
        const double un = sqrt(un2);
        ct = zero_user ? 1.0 : acc / un;
        ct = ct > 1.0 ? 1.0 : (ct < -1.0 ? -1.0 : ct);
        a.unorm[p] = (float)un;
        a.cos_t[p] = (float)ct;
        a.sin_t[p] = (float)sqrt(fmax(0.0, 1.0 - ct * ct));
        a.user_block[p] = (int)b;
    }
    ok = ok && !(ballot64(zero_user));
    double cw = wave_min(mine ? ct : 2.0);
    // widen the cone a little so rounding of the stored pairs cannot make it too narrow
    cw = cw - 1e-6;
    if (cw < -1.0) cw = -1.0;
    if (l == 0) {
        a.cos_w[b] = ok ? (float)cw : -1.f;
        a.sin_w[b] = ok ? (float)sqrt(fmax(0.0, 1.0 - cw * cw)) : 0.f;
        a.block_ok[b] = ok ? 1 : 0;
    }
}

// L^j(B) = min over the block of lambda_u^(j) / ||u||, rounded down to FP32 (-inf for a
// block without usable angles, so it is never pruned).
__device__ __forceinline__ float block_lb_round(double mn, bool ok)
{
    if (!ok) return -__builtin_inff();
    float f = (float)mn;
    if ((double)f > mn) {   // step one ulp towards -inf
        const uint32_t u = __float_as_uint(f);
        f = f == 0.f ? -__uint_as_float(1u) : __uint_as_float(f > 0.f ? u - 1u : u + 1u);
    }
    return f;
}

// From the lambda rows in original user order: one wave per block, one user per lane
// (blocks hold at most 64 users), gathering each lambda_u^(j) from row j.
__global__ __launch_bounds__(256) void k_block_lb(const double* lam64, const uint32_t* perm, const double* user_n2,
                                                  const int64_t* block_start, const int* block_ok, int64_t nblocks,
                                                  int64_t m, int k_max, float* lb)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nblocks) return;
    const int l = lane_id();
    const int64_t st = block_start[b], en = block_start[b + 1];
    const bool ok = block_ok[b] != 0;
    const double un0 = st + l < en ? sqrt(user_n2[st + l]) : 1.0;
    const int64_t o0 = st + l < en ? (int64_t)perm[st + l] : 0;
    for (int j = 0; j < k_max; j++) {
        double mn = __builtin_inf();
        for (int64_t q = st + l; q < en; q += 64) {
            const double v = q == st + l ? lam64[(int64_t)j * m + o0] / un0
                                         : lam64[(int64_t)j * m + perm[q]] / sqrt(user_n2[q]);
            mn = v < mn ? v : mn;
        }
        mn = wave_min(mn);
        if (l == 0) lb[(int64_t)j * nblocks + b] = block_lb_round(mn, ok);
    }
}

// From rows[q x k_max + j] = lambda^(j+1) / ||u|| of the user at leaf position q (written
// by the lambda refine): a block's rows are contiguous, so one wave per block reads them
// in order, lane j keeping the minimum of column j.  The quotients are the ones the
// gathering form computes (same operands, same operations), so the bounds are the same.
__global__ __launch_bounds__(256) void k_block_lb_rows(const double* rows, const int64_t* block_start,
                                                       const int* block_ok, int64_t nblocks, int k_max, float* lb)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nblocks) return;
    const int l = lane_id();
    const int64_t st = block_start[b], en = block_start[b + 1];
    const bool ok = block_ok[b] != 0;
    for (int j = l; j < k_max; j += 64) {
        double mn = __builtin_inf();
        const double* r = rows + st * k_max + j;
#pragma unroll 8
        for (int64_t q = st; q < en; q++, r += k_max) {
            const double v = *r;
            mn = v < mn ? v : mn;
        }
        lb[(int64_t)j * nblocks + b] = block_lb_round(mn, ok);
    }
}

// ------------------------------------------------------------------ host orchestration
void build_cone(Index& x, const void* users, const float* user_scales, const double* n2_orig, hipStream_t s,
                const std::function<void()>& enqueued, ConeWork& cw, const std::atomic<bool>* cancel,
                const uint8_t* codes_padded)
{
    const int64_t m = x.m;
    const int ld = x.ld;
    DevBuf &unit = cw.unit, &perm_a = cw.perm_a, &perm_b = cw.perm_b, &seg_a = cw.seg_a, &seg_b = cw.seg_b;
    DevBuf &dot_l = cw.dot_l, &left = cw.left, &lrank = cw.lrank, &blk_cnt = cw.blk_cnt;
    // FP8 users with their padded code rows at hand: the split products run on the codes
    // (half the bytes of BF16 unit rows), each row's factor scale / ||u|| applied after
    const bool f8 = x.dtype == DT_FP8 && codes_padded;
    if (f8) {
        unit.alloc(sizeof(float) * (size_t)m);
        hipLaunchKernelGGL(k_unit_fac, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, user_scales, n2_orig, m,
                           unit.f());
    } else {
        unit.alloc(sizeof(uint16_t) * (size_t)m * ld);
        const int64_t tot = m * ld / 8;
        dim3 g((unsigned)((tot + 255) / 256)), b(256);
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_unit<DT_F32>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.u16());
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_unit<DT_BF16>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.u16());
        else hipLaunchKernelGGL(k_unit<DT_FP8>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.u16());
    }
    HIPC(hipGetLastError());
    perm_a.alloc(sizeof(uint32_t) * m);
    perm_b.alloc(sizeof(uint32_t) * m);
    dot_l.alloc(sizeof(float) * m);
    left.alloc(sizeof(int) * m);
    lrank.alloc(sizeof(int) * m);
    blk_cnt.alloc(sizeof(int) * ((m + 255) / 256));
    seg_a.alloc(sizeof(int) * m);
    seg_b.alloc(sizeof(int) * m);

    // Levels run on the device, several per check of the host: each level's segment
    // table is built by k_cone_next from the previous one; a level without active
    // segments changes nothing, so levels past the last split are harmless.
    const int64_t cap = m + 2;
    const int64_t act_cap = m / ((int64_t)x.prm.leaf_size + 1) + 1;   // active segments hold > N0 users
    DevBuf(&d_start)[2] = cw.d_start;
    DevBuf(&d_act)[2] = cw.d_act;
    DevBuf(&d_key1)[2] = cw.d_key1;
    DevBuf(&d_key2)[2] = cw.d_key2;
    DevBuf &d_ctl = cw.d_ctl, &d_nleft = cw.d_nleft, &d_degen = cw.d_degen, &d_next_index = cw.d_next_index;
    for (int i = 0; i < 2; i++) {
        d_start[i].alloc(sizeof(int64_t) * (cap + 1));
        d_act[i].alloc(sizeof(int) * cap);
        d_key1[i].alloc(sizeof(uint64_t) * act_cap * KEY_WAYS);
        d_key2[i].alloc(sizeof(uint64_t) * act_cap * KEY_WAYS);
    }
    d_ctl.alloc(sizeof(int64_t) * 4);
    d_nleft.alloc(sizeof(int) * cap);
    d_degen.alloc(sizeof(int) * cap);
    d_next_index.alloc(sizeof(int) * cap);
    PinBuf& h_ctl = cw.h_ctl;
    h_ctl.alloc(sizeof(int64_t) * 4);
    hipEvent_t ev_ctl = nullptr;
    HIPC(hipEventCreateWithFlags(&ev_ctl, hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t e;
        ~EvGuard() { (void)hipEventDestroy(e); }
    } ev_guard{ev_ctl};
    auto level_args = [&](int level) {
        const int c = level & 1, n = c ^ 1;
        ConeLevelArgs a{};
        if (f8) {
            a.codes = codes_padded;
            a.fac = unit.f();
        } else {
            a.unit = unit.u16();
        }
        a.ld = ld; a.d = x.d; a.perm = perm_a.u32();
        a.seg_start = d_start[c].i64(); a.next_start = d_start[n].i64();
        a.ctl = d_ctl.i64(); a.ctl_cur = c; a.level = level; a.leaf = x.prm.leaf_size;
        a.seed = x.prm.seed; a.m = m;
        a.act = d_act[c].i(); a.next_act = d_act[n].i();
        a.key1 = (unsigned long long*)d_key1[c].p; a.key2 = (unsigned long long*)d_key2[c].p;
        a.next_key1 = (unsigned long long*)d_key1[n].p; a.next_key2 = (unsigned long long*)d_key2[n].p;
        a.dot_l = dot_l.f(); a.left = left.i(); a.nleft = d_nleft.i(); a.degen = d_degen.i();
        a.seg = seg_a.i(); a.next_seg = seg_b.i(); a.next_index = d_next_index.i();
        a.lrank = lrank.i(); a.blk_cnt = blk_cnt.i();
        return a;
    };
    const unsigned grid = (unsigned)((m + 255) / 256);
    {
        ConeLevelArgs a = level_args(0);
        a.perm_init = perm_a.u32(); a.seg_init = seg_a.i(); a.seg_start_init = d_start[0].i64();
        a.act_init = d_act[0].i();
        hipLaunchKernelGGL(k_cone_init, dim3(grid), dim3(256), 0, s, a);
        HIPC(hipGetLastError());
    }
    // Grid-wide levels until segments average about CL_TARGET users (one launch per phase
    // and level: the work of a level is a pass over all users), then one workgroup per
    // segment completes the tree locally.
    int L0 = 0;
    while ((m >> L0) > CL_TARGET) L0++;
    for (int level = 0; level < L0; level++) {
        const ConeLevelArgs a = level_args(level);
        for (int ph = 0; ph < 3; ph++) {
            if (f8) hipLaunchKernelGGL(k_cone_phase<true>, dim3(grid), dim3(256), 0, s, a, ph);
            else hipLaunchKernelGGL(k_cone_phase<false>, dim3(grid), dim3(256), 0, s, a, ph);
        }
        hipLaunchKernelGGL(k_cone_next, dim3(1), dim3(CN_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_cone_scatter, dim3(grid), dim3(256), 0, s, a, perm_b.u32());
        HIPC(hipGetLastError());
        perm_a.swap(perm_b);
        seg_a.swap(seg_b);
    }
    // local completion; the leaf-start flags reuse the level ranks, the block counts the
    // level block counts, and ctl[3] receives the block count
    int* is_start = lrank.i();
    HIPC(hipMemsetAsync(is_start, 0, sizeof(int) * (size_t)m, s));
    {
        const ConeLevelArgs a = level_args(L0);
        const unsigned lgrid = (unsigned)std::min<int64_t>((int64_t)1 << L0, m);
        if (f8) hipLaunchKernelGGL(k_cone_local<true>, dim3(lgrid), dim3(256), 0, s, a, perm_b.u32(), is_start);
        else hipLaunchKernelGGL(k_cone_local<false>, dim3(lgrid), dim3(256), 0, s, a, perm_b.u32(), is_start);
        HIPC(hipGetLastError());
    }
    x.block_start.alloc(sizeof(int64_t) * (size_t)(m + 1));
    {
        const int64_t nb = (m + 1023) / 1024;
        int64_t* nblocks_dev = d_ctl.i64() + 3;
        hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nb), dim3(256), 0, s, (const int*)is_start, m, blk_cnt.i());
        hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, s, blk_cnt.i(), nb, nblocks_dev);
        hipLaunchKernelGGL(k_flag_emit, dim3((unsigned)nb), dim3(256), 0, s, (const int*)is_start, m,
                           (const int*)blk_cnt.i(), (const int64_t*)nblocks_dev, x.block_start.i64());
        HIPC(hipGetLastError());
    }
    HIPC(hipMemcpyAsync(h_ctl.p, d_ctl.p, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s));
    HIPC(hipEventRecord(ev_ctl, s));
    if (enqueued) enqueued();
    host_wait(ev_ctl);
    if (cancel && cancel->load()) return;
    const int64_t nseg_final = ((const int64_t*)h_ctl.p)[3];

    // ---- leaves are the blocks; users move into leaf order
    x.nblocks = nseg_final;
    x.user_perm.swap(perm_a);
    make_user_inverse(x, s);
    const int eb = elt_bytes(x.dtype);
    x.users.alloc((size_t)m * ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) x.user_scales.alloc(sizeof(float) * m);
    launch_gather_rows(x.dtype, users, x.d, user_scales, x.user_perm.u32(), m, x.d, x.users.p, ld,
                       x.user_scales.f(), s);
    if (x.mma_dtype != x.dtype) {   // matrix-core rows for the query-side inner-product test
        x.users_mma.alloc(sizeof(uint16_t) * (size_t)m * x.mma_ld);
        launch_mma_operand(x.mma_dtype, x.dtype, x.users.p, m, x.ld, x.users_mma.u16(), 1, s);
    }
    x.user_n2.alloc(sizeof(double) * m);
    launch_permute_f64(n2_orig, x.user_perm.u32(), m, x.user_n2.d(), s);

    x.center.alloc(sizeof(float) * (size_t)x.nblocks * ld);
    x.cos_w.alloc(sizeof(float) * x.nblocks);
    x.sin_w.alloc(sizeof(float) * x.nblocks);
    x.block_ok.alloc(sizeof(int) * x.nblocks);
    x.unorm.alloc(sizeof(float) * m);
    x.cos_t.alloc(sizeof(float) * m);
    x.sin_t.alloc(sizeof(float) * m);
    x.user_block.alloc(sizeof(int) * m);
    LeafArgs la{};
    la.dtype = x.dtype; la.users = x.users.p; la.user_scales = x.user_scales.f(); la.user_n2 = x.user_n2.d();
    la.perm = x.user_perm.u32(); la.block_start = x.block_start.i64();
    la.nblocks = x.nblocks; la.m = m; la.d = x.d; la.ld = ld; la.k_max = x.prm.k_max;
    la.center = x.center.f(); la.cos_w = x.cos_w.f(); la.sin_w = x.sin_w.f(); la.block_ok = x.block_ok.i();
    la.unorm = x.unorm.f(); la.cos_t = x.cos_t.f(); la.sin_t = x.sin_t.f(); la.user_block = x.user_block.i();
    dim3 g((unsigned)((x.nblocks + 3) / 4)), b(256);
    if (x.dtype == DT_F32) hipLaunchKernelGGL(k_leaf_stats<DT_F32>, g, b, 0, s, la);
    else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_leaf_stats<DT_BF16>, g, b, 0, s, la);
    else hipLaunchKernelGGL(k_leaf_stats<DT_FP8>, g, b, 0, s, la);
    HIPC(hipGetLastError());
    make_center_operand(x, s);
}

__global__ void k_inv_perm(const uint32_t* perm, int64_t m, uint32_t* inv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) inv[perm[i]] = (uint32_t)i;
}

void make_user_inverse(Index& x, hipStream_t s)
{
    x.user_inv.alloc(sizeof(uint32_t) * (size_t)x.m);
    hipLaunchKernelGGL(k_inv_perm, dim3((unsigned)((x.m + 255) / 256)), dim3(256), 0, s, x.user_perm.u32(), x.m,
                       x.user_inv.u32());
    HIPC(hipGetLastError());
}

void make_center_operand(Index& x, hipStream_t s)
{
    if (x.mma_dtype == DT_F32) return;   // the FP32 matrix cores take the FP32 centres
    x.center_mma.alloc(sizeof(uint16_t) * (size_t)x.nblocks * 2 * x.ld);
    launch_split_bf16(x.center.f(), x.nblocks, x.ld, x.center_mma.u16(), 2, s);
}

void finish_blocks(Index& x, hipStream_t s, const double* lb_rows)
{
    const int64_t tot = x.nblocks * x.prm.k_max;
    x.block_lb.alloc(sizeof(float) * tot);
    const dim3 g((unsigned)((x.nblocks + 3) / 4)), b(256);
    if (lb_rows)
        hipLaunchKernelGGL(k_block_lb_rows, g, b, 0, s, lb_rows, x.block_start.i64(), x.block_ok.i(), x.nblocks,
                           x.prm.k_max, x.block_lb.f());
    else
        hipLaunchKernelGGL(k_block_lb, g, b, 0, s, x.lam64.d(), x.user_perm.u32(), x.user_n2.d(), x.block_start.i64(),
                           x.block_ok.i(), x.nblocks, x.m, x.prm.k_max, x.block_lb.f());
    HIPC(hipGetLastError());
}

}  // namespace rk
