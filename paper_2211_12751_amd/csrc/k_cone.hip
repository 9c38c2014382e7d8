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
__device__ __forceinline__ float row_dot(const uint16_t* a, const uint16_t* b, int ld)
{
    float acc = 0.f;
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
            const uint16_t* up = a.unit + (int64_t)a.perm[p] * a.ld;
            if (phase == 0) {
                const int64_t st = a.seg_start[s], sz = a.seg_start[s + 1] - st;
                const float dv = row_dot(up, a.unit + (int64_t)a.perm[cone_pivot(a, st, sz)] * a.ld, a.ld);
                key = ((unsigned long long)f32_ord(dv) << 32) | (unsigned long long)p;
            } else if (phase == 1) {
                const int64_t pl = (int64_t)(key_min(a.key1, ai) & 0xffffffffull);
                const float dl = row_dot(up, a.unit + (int64_t)a.perm[pl] * a.ld, a.ld);
                a.dot_l[p] = dl;
                key = ((unsigned long long)f32_ord(dl) << 32) | (unsigned long long)p;
            } else {
                const int64_t pr = (int64_t)(key_min(a.key2, ai) & 0xffffffffull);
                const float dr = row_dot(up, a.unit + (int64_t)a.perm[pr] * a.ld, a.ld);
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


// BF16 unit rows (original order) for the split phases.
template <int DT>
__global__ void k_unit(const void* X, const float* scales, const double* n2, int64_t rows, int d, int ld,
                       uint16_t* out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * ld) return;
    const int64_t r = t / ld;
    const int i = (int)(t - r * ld);
    float v = 0.f;
    if (i < d && n2[r] > 0.0) {
        double x = (double)elem_f32<DT>(X, r * d + i);
        if constexpr (DT == DT_FP8) x *= (double)scales[r];
        v = (float)(x / sqrt(n2[r]));
    }
    const uint32_t b = __float_as_uint(v);
    out[t] = (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);   // round to nearest even
}

// Per block (one wave, one user per lane): unit centre (FP64 mean of the unit user
// rows, normalised), per-user cos/sin of the angle theta_u between u and the centre
// (FP64 from the stored values), and cos/sin of a cone angle omega >= max theta_u.
template <int DT>
__global__ __launch_bounds__(256) void k_leaf_stats(LeafArgs a)
{
    __shared__ float cen[4][256];
    const int l = lane_id(), w = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * 4 + w;
    if (b >= a.nblocks) return;
    const int64_t st = a.block_start[b], en = a.block_start[b + 1];
    const int sz = (int)(en - st);
    const bool mine = l < sz;
    const int64_t p = st + l;
    // FP64 unit vector of this lane's user, read from the stored row (leaf order)
    const double un_l = mine ? sqrt(a.user_n2[p]) : 0.0;
    const double inv = un_l > 0.0 ? 1.0 / un_l : 0.0;
    const double sc_l = (DT == DT_FP8 && mine) ? (double)a.user_scales[p] : 1.0;
    double cn2 = 0.0;
    for (int i = 0; i < a.d; i++) {
        double v = mine ? (double)elem_f32<DT>(a.users, p * a.ld + i) * sc_l * inv : 0.0;
        v = wave_sum(v) / (double)sz;
        cn2 += v * v;
        if (l == 0) cen[w][i] = (float)v;
    }
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
        double acc = 0.0;
        for (int i = 0; i < a.d; i++) acc = __fma_rn((double)elem_f32<DT>(a.users, p * a.ld + i), (double)cen[w][i], acc);
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
// block without usable angles, so it is never pruned).  One wave per block, one user
// per lane (blocks hold at most 64 users); lambda rows are in original user order.
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
        if (l == 0) {
            float out = -__builtin_inff();
            if (ok) {
                float f = (float)mn;
                if ((double)f > mn) {   // step one ulp towards -inf
                    const uint32_t u = __float_as_uint(f);
                    f = f == 0.f ? -__uint_as_float(1u) : __uint_as_float(f > 0.f ? u - 1u : u + 1u);
                }
                out = f;
            }
            lb[(int64_t)j * nblocks + b] = out;
        }
    }
}

// ------------------------------------------------------------------ host orchestration
void build_cone(Index& x, const void* users, const float* user_scales, const double* n2_orig, hipStream_t s,
                const std::function<void()>& enqueued, ConeWork& cw, const std::atomic<bool>* cancel)
{
    const int64_t m = x.m;
    const int ld = x.ld;
    DevBuf &unit = cw.unit, &perm_a = cw.perm_a, &perm_b = cw.perm_b, &seg_a = cw.seg_a, &seg_b = cw.seg_b;
    DevBuf &dot_l = cw.dot_l, &left = cw.left, &lrank = cw.lrank, &blk_cnt = cw.blk_cnt;
    unit.alloc(sizeof(uint16_t) * (size_t)m * ld);
    {
        const int64_t tot = m * ld;
        dim3 g((unsigned)((tot + 255) / 256)), b(256);
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_unit<DT_F32>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.u16());
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_unit<DT_BF16>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.u16());
        else hipLaunchKernelGGL(k_unit<DT_FP8>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.u16());
    }
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
        a.unit = unit.u16(); a.ld = ld; a.d = x.d; a.perm = perm_a.u32();
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
    int level = 0;
    bool more = m > x.prm.leaf_size;
    // the first batch is the depth of a perfectly balanced tree plus a margin for uneven
    // splits (levels without an active segment cost one early exit per kernel), so the
    // host usually checks once; later batches are short
    int batch = 1;
    while (((int64_t)x.prm.leaf_size << batch) < m) batch++;
    batch += 3;
    int64_t nseg_final = 1;
    bool hooked = false;
    while (more) {
        for (int rep = 0; rep < batch; rep++, level++) {
            const ConeLevelArgs a = level_args(level);
            for (int ph = 0; ph < 3; ph++) hipLaunchKernelGGL(k_cone_phase, dim3(grid), dim3(256), 0, s, a, ph);
            hipLaunchKernelGGL(k_cone_next, dim3(1), dim3(CN_THREADS), 0, s, a);
            hipLaunchKernelGGL(k_cone_scatter, dim3(grid), dim3(256), 0, s, a, perm_b.u32());
            HIPC(hipGetLastError());
            perm_a.swap(perm_b);
            seg_a.swap(seg_b);
        }
        HIPC(hipMemcpyAsync(h_ctl.p, d_ctl.p, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s));
        HIPC(hipEventRecord(ev_ctl, s));
        if (!hooked) {
            hooked = true;
            if (enqueued) enqueued();
        }
        host_wait(ev_ctl);
        if (cancel && cancel->load()) return;
        more = ((const int64_t*)h_ctl.p)[2] > 0;
        nseg_final = ((const int64_t*)h_ctl.p)[level & 1];
        batch = 2;
    }
    if (!hooked && enqueued) enqueued();
    if (level == 0) {   // the caller reads host copies made before the build
        HIPC(hipEventRecord(ev_ctl, s));
        host_wait(ev_ctl);
    }

    // ---- leaves are the blocks; users move into leaf order
    x.nblocks = nseg_final;
    x.block_start.alloc(sizeof(int64_t) * (nseg_final + 1));
    HIPC(hipMemcpyAsync(x.block_start.p, d_start[level & 1].p, sizeof(int64_t) * (nseg_final + 1),
                        hipMemcpyDeviceToDevice, s));
    x.user_perm.swap(perm_a);
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
}

void finish_blocks(Index& x, hipStream_t s)
{
    const int64_t tot = x.nblocks * x.prm.k_max;
    x.block_lb.alloc(sizeof(float) * tot);
    hipLaunchKernelGGL(k_block_lb, dim3((unsigned)((x.nblocks + 3) / 4)), dim3(256), 0, s, x.lam64.d(),
                       x.user_perm.u32(), x.user_n2.d(), x.block_start.i64(), x.block_ok.i(), x.nblocks, x.m, x.prm.k_max,
                       x.block_lb.f());
    HIPC(hipGetLastError());
}

}  // namespace rk
