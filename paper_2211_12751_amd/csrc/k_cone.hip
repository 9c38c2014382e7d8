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

__device__ __forceinline__ int64_t seg_of(const int64_t* starts, int64_t nseg, int64_t p)
{
    int64_t lo = 0, hi = nseg - 1;   // largest s with starts[s] <= p
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

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

// <a, b> of two unit rows, one lane per row (16-byte loads; the rows of a wave are
// independent, so their loads overlap).
__device__ __forceinline__ float row_dot(const float* a, const float* b, int ld)
{
    float acc = 0.f;
    for (int c = 0; c < ld; c += 4) {
        const f32x4 x = *(const f32x4*)(a + c), y = *(const f32x4*)(b + c);
        acc += x[0] * y[0] + x[1] * y[1] + x[2] * y[2] + x[3] * y[3];
    }
    return acc;
}

// One lane per position, 64 consecutive positions per wave.  Positions of one segment
// are contiguous, so a wave meets few segments: the per-segment reduction runs inside
// the wave and only one atomic per (wave, segment) reaches memory.
// phase 0: argmin <u, v> -> key1;  phase 1: dot_l and argmin <u, u_l> -> key2;
// phase 2: side flags and left counts.
__global__ __launch_bounds__(256) void k_cone_phase(ConeLevelArgs a, int phase)
{
    const int l = lane_id();
    const int64_t nseg = a.ctl[a.ctl_cur];
    const int64_t p = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64 + l;
    const bool in = p < a.m;
    const int64_t s = in ? seg_of(a.seg_start, nseg, p) : -1;
    bool act = false;
    unsigned long long key = ~0ull;
    int lf = 0;
    if (in) {
        const int64_t st = a.seg_start[s], sz = a.seg_start[s + 1] - st;
        act = sz > a.leaf;
        if (act) {
            const float* up = a.unit + (int64_t)a.perm[p] * a.ld;
            if (phase == 0) {
                const float dv = row_dot(up, a.unit + (int64_t)a.perm[cone_pivot(a, st, sz)] * a.ld, a.ld);
                key = ((unsigned long long)f32_ord(dv) << 32) | (unsigned long long)p;
            } else if (phase == 1) {
                const int64_t pl = (int64_t)(a.key1[s] & 0xffffffffull);
                const float dl = row_dot(up, a.unit + (int64_t)a.perm[pl] * a.ld, a.ld);
                a.dot_l[p] = dl;
                key = ((unsigned long long)f32_ord(dl) << 32) | (unsigned long long)p;
            } else {
                const int64_t pr = (int64_t)(a.key2[s] & 0xffffffffull);
                const float dr = row_dot(up, a.unit + (int64_t)a.perm[pr] * a.ld, a.ld);
                lf = a.dot_l[p] >= dr ? 1 : 0;
            }
        }
    }
    if (phase == 2 && in) a.left[p] = lf;
    uint64_t rem = ballot64(act);
    while (rem) {
        const int leader = __builtin_ctzll(rem);
        const int64_t s0 = __shfl(s, leader);
        const bool mine = act && s == s0;
        rem &= ~ballot64(mine);
        if (phase < 2) {
            const unsigned long long mn = wave_min_u64(mine ? key : ~0ull);
            if (l == leader) atomicMin(phase == 0 ? &a.key1[s0] : &a.key2[s0], mn);
        } else {
            const int c = wave_sum(mine ? lf : 0);
            if (l == leader && c) atomicAdd(&a.nleft[s0], c);
        }
    }
}

// Reset of the per-segment reductions of a level.
__global__ void k_cone_init(ConeLevelArgs a)
{
    const int64_t nseg = a.ctl[a.ctl_cur];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += (int64_t)gridDim.x * blockDim.x) {
        a.key1[i] = ~0ull;
        a.key2[i] = ~0ull;
        a.nleft[i] = 0;
    }
}

// The next level's segments, by one workgroup: an active segment becomes its left and
// right parts (index halves when one side is empty), an inactive one stays.  Also
// counts the next level's active segments.
__global__ __launch_bounds__(1024) void k_cone_next(ConeLevelArgs a)
{
    __shared__ int64_t wtot[16];
    __shared__ int64_t carry_s, active_s;
    const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
    const int64_t nseg = a.ctl[a.ctl_cur];
    if (tid == 0) {
        carry_s = 0;
        active_s = 0;
    }
    __syncthreads();
    int64_t nact = 0;
    for (int64_t c0 = 0; c0 < nseg; c0 += 1024) {
        const int64_t s = c0 + tid;
        int64_t st = 0, sz = 0, nl = 0;
        int kids = 0;
        bool act = false, dg = false;
        if (s < nseg) {
            st = a.seg_start[s];
            sz = a.seg_start[s + 1] - st;
            act = sz > a.leaf;
            kids = act ? 2 : 1;
            if (act) {
                nl = a.nleft[s];
                dg = nl == 0 || nl == sz;
                if (dg) nl = sz / 2;
                nact += (nl > a.leaf) + (sz - nl > a.leaf);
            }
            a.degen[s] = dg ? 1 : 0;
        }
        // block-exclusive prefix of kids
        const int incl = wave_incl_scan(kids);
        if (l == 63) wtot[w] = incl;
        __syncthreads();
        int64_t off = carry_s;
        for (int q = 0; q < w; q++) off += wtot[q];
        off += incl - kids;
        if (s < nseg) {
            a.next_start[off] = st;
            if (act) a.next_start[off + 1] = st + nl;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t t = 0;
            for (int q = 0; q < 16; q++) t += wtot[q];
            carry_s += t;
        }
        __syncthreads();
    }
    nact = wave_sum((unsigned long long)nact);
    if (l == 0 && nact) atomicAdd((unsigned long long*)&active_s, (unsigned long long)nact);
    __syncthreads();
    if (tid == 0) {
        a.next_start[carry_s] = a.m;
        a.ctl[1 - a.ctl_cur] = carry_s;
        a.ctl[2] = active_s;
    }
    // the next level's reductions start from their identities
    for (int64_t i = tid; i < carry_s; i += 1024) {
        a.next_key1[i] = ~0ull;
        a.next_key2[i] = ~0ull;
        a.next_nleft[i] = 0;
    }
}

__global__ void k_cone_scatter(ConeLevelArgs a, const int* lscan, uint32_t* new_perm)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.m) return;
    const int64_t nseg = a.ctl[a.ctl_cur];
    const int64_t s = seg_of(a.seg_start, nseg, p);
    int64_t np = p;
    const int64_t st = a.seg_start[s], sz = a.seg_start[s + 1] - st;
    if (sz > a.leaf && !a.degen[s]) {
        const int64_t lb = lscan[p] - lscan[st];
        np = a.left[p] ? st + lb : st + a.nleft[s] + (p - st - lb);
    }
    new_perm[np] = a.perm[p];
}

__global__ void k_iota(uint32_t* v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

template <int DT>
__global__ void k_unit(const void* X, const float* scales, const double* n2, int64_t rows, int d, int ld,
                       float* out)
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
    out[t] = v;
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
    const uint32_t ou = mine ? a.perm[p] : 0u;
    double cn2 = 0.0;
    for (int i = 0; i < a.d; i++) {
        double v = mine ? (double)a.unit[(int64_t)ou * a.ld + i] : 0.0;
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
// block without usable angles, so it is never pruned).
__global__ void k_block_lb(const double* lam64, const double* user_n2, const int64_t* block_start,
                           const int* block_ok, int64_t nblocks, int64_t m, int k_max, float* lb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblocks * k_max) return;
    const int64_t b = t % nblocks;
    const int j = (int)(t / nblocks);
    float out = -__builtin_inff();
    if (block_ok[b]) {
        double mn = __builtin_inf();
        for (int64_t p = block_start[b]; p < block_start[b + 1]; p++) {
            const double v = lam64[(int64_t)j * m + p] / sqrt(user_n2[p]);
            mn = v < mn ? v : mn;
        }
        float f = (float)mn;
        if ((double)f > mn) {   // step one ulp towards -inf
            const uint32_t u = __float_as_uint(f);
            f = f == 0.f ? -__uint_as_float(1u) : __uint_as_float(f > 0.f ? u - 1u : u + 1u);
        }
        out = f;
    }
    lb[(int64_t)j * nblocks + b] = out;
}

// ------------------------------------------------------------------ host orchestration
void build_cone(Index& x, const void* users, const float* user_scales, const double* n2_orig, hipStream_t s)
{
    const int64_t m = x.m;
    const int ld = x.ld;
    DevBuf unit, perm_a, perm_b, dot_l, left, lscan, scan_tmp;
    unit.alloc(sizeof(float) * (size_t)m * ld);
    {
        const int64_t tot = m * ld;
        dim3 g((unsigned)((tot + 255) / 256)), b(256);
        if (x.dtype == DT_F32) hipLaunchKernelGGL(k_unit<DT_F32>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.f());
        else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_unit<DT_BF16>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.f());
        else hipLaunchKernelGGL(k_unit<DT_FP8>, g, b, 0, s, users, user_scales, n2_orig, m, x.d, ld, unit.f());
    }
    perm_a.alloc(sizeof(uint32_t) * m);
    perm_b.alloc(sizeof(uint32_t) * m);
    dot_l.alloc(sizeof(float) * m);
    left.alloc(sizeof(int) * m);
    lscan.alloc(sizeof(int) * m);
    scan_tmp.alloc(sizeof(int) * scan_tmp_elems(m));
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, perm_a.u32(), m);

    // Levels run on the device, four per check of the host: each level's segment table
    // is built by k_cone_next from the previous one; a level without active segments
    // changes nothing, so levels past the last split are harmless.
    const int64_t cap = m + 2;
    DevBuf d_start[2], d_ctl, d_key1[2], d_key2[2], d_nleft[2], d_degen;
    for (int i = 0; i < 2; i++) {
        d_start[i].alloc(sizeof(int64_t) * (cap + 1));
        d_key1[i].alloc(sizeof(uint64_t) * cap);
        d_key2[i].alloc(sizeof(uint64_t) * cap);
        d_nleft[i].alloc(sizeof(int) * cap);
    }
    d_ctl.alloc(sizeof(int64_t) * 4);
    d_degen.alloc(sizeof(int) * cap);
    PinBuf h_ctl;
    h_ctl.alloc(sizeof(int64_t) * 4);
    auto level_args = [&](int level) {
        const int c = level & 1, n = c ^ 1;
        ConeLevelArgs a{};
        a.unit = unit.f(); a.ld = ld; a.d = x.d; a.perm = perm_a.u32();
        a.seg_start = d_start[c].i64(); a.next_start = d_start[n].i64();
        a.ctl = d_ctl.i64(); a.ctl_cur = c; a.level = level; a.leaf = x.prm.leaf_size;
        a.seed = x.prm.seed; a.m = m;
        a.key1 = (unsigned long long*)d_key1[c].p; a.key2 = (unsigned long long*)d_key2[c].p;
        a.nleft = d_nleft[c].i();
        a.next_key1 = (unsigned long long*)d_key1[n].p; a.next_key2 = (unsigned long long*)d_key2[n].p;
        a.next_nleft = d_nleft[n].i();
        a.dot_l = dot_l.f(); a.left = left.i(); a.degen = d_degen.i();
        return a;
    };
    {
        int64_t* hc = (int64_t*)h_ctl.p;
        hc[0] = 1; hc[1] = 0; hc[2] = m > x.prm.leaf_size ? 1 : 0; hc[3] = 0;
        HIPC(hipMemcpyAsync(d_ctl.p, hc, sizeof(int64_t) * 4, hipMemcpyHostToDevice, s));
        const int64_t init[2] = {0, m};
        HIPC(hipMemcpyAsync(d_start[0].p, init, sizeof init, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_cone_init, dim3(1), dim3(64), 0, s, level_args(0));
        HIPC(hipStreamSynchronize(s));   // the host copies above are in pageable memory
    }
    int level = 0;
    bool more = m > x.prm.leaf_size;
    const unsigned grid = (unsigned)((m + 255) / 256);
    // the first batch is the depth of a perfectly balanced tree, later ones are short
    int batch = 1;
    while (((int64_t)x.prm.leaf_size << batch) < m) batch++;
    while (more) {
        for (int rep = 0; rep < batch; rep++, level++) {
            const ConeLevelArgs a = level_args(level);
            for (int ph = 0; ph < 3; ph++) hipLaunchKernelGGL(k_cone_phase, dim3(grid), dim3(256), 0, s, a, ph);
            hipLaunchKernelGGL(k_cone_next, dim3(1), dim3(1024), 0, s, a);
            exclusive_scan_i32(left.i(), lscan.i(), m, scan_tmp.i(), s);
            hipLaunchKernelGGL(k_cone_scatter, dim3(grid), dim3(256), 0, s, a, (const int*)lscan.i(), perm_b.u32());
            HIPC(hipGetLastError());
            perm_a.swap(perm_b);
        }
        HIPC(hipMemcpyAsync(h_ctl.p, d_ctl.p, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        more = ((const int64_t*)h_ctl.p)[2] > 0;
        batch = 2;
    }
    const int64_t nseg_final = ((const int64_t*)h_ctl.p)[level & 1];
    std::vector<int64_t> starts(nseg_final + 1);
    HIPC(hipMemcpy(starts.data(), d_start[level & 1].p, sizeof(int64_t) * (nseg_final + 1), hipMemcpyDeviceToHost));

    // ---- leaves are the blocks; users move into leaf order
    x.nblocks = (int64_t)starts.size() - 1;
    x.block_start_h = starts;
    x.block_start.alloc(sizeof(int64_t) * starts.size());
    HIPC(hipMemcpyAsync(x.block_start.p, starts.data(), sizeof(int64_t) * starts.size(), hipMemcpyHostToDevice, s));
    x.user_perm.swap(perm_a);
    const int eb = elt_bytes(x.dtype);
    x.users.alloc((size_t)m * ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) x.user_scales.alloc(sizeof(float) * m);
    launch_gather_rows(x.dtype, users, x.d, user_scales, x.user_perm.u32(), m, x.d, x.users.p, ld,
                       x.user_scales.f(), s);
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
    la.unit = unit.f(); la.perm = x.user_perm.u32(); la.block_start = x.block_start.i64();
    la.nblocks = x.nblocks; la.m = m; la.d = x.d; la.ld = ld; la.k_max = x.prm.k_max;
    la.center = x.center.f(); la.cos_w = x.cos_w.f(); la.sin_w = x.sin_w.f(); la.block_ok = x.block_ok.i();
    la.unorm = x.unorm.f(); la.cos_t = x.cos_t.f(); la.sin_t = x.sin_t.f(); la.user_block = x.user_block.i();
    dim3 g((unsigned)((x.nblocks + 3) / 4)), b(256);
    if (x.dtype == DT_F32) hipLaunchKernelGGL(k_leaf_stats<DT_F32>, g, b, 0, s, la);
    else if (x.dtype == DT_BF16) hipLaunchKernelGGL(k_leaf_stats<DT_BF16>, g, b, 0, s, la);
    else hipLaunchKernelGGL(k_leaf_stats<DT_FP8>, g, b, 0, s, la);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));
}

void finish_blocks(Index& x, hipStream_t s)
{
    const int64_t tot = x.nblocks * x.prm.k_max;
    x.block_lb.alloc(sizeof(float) * tot);
    hipLaunchKernelGGL(k_block_lb, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x.lam64.d(),
                       x.user_n2.d(), x.block_start.i64(), x.block_ok.i(), x.nblocks, x.m, x.prm.k_max,
                       x.block_lb.f());
    HIPC(hipGetLastError());
}

}  // namespace rk
