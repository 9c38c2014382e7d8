// Query batches: workspaces, the enqueue side (rkmips_query_batch) and the completion
// side (rkmips_result_wait: FP64 recheck of the close calls, sorted result lists).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "index.h"
#include "internal.h"
#include "mem.h"
#include "query.h"

namespace rk {

static const int kMaxSlots = 8;
// largest answer-bit array of one workspace (nq x ceil(m / 32) words); larger batches
// collect their answers in the pool and sort the lists
static const int64_t kBitmapBytes = (int64_t)64 << 20;

PinBuf::~PinBuf() { reset(); }
void PinBuf::reset()
{
    if (p) mem::host_free(p, bytes);
    p = nullptr;
    bytes = 0;
}
void PinBuf::alloc(size_t b)
{
    reset();
    if (b == 0) b = 16;
    p = mem::host_alloc(b, nullptr);
    if (!p) fail(RKMIPS_ENOMEM, "pinned host allocation failed");
    bytes = b;
}

static int64_t pow2ceil64(int64_t n)
{
    int64_t p = 2;
    while (p < n) p <<= 1;
    return p;
}

Workspace::Workspace() {}
Workspace::~Workspace()
{
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev_ctr) (void)hipEventDestroy(ev_ctr);
}

int64_t Workspace::bytes_for(const Index& x, int64_t nq, int64_t pool_cap, int64_t amb_cap)
{
    const int64_t eb = elt_bytes(x.dtype);
    return nq * x.ld * eb + nq * 5 * 4 + (nq + 1) * 8 + pool_cap * (8 + 4 + 4) + amb_cap * 8 + 256 +
           nq * x.nblocks * 4 + ((nq + 31) / 32 + 1) * x.nblocks * 4 + (x.mma_dtype != x.dtype ? nq * x.mma_ld * 2 : 0) +
           (nq * ((x.m + 31) / 32) * 4 <= kBitmapBytes ? nq * ((x.m + 31) / 32) * 4 : 0);
}

void Workspace::ensure(const Index& x, int64_t nq, int64_t pool_cap_req, int64_t amb_cap_req)
{
    if (!ev0) {
        HIPC(hipEventCreate(&ev0));
        HIPC(hipEventCreate(&ev1));
        HIPC(hipEventCreateWithFlags(&ev_ctr, hipEventDisableTiming));
    }
    if (nq > nq_cap || nq_cap == 0) {
        const int64_t c = std::max<int64_t>(nq, 64);
        qpad.alloc((size_t)c * x.ld * elt_bytes(x.dtype));
        if (x.mma_dtype != x.dtype) qsplit.alloc(sizeof(uint16_t) * (size_t)c * x.mma_ld);
        if (x.dtype == RKMIPS_FP8_E4M3) qsc.alloc(sizeof(float) * c);
        qnorm.alloc(sizeof(float) * c);
        meta.alloc(sizeof(int) * (3 * c + kMaxSlots * (c + 1)));
        h_meta.alloc(sizeof(int) * (3 * c + kMaxSlots * (c + 1)));
        offsets.alloc(sizeof(int64_t) * (c + 1));
        qcnt.alloc(sizeof(int) * c);
        h_offsets.alloc(sizeof(int64_t) * (c + 1));
        cphi.alloc(sizeof(float) * (size_t)c * std::max<int64_t>(x.nblocks, 1));
        prune.alloc(sizeof(uint32_t) * (size_t)((c + 31) / 32) * std::max<int64_t>(x.nblocks, 1));
        bm_words = (x.m + 31) / 32;
        if (c * bm_words * 4 <= kBitmapBytes) bitmap.alloc(sizeof(uint32_t) * (size_t)(c * bm_words));
        else bitmap.reset();
        nq_cap = c;
    }
    const int64_t pc = pow2ceil64(std::max<int64_t>(pool_cap_req, 1 << 12));
    if (pc > pool_cap) {
        pool.alloc(sizeof(uint64_t) * pc);
        ids.alloc(sizeof(int32_t) * pc);
        ids2.alloc(sizeof(int32_t) * pc);
        h_ids.alloc(sizeof(int32_t) * pc);
        pool_cap = pc;
    }
    const int64_t ac = std::max<int64_t>(amb_cap_req, 1 << 12);
    if (ac > amb_cap) {
        amb.alloc(sizeof(uint64_t) * ac);
        if (x.prm.mode != RKMIPS_MODE_EXACT) {
            sah_pairs.alloc(sizeof(uint64_t) * ac);
            sah_score.alloc(sizeof(double) * ac);
        }
        amb_cap = ac;
    }
    if (!ctr.p) {
        ctr.alloc(sizeof(unsigned long long) * 16);
        h_ctr.alloc(sizeof(unsigned long long) * 16);
    }
    if (x.prm.mode != RKMIPS_MODE_EXACT && !sah_need.p) {
        sah_need.alloc((size_t)x.m);
        sah_slot.alloc(sizeof(int) * (size_t)x.m);
        sah_user.alloc(sizeof(int) * (size_t)x.m);
        // tables of at most 1 GiB: chunk users at a time
        const int64_t row = (int64_t)(x.t + 1) * x.prm.k_max * (int64_t)sizeof(double);
        sah_chunk = std::max<int64_t>(1, std::min<int64_t>(x.m, (int64_t(1) << 30) / row));
        sah_tab.alloc((size_t)(sah_chunk * row));
    }
}

Workspace* Index::take_ws()
{
    std::lock_guard<std::mutex> g(ws_mu);
    if (!ws_free.empty()) {
        Workspace* w = ws_free.back();
        ws_free.pop_back();
        return w;
    }
    ws_all.emplace_back(new Workspace());
    return ws_all.back().get();
}
void Index::give_ws(Workspace* w)
{
    std::lock_guard<std::mutex> g(ws_mu);
    ws_free.push_back(w);
}

// bound constants
// Error bound of cos(phi) from the matrix cores (relative to ||q||, centres of unit norm),
// plus 2e-6 for the query norm, the stored centre and the final division:
//  - BF16 and widened FP8 queries are exact BF16 values and the centres enter as
//    hi + lo BF16 pairs: the lost part of a centre is below 2^-18 of it, and the 2d exact
//    products accumulate in FP32 (factor 2 for the matrix core's order);
//  - split FP32 queries take the three-product form of the fast scores;
//  - FP32 matrix cores: the fast-score bound itself.
static float phi_err(const Index& x)
{
    const int d = x.d;
    double e;
    if (x.mma_dtype == DT_SPLIT) e = split_err_rel(d);
    else if (x.mma_dtype == DT_F32) e = fast_err_rel(d);
    else {
        const double u = std::ldexp(1.0, -24), n = 2.0 * d + 2.0;
        e = std::ldexp(1.0, -18) + 2.0 * (n * u / (1.0 - n * u)) * (1.0 + std::ldexp(1.0, -8));
    }
    return (float)(e + 2e-6);
}
static const float kBoundSlack = 4e-6f;

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static void fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    HIPC(hipGetLastError());
}

QueryArgs make_query_args(const Index& x, Workspace& w, int64_t nq, int flags)
{
    QueryArgs a{};
    a.dtype = x.dtype;
    a.users = x.users.p; a.user_scales = x.user_scales.f(); a.m = x.m; a.d = x.d; a.ld = x.ld;
    a.unorm = x.unorm.f(); a.cos_t = x.cos_t.f(); a.sin_t = x.sin_t.f(); a.user_block = x.user_block.i();
    a.center = x.center.f(); a.cos_w = x.cos_w.f(); a.sin_w = x.sin_w.f(); a.block_ok = x.block_ok.i();
    a.center_mma = x.center_mma.u16();
    a.block_lb = x.block_lb.f(); a.nblocks = x.nblocks; a.perm = x.user_perm.u32();
    a.lam32 = x.lam32.f(); a.lam64 = x.lam64.d(); a.k_max = x.prm.k_max;
    a.queries = w.qpad.p; a.query_scales = w.qsc.f(); a.nq = nq; a.qnorm = w.qnorm.f(); a.cphi = w.cphi.f();
    a.prune = w.prune.u32(); a.ntq = (nq + 31) / 32;
    const bool split = x.mma_dtype != x.dtype;
    a.mma_users = split ? x.users_mma.p : x.users.p;
    a.mma_queries = split ? w.qsplit.p : w.qpad.p;
    a.mma_dtype = x.mma_dtype;
    a.mma_ld = x.mma_ld;
    a.qslot = w.qslot; a.qorig = w.qorig; a.qk = w.qk; a.slot_k = w.slotk;
    a.flags = flags | x.prm.flags;
    a.err_rel = x.err_fast;
    a.err_phi = phi_err(x);
    a.bound_slack = kBoundSlack;
    unsigned long long* c = (unsigned long long*)w.ctr.p;
    a.pool = (unsigned long long*)w.pool.p; a.pool_count = c + 0; a.pool_cap = w.pool_cap;
    a.bitmap = w.bm_mode ? w.bitmap.u32() : nullptr;
    a.bm_words = w.bm_words;
    a.amb = (unsigned long long*)w.amb.p; a.amb_count = c + 1; a.amb_cap = w.amb_cap;
    a.bad = (int*)(c + 2);
    a.stats = c + 8;
    a.sah = x.prm.mode != RKMIPS_MODE_EXACT;
    a.norm_widen = x.prm.mode == RKMIPS_MODE_LAZY ? std::ldexp(1.0, -40) : 0.0;
    a.item_n2 = x.item_n2.d(); a.n_items = x.n; a.user_n2 = x.user_n2.d();
    a.sah_pairs = (unsigned long long*)w.sah_pairs.p; a.sah_count = c + 6;
    a.sah_score = w.sah_score.d(); a.sah_need = (unsigned char*)w.sah_need.p;
    return a;
}

// Enqueue query prep and the fused bound/verify kernels for a batch whose host side
// (h_meta, groups) is already filled; without the SA-ALSH filter the FP64 recheck and
// the per-query lists follow on the device, with no host round trip in between.
void enqueue_batch(const Index& x, Workspace& w, const void* queries, const float* qscales, int64_t nq,
                   int flags, hipStream_t s)
{
    HIPC(hipMemsetAsync(w.ctr.p, 0, sizeof(unsigned long long) * 16, s));
    const int fl = flags | x.prm.flags;
    const bool sah = x.prm.mode != RKMIPS_MODE_EXACT;
    w.device_tail = nq > 0 && (sah || !((fl & RKMIPS_FLAG_SAALSH_FILTER) && !(fl & RKMIPS_FLAG_NO_SAALSH)));
    w.bm_mode = w.device_tail && w.bitmap.p != nullptr && !(fl & RKMIPS_FLAG_POOL_LISTS);
    if (w.bm_mode) HIPC(hipMemsetAsync(w.bitmap.p, 0, sizeof(uint32_t) * (size_t)(nq * w.bm_words), s));
    if (sah && nq > 0) HIPC(hipMemsetAsync(w.sah_need.p, 0, (size_t)x.m, s));
    if (nq > 0) {
        HIPC(hipMemcpyAsync(w.meta.p, w.h_meta.p, sizeof(int) * w.meta_ints, hipMemcpyHostToDevice, s));
        launch_gather_rows(x.dtype, queries, x.d, qscales, w.qorig, nq, x.d, w.qpad.p, x.ld, w.qsc.f(), s);
        QueryArgs a = make_query_args(x, w, nq, flags);
        launch_qnorm(x.dtype, w.qpad.p, w.qsc.f(), nq, x.d, x.ld, w.qnorm.f(), a.bad, s);
        if (x.mma_dtype != x.dtype) launch_mma_operand(x.mma_dtype, x.dtype, w.qpad.p, nq, x.ld, w.qsplit.u16(), 0, s);
        // the ring form of the verify pass reads the prune words only
        if (!(a.flags & RKMIPS_FLAG_NO_BOUNDS)) launch_phi(a, verify_uses_ring(a) ? nullptr : w.cphi.f(), s);
        for (size_t g = 0; g < w.groups.size(); g++) {
            QueryArgs ag = a;
            ag.slot_k = w.slotk + kMaxSlots * g;
            ag.nslots = w.groups[g].nslots;
            launch_verify_range(ag, w.groups[g].begin, w.groups[g].end, s);
        }
        if (w.device_tail) {
            // the FP64 recheck and the list building read the counts on the device; the
            // host checks them (bad values, overflow) once the offsets are back
            unsigned long long* c = (unsigned long long*)w.ctr.p;
            launch_recheck_device(a, s);
            if (sah) run_sah(x, w, a, s);
            if (w.bm_mode)
                launch_bitmap_lists(w.bitmap.u32(), w.bm_words, nq, w.qcnt.i(), w.offsets.i64(), (long long*)(c + 13),
                                    (int32_t*)w.ids.p, w.pool_cap, s);
            else
                launch_result_lists((const uint64_t*)w.pool.p, w.pool_cap, c + 5, nq, w.qcnt.i(), w.offsets.i64(),
                                    (long long*)(c + 13), (int32_t*)w.ids2.p, (int32_t*)w.ids.p, s);
            HIPC(hipMemcpyAsync(w.h_offsets.p, w.offsets.p, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToHost, s));
        }
    }
    HIPC(hipMemcpyAsync(w.h_ctr.p, w.ctr.p, sizeof(unsigned long long) * 16, hipMemcpyDeviceToHost, s));
    HIPC(hipEventRecord(w.ev_ctr, s));
}

// Host side of a batch: sort queries by k, split into groups of <= 8 distinct k.
void plan_batch(const Index& x, Workspace& w, const int32_t* ks, int64_t nq)
{
    std::vector<int64_t> ord(nq);
    for (int64_t i = 0; i < nq; i++) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return ks[a] < ks[b]; });
    w.groups.clear();
    // packed tables (host and device share the layout)
    int* hm = (int*)w.h_meta.p;
    uint32_t* qo = (uint32_t*)hm;
    int* qsl = hm + nq;
    int* qkk = hm + 2 * nq;
    int* sk = hm + 3 * nq;
    int* dm = w.meta.i();
    w.qorig = (uint32_t*)dm;
    w.qslot = dm + nq;
    w.qk = dm + 2 * nq;
    w.slotk = dm + 3 * nq;
    int64_t i = 0;
    while (i < nq) {
        Group g{};
        g.begin = i;
        g.nslots = 0;
        int* tab = sk + kMaxSlots * w.groups.size();
        while (i < nq) {
            const int k = ks[ord[i]];
            if (g.nslots == 0 || tab[g.nslots - 1] != k) {
                if (g.nslots == kMaxSlots) break;
                tab[g.nslots++] = k;
            }
            qo[i] = (uint32_t)ord[i];
            qsl[i] = g.nslots - 1;
            qkk[i] = k;
            i++;
        }
        g.end = i;
        w.groups.push_back(g);
    }
    w.meta_ints = 3 * nq + kMaxSlots * (int64_t)w.groups.size();
    w.sah_kstar = nq > 0 ? ks[ord[nq - 1]] : 0;   // queries sorted by k
    (void)x;
}

SaQueryArgs make_sa_args(const Index& x, const void* queries, const float* qscales, const int* qk,
                         const unsigned long long* pairs, int64_t npairs, float beta, double* phi, int* answer)
{
    SaQueryArgs sa{};
    sa.dtype = x.dtype;
    sa.items = x.items.p; sa.item_scales = x.item_scales.f(); sa.n = x.n; sa.d = x.d; sa.ld = x.ld;
    sa.users = x.users.p; sa.user_scales = x.user_scales.f();
    sa.queries = queries; sa.query_scales = qscales;
    sa.item_n2 = x.item_n2.d(); sa.user_n2 = x.user_n2.d();
    sa.part_start = x.part_start.i64(); sa.t = x.t;
    sa.item_codes = x.item_codes.u32(); sa.user_codes = x.user_codes.u32(); sa.K = x.prm.num_hash;
    sa.beta = beta;
    sa.pairs = pairs; sa.npairs = npairs; sa.qk = qk;
    sa.phi = phi; sa.answer = answer;
    return sa;
}

int64_t saalsh_scratch_stride(const Index& x, float beta)
{
    // probed candidates (at most ceil(beta |S_j|) per partition) plus SAH's P' scores
    return (int64_t)std::ceil((double)beta * (double)x.n) + x.t + 1 + x.prm.k_max;
}

void run_saalsh(const Index& x, Workspace& w, const QueryArgs& a, int64_t npairs, hipStream_t s)
{
    const int grid = (int)std::min<int64_t>(npairs, 128);
    const int64_t stride = saalsh_scratch_stride(x, x.prm.probe_frac);
    if ((int64_t)w.sa_scratch.bytes < (int64_t)sizeof(double) * grid * stride) w.sa_scratch.alloc(sizeof(double) * grid * stride);
    if ((int64_t)w.sa_answer.bytes < (int64_t)sizeof(int) * w.amb_cap) {
        w.sa_answer.alloc(sizeof(int) * w.amb_cap);
        w.sa_phi.alloc(sizeof(double) * w.amb_cap);
    }
    SaQueryArgs sa = make_sa_args(x, a.queries, a.query_scales, a.qk, a.amb, npairs, x.prm.probe_frac, w.sa_phi.d(),
                                  w.sa_answer.i());
    sa.overflow = a.bad;
    launch_saalsh_query(sa, w.sa_scratch.d(), w.sa_scratch.bytes, stride, grid, s);
}

// SAH mode (Alg. 5): Alg. 2 for the pairs the recheck left undecided, their count read
// on the device; a "yes" goes to the answers directly.
void run_sah(const Index& x, Workspace& w, const QueryArgs& a, hipStream_t s)
{
    const int64_t stride = saalsh_scratch_stride(x, x.prm.probe_frac);
    // candidate scratch of at most 2 GiB (the lazy mode takes whole partitions)
    const int grid = (int)std::min<int64_t>(std::min<int64_t>(w.sah_chunk, 2048),
                                            std::max<int64_t>(64, (int64_t(1) << 31) / (8 * stride)));
    if ((int64_t)w.sa_scratch.bytes < (int64_t)sizeof(double) * grid * stride) w.sa_scratch.alloc(sizeof(double) * grid * stride);
    SaQueryArgs sa = make_sa_args(x, a.queries, a.query_scales, a.qk, a.sah_pairs, w.amb_cap, x.prm.probe_frac,
                                  nullptr, nullptr);
    sa.npairs_dev = a.sah_count;
    sa.lam64 = x.lam64.d(); sa.perm = x.user_perm.u32(); sa.m = x.m; sa.n_init = x.n_lam;
    sa.bitmap = a.bitmap; sa.bm_words = a.bm_words;
    sa.pool = a.pool; sa.pool_count = a.pool_count; sa.pool_cap = a.pool_cap;
    sa.qorig = a.qorig;
    sa.rejects = a.stats + 4;
    sa.overflow = a.bad;
    sa.mu_scale = x.prm.mode == RKMIPS_MODE_LAZY ? 1.0 + 0x1p-40 : 1.0;
    unsigned long long* c = (unsigned long long*)w.ctr.p;
    launch_sah(sa, (const unsigned char*)w.sah_need.p, w.sah_slot.i(), w.sah_user.i(), (int*)(c + 7),
               w.sah_score.d(), w.sah_kstar, w.sah_tab.d(), w.sah_chunk, w.sa_scratch.d(), w.sa_scratch.bytes, stride,
               grid, s);
}

// Completion: overflow handling, FP64 recheck, sorted per-query lists, host copies.
void finish_batch(Index& x, Workspace& w, const void* queries, const float* qscales, int64_t nq, int flags,
                  hipStream_t s, std::vector<int64_t>& offsets, std::vector<int32_t>& ids, rkmips_query_stats& st)
{
    host_wait(w.ev_ctr);
    unsigned long long* hc = (unsigned long long*)w.h_ctr.p;
    if (hc[2] & 1ull) fail(RKMIPS_EINVAL, "non-finite value (or NaN code / non-finite scale) in the queries");
    if (hc[2] & 2ull) fail(RKMIPS_ERANGE, "a query norm is outside [1e-30, 1e30]");
    if (hc[2] & (unsigned long long)kSaalshOverflowBit) fail(RKMIPS_EDEVICE, "internal: SA-ALSH candidates overflowed");
    int64_t cnt = (int64_t)hc[0], namb = (int64_t)hc[1];
    // with answer bits the pool only holds the lists (offsets[nq] ids), else the yes
    // answers and the rechecked close calls
    auto need = [&] { return w.bm_mode ? ((const int64_t*)w.h_offsets.p)[nq] : cnt + namb; };
    if (need() > w.pool_cap || namb > w.amb_cap) {
        // the result pool was too small: grow it and run the batch again
        w.ensure(x, nq, 2 * need() + 1, 2 * namb + 1);
        enqueue_batch(x, w, queries, qscales, nq, flags, s);
        host_wait(w.ev_ctr);
        cnt = (int64_t)hc[0];
        namb = (int64_t)hc[1];
        if (need() > w.pool_cap || namb > w.amb_cap) fail(RKMIPS_ENOMEM, "result pool overflow");
    }
    st = rkmips_query_stats{};
    st.pairs_total = nq * x.m;
    st.pairs_block_pruned = (int64_t)hc[8];
    st.pairs_vector_pruned = (int64_t)hc[9];
    st.pairs_scored = (int64_t)hc[10];
    st.pairs_rechecked = namb;
    if (x.prm.mode != RKMIPS_MODE_EXACT) {
        st.saalsh_checked = (int64_t)hc[6];
        st.saalsh_rejects = (int64_t)hc[12];
    }
    const int* reject = nullptr;
    if (!w.device_tail) {
        QueryArgs a = make_query_args(x, w, nq, flags);
        fill_u64((unsigned long long*)w.pool.p + cnt, namb, ~0ull, s);
        if (namb > 0 && !w.device_tail) {
            // Alg. 2 as a proof-only filter on the close calls: a "no" there is exact
            run_saalsh(x, w, a, namb, s);
            reject = w.sa_answer.i();
            st.saalsh_checked = namb;
        }
        if (namb > 0) launch_recheck(a, namb, reject, s);
        const int64_t span = cnt + namb;
        long long* maxc = (long long*)((unsigned long long*)w.ctr.p + 13);
        launch_result_lists((const uint64_t*)w.pool.p, std::max<int64_t>(span, 0), nullptr, nq, w.qcnt.i(),
                            w.offsets.i64(), maxc, (int32_t*)w.ids2.p, (int32_t*)w.ids.p, s);
        if (nq > 0) {
            HIPC(hipMemcpyAsync(w.h_offsets.p, w.offsets.p, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToHost, s));
            HIPC(hipMemcpyAsync((unsigned long long*)w.h_ctr.p + 13, maxc, sizeof(long long), hipMemcpyDeviceToHost, s));
        }
        HIPC(hipStreamSynchronize(s));
    }
    if (nq == 0) ((int64_t*)w.h_offsets.p)[0] = 0;
    const int64_t* ho = (const int64_t*)w.h_offsets.p;
    const int64_t total = ho[nq];
    if (nq > 0 && !w.bm_mode) {
        // lists longer than one LDS chunk are merged now that their length is known
        const long long mc = (long long)((const unsigned long long*)w.h_ctr.p)[13];
        launch_result_merges(nq, mc, w.offsets.i64(), (int32_t*)w.ids2.p, (int32_t*)w.ids.p, s);
    }
    if (total > 0) {
        HIPC(hipMemcpyAsync(w.h_ids.p, w.ids.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
    }
    if (reject) HIPC(hipMemcpyAsync(w.h_ctr.p, w.ctr.p, sizeof(unsigned long long) * 16, hipMemcpyDeviceToHost, s));
    HIPC(hipEventRecord(w.ev1, s));
    host_wait(w.ev1);
    if (reject && (((unsigned long long*)w.h_ctr.p)[2] & (unsigned long long)kSaalshOverflowBit))
        fail(RKMIPS_EDEVICE, "internal: SA-ALSH candidates overflowed");
    if (reject) st.saalsh_rejects = (int64_t)((unsigned long long*)w.h_ctr.p)[12];
    offsets.assign(ho, ho + nq + 1);
    ids.assign((const int32_t*)w.h_ids.p, (const int32_t*)w.h_ids.p + total);
    st.results = total;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, w.ev0, w.ev1) != hipSuccess) (void)hipGetLastError();
    st.ms_total = ms;
}

}  // namespace rk

using namespace rk;

namespace rk {
rkmips_status guarded_call(void (*fn)(void*), void* ctx);
}

template <typename F>
static rkmips_status qguard(F&& f)
{
    struct Ctx { F* f; } c{&f};
    return rk::guarded_call([](void* p) { (*((Ctx*)p)->f)(); }, &c);
}

extern "C" {

}  // extern "C"

// Both query entry points: ks are host values here.
static void query_batch_host(rkmips_index* idx, const void* queries, const float* query_scales, int64_t nq,
                             const int32_t* ks, int32_t flags, void* stream, rkmips_result** out)
{
    {
        Index& x = *(Index*)idx;
        const bool fp8 = x.dtype == RKMIPS_FP8_E4M3;
        if (nq > 0 && fp8 && !query_scales) fail(RKMIPS_EINVAL, "FP8 queries need scales");
        if (!fp8 && query_scales) fail(RKMIPS_EINVAL, "scales are only for FP8 data");
        for (int64_t i = 0; i < nq; i++)
            if (ks[i] < 1 || ks[i] > x.prm.k_max) fail(RKMIPS_ERANGE, "k outside [1, k_max]");
        std::unique_ptr<rkmips_result> r(new rkmips_result());
        r->idx = &x;
        r->s = (hipStream_t)stream;
        r->nq = nq;
        r->flags = flags;
        r->queries = queries;
        r->qscales = query_scales;
        mem::StreamScope scope(r->s);
        Workspace* w = x.take_ws();
        try {
            // SAH mode hands every pair that passes the L_u^k test to the recheck: start
            // its list at a quarter of the pairs (at most 2^25; a longer list reruns the
            // batch once with room for all, and the workspace keeps that room)
            const int64_t amb0 = x.prm.mode != RKMIPS_MODE_EXACT
                                     ? std::min<int64_t>(int64_t(1) << 25, std::max<int64_t>(4 * nq, nq * x.m / 4))
                                     : 4 * nq;
            w->ensure(x, nq, std::max<int64_t>(1 << 16, 8 * nq * std::max(1, x.prm.k_max)), std::max<int64_t>(1 << 14, amb0));
            plan_batch(x, *w, ks, nq);
            x.ready_on(r->s);   // a batch on another stream waits for the build on the device
            HIPC(hipEventRecord(w->ev0, r->s));
            enqueue_batch(x, *w, queries, query_scales, nq, flags | x.prm.flags, r->s);
        } catch (...) {
            x.give_ws(w);
            throw;
        }
        r->ws = w;
        *out = r.release();
    }
}

static void query_batch_checks(rkmips_index* idx, const void* queries, int64_t nq, const int32_t* ks,
                               rkmips_result** out)
{
    if (!out) fail(RKMIPS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!idx) fail(RKMIPS_EINVAL, "index is NULL");
    if (nq < 0 || nq > ((int64_t)1 << 31) - 2) fail(RKMIPS_EINVAL, "nq out of range");
    if (nq > 0 && (!queries || !ks)) fail(RKMIPS_EINVAL, "queries/ks is NULL");
}

// ------------------------------------------------------------ no-allocation Alg. 2 probe
// rkmips_saalsh_probe_noalloc takes every device buffer it needs from this array: one
// copy per GPU, held until the process ends.  In host code the array's name is only a
// stand-in; host code uses the address hipGetSymbolAddress returns for the current
// device (noalloc_base).
static constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static unsigned char* noalloc_base()
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned char* base[kMaxDevices] = {};
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(RKMIPS_EDEVICE, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> g(mu);
    if (!base[dev]) {   // once per device, with that device current
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(RKMIPS_EDEVICE, std::string("no-allocation scratch: hipGetSymbolAddress: ") + hipGetErrorString(e));
        }
        base[dev] = (unsigned char*)p;
    }
    return base[dev];
}

// Consecutive 256-byte aligned pieces of the scratch array.
struct ScratchCarve {
    unsigned char* base;
    size_t used = 0;
    void* take(size_t bytes)
    {
        const size_t o = (used + 255) & ~(size_t)255;
        if (o > kNoAllocBytes || bytes > kNoAllocBytes - o)
            fail(RKMIPS_ERANGE, "batch exceeds the 64 MiB no-allocation scratch");
        used = o + bytes;
        return base + o;
    }
    size_t left() const
    {
        const size_t o = (used + 255) & ~(size_t)255;
        return o < kNoAllocBytes ? kNoAllocBytes - o : 0;
    }
};

// (query, original user) -> (query << 32 | leaf position of the user)
__global__ void k_pack_pairs(const int64_t* pq, const int64_t* pu, const uint32_t* inv, int64_t n,
                             unsigned long long* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = ((unsigned long long)pq[i] << 32) | inv[pu[i]];
}

extern "C" {

rkmips_status rkmips_query_batch(rkmips_index* idx, const void* queries, const float* query_scales, int64_t nq,
                                 const int32_t* ks, int32_t flags, void* stream, rkmips_result** out)
{
    return qguard([&] {
        query_batch_checks(idx, queries, nq, ks, out);
        // the k values are read on the host, which groups the queries by k: a copy
        // ordered after the stream's earlier work, then a host wait for that copy alone
        PinBuf hk;
        if (nq > 0) {
            hipStream_t s = (hipStream_t)stream;
            mem::StreamScope scope(s);
            hk.alloc(sizeof(int32_t) * (size_t)nq);
            HIPC(hipMemcpyAsync(hk.p, ks, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost, s));
            struct Ev {
                hipEvent_t e = nullptr;
                ~Ev() { if (e) (void)hipEventDestroy(e); }
            } ev;
            HIPC(hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
            HIPC(hipEventRecord(ev.e, s));
            host_wait(ev.e);
        }
        query_batch_host(idx, queries, query_scales, nq, (const int32_t*)hk.p, flags, stream, out);
    });
}

rkmips_status rkmips_query_batch_hostk(rkmips_index* idx, const void* queries, const float* query_scales,
                                       int64_t nq, const int32_t* ks, int32_t flags, void* stream,
                                       rkmips_result** out)
{
    return qguard([&] {
        query_batch_checks(idx, queries, nq, ks, out);
        query_batch_host(idx, queries, query_scales, nq, ks, flags, stream, out);
    });
}

rkmips_status rkmips_result_wait(rkmips_result* r)
{
    if (!r) return RKMIPS_EINVAL;
    if (r->done) return r->status;
    rkmips_status st = qguard([&] {
        mem::StreamScope scope(r->s);
        finish_batch(*r->idx, *r->ws, r->queries, r->qscales, r->nq, r->flags | r->idx->prm.flags, r->s, r->offsets,
                     r->ids, r->st);
    });
    r->done = true;
    r->status = st;
    if (st != RKMIPS_OK) {
        r->offsets.assign(r->nq + 1, 0);
        r->ids.clear();
    } else {
        r->idx->add_batch_stats(r->nq, r->st);
    }
    r->idx->give_ws(r->ws);
    r->ws = nullptr;
    return st;
}

rkmips_status rkmips_result_view(const rkmips_result* r, int64_t* nq, const int64_t** offsets, const int32_t** ids)
{
    if (!r) return RKMIPS_EINVAL;
    if (!r->done) return RKMIPS_EBUSY;
    if (r->status != RKMIPS_OK) return r->status;
    if (nq) *nq = r->nq;
    if (offsets) *offsets = r->offsets.data();
    if (ids) *ids = r->ids.data();
    return RKMIPS_OK;
}

rkmips_status rkmips_result_stats(const rkmips_result* r, rkmips_query_stats* out)
{
    if (!r || !out) return RKMIPS_EINVAL;
    if (!r->done) return RKMIPS_EBUSY;
    *out = r->st;
    return r->status;
}

void rkmips_result_free(rkmips_result* r)
{
    if (!r) return;
    if (!r->done) (void)rkmips_result_wait(r);
    delete r;
}

rkmips_status rkmips_saalsh_kmips(rkmips_index* idx, const int64_t* users, int64_t nu, int32_t k, float probe_frac,
                                  void* stream, double* scores_out)
{
    return qguard([&] {
        if (!idx) fail(RKMIPS_EINVAL, "index is NULL");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (nu < 0 || (nu > 0 && (!users || !scores_out))) fail(RKMIPS_EINVAL, "user or output array missing");
        // SAH and lazy indexes know u's scores on P' only to rank k_max
        const int kcap = x.prm.mode == RKMIPS_MODE_EXACT ? 256 : x.prm.k_max;
        if (k < 1 || k > kcap) fail(RKMIPS_ERANGE, "k outside [1, 256] (SAH and lazy indexes: [1, k_max])");
        if (!(probe_frac > 0.f && probe_frac <= 1.f)) fail(RKMIPS_EINVAL, "probe_frac must be in (0, 1]");
        if (nu == 0) return;
        std::vector<uint32_t> perm(x.m), inv(x.m);
        HIPC(hipMemcpy(perm.data(), x.user_perm.p, sizeof(uint32_t) * x.m, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < x.m; i++) inv[perm[i]] = (uint32_t)i;
        std::vector<int> leaf(nu);
        for (int64_t i = 0; i < nu; i++) {
            if (users[i] < 0 || users[i] >= x.m) fail(RKMIPS_EINVAL, "user index out of range");
            leaf[i] = (int)inv[users[i]];
        }
        hipStream_t s = (hipStream_t)stream;
        mem::StreamScope scope(s);
        const int64_t row = (int64_t)(x.t + 1) * k;
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nu, (int64_t(1) << 27) / row));   // 1 GiB
        const int64_t stride = saalsh_scratch_stride(x, probe_frac) + k;
        const int grid = (int)std::min<int64_t>(std::min<int64_t>(chunk, 2048),
                                                std::max<int64_t>(64, (int64_t(1) << 31) / (8 * stride)));
        DevBuf dleaf, dcount, tab, jl, scratch;
        dleaf.alloc(sizeof(int) * chunk);
        dcount.alloc(sizeof(int) * 2);   // [0]: users of the chunk, [1]: overflow flag
        tab.alloc(sizeof(double) * (size_t)(chunk * row));
        jl.alloc(sizeof(int) * chunk);
        scratch.alloc(sizeof(double) * (size_t)grid * stride);
        SaQueryArgs sa = make_sa_args(x, nullptr, nullptr, nullptr, nullptr, 0, probe_frac, nullptr, nullptr);
        // exact mode: the partitions cover all of P and the probes start from nothing; SAH
        // and lazy: they cover P minus P' and start from the scores on P' (the lambda rows)
        sa.lam64 = x.lam64.d(); sa.perm = x.user_perm.u32(); sa.m = x.m;
        sa.n_init = x.prm.mode == RKMIPS_MODE_EXACT ? 0 : x.n_lam;
        sa.mu_scale = 1.0;
        sa.overflow = dcount.i() + 1;
        std::vector<double> htab;
        std::vector<int> hj;
        for (int64_t c0 = 0; c0 < nu; c0 += chunk) {
            const int cn = (int)std::min<int64_t>(chunk, nu - c0);
            HIPC(hipStreamSynchronize(s));   // the previous chunk's kernel has read them
            HIPC(hipMemcpy(dleaf.p, leaf.data() + c0, sizeof(int) * cn, hipMemcpyHostToDevice));
            const int hc[2] = {cn, 0};
            HIPC(hipMemcpy(dcount.p, hc, sizeof(hc), hipMemcpyHostToDevice));
            launch_saalsh_kmips(sa, dleaf.i(), dcount.i(), cn, k, tab.d(), jl.i(), scratch.d(), scratch.bytes, stride,
                                grid, s);
            htab.resize((size_t)cn * row);
            hj.resize(cn);
            int flag = 0;
            HIPC(hipMemcpyAsync(htab.data(), tab.p, sizeof(double) * htab.size(), hipMemcpyDeviceToHost, s));
            HIPC(hipMemcpyAsync(hj.data(), jl.p, sizeof(int) * cn, hipMemcpyDeviceToHost, s));
            HIPC(hipMemcpyAsync(&flag, dcount.i() + 1, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (flag & kSaalshOverflowBit) fail(RKMIPS_EDEVICE, "internal: SA-ALSH candidates overflowed");
            for (int i = 0; i < cn; i++)
                std::memcpy(scores_out + (c0 + i) * k, htab.data() + (size_t)i * row + (size_t)hj[i] * k,
                            sizeof(double) * k);
        }
    });
}

rkmips_status rkmips_saalsh_probe_noalloc(rkmips_index* idx, const void* queries, const float* query_scales,
                                          int64_t nq, const int32_t* ks, const int64_t* pair_query,
                                          const int64_t* pair_user, int64_t npairs, float probe_frac, void* stream,
                                          double* phi_out, int32_t* answer_out)
{
    return qguard([&] {
        if (!idx) fail(RKMIPS_EINVAL, "index is NULL");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (nq < 1 || !queries || !ks) fail(RKMIPS_EINVAL, "queries/ks missing");
        if (npairs < 0 || (npairs > 0 && (!pair_query || !pair_user || !phi_out || !answer_out)))
            fail(RKMIPS_EINVAL, "pair arrays missing");
        if (!(probe_frac > 0.f && probe_frac <= 1.f)) fail(RKMIPS_EINVAL, "probe_frac must be in (0, 1]");
        const bool fp8 = x.dtype == RKMIPS_FP8_E4M3;
        if (fp8 != (query_scales != nullptr)) fail(RKMIPS_EINVAL, "scales are required exactly for FP8 data");
        for (int64_t i = 0; i < nq; i++)
            if (ks[i] < 1 || ks[i] > x.prm.k_max) fail(RKMIPS_ERANGE, "k outside [1, k_max]");
        for (int64_t i = 0; i < npairs; i++)
            if (pair_query[i] < 0 || pair_query[i] >= nq || pair_user[i] < 0 || pair_user[i] >= x.m)
                fail(RKMIPS_EINVAL, "pair index out of range");
        if (nq > ((int64_t)1 << 31) - 1) fail(RKMIPS_EINVAL, "nq out of range");
        if (npairs == 0) return;
        // every piece is carved (and the sizes checked) before the first device call
        ScratchCarve sc{noalloc_base()};
        void* qpad = sc.take((size_t)nq * x.ld * elt_bytes(x.dtype));
        float* qsc = fp8 ? (float*)sc.take(sizeof(float) * (size_t)nq) : nullptr;
        int* qk = (int*)sc.take(sizeof(int) * (size_t)nq);
        int64_t* dq = (int64_t*)sc.take(sizeof(int64_t) * (size_t)npairs);
        int64_t* du = (int64_t*)sc.take(sizeof(int64_t) * (size_t)npairs);
        unsigned long long* dpairs = (unsigned long long*)sc.take(sizeof(unsigned long long) * (size_t)npairs);
        double* phi = (double*)sc.take(sizeof(double) * (size_t)npairs);
        int* ans = (int*)sc.take(sizeof(int) * (size_t)npairs);
        int* dflag = (int*)sc.take(sizeof(unsigned long long));
        const int64_t stride = saalsh_scratch_stride(x, probe_frac);
        const int64_t fit = (int64_t)(sc.left() / (sizeof(double) * (size_t)stride + 256));
        const int grid = (int)std::min<int64_t>(std::min<int64_t>(npairs, 128), fit);
        if (grid < 1) fail(RKMIPS_ERANGE, "batch exceeds the 64 MiB no-allocation scratch");
        double* cand = (double*)sc.take(sizeof(double) * (size_t)grid * stride);
        hipStream_t s = (hipStream_t)stream;
        fill_u64((unsigned long long*)dflag, 1, 0ull, s);   // a kernel, not a memset node
        launch_gather_rows(x.dtype, queries, x.d, query_scales, nullptr, nq, x.d, qpad, x.ld, qsc, s);
        HIPC(hipMemcpyAsync(qk, ks, sizeof(int) * nq, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(dq, pair_query, sizeof(int64_t) * npairs, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(du, pair_user, sizeof(int64_t) * npairs, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_pack_pairs, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, dq, du,
                           x.user_inv.u32(), npairs, dpairs);
        HIPC(hipGetLastError());
        SaQueryArgs sa = make_sa_args(x, qpad, qsc, qk, dpairs, npairs, probe_frac, phi, ans);
        sa.overflow = dflag;
        launch_saalsh_query(sa, cand, sizeof(double) * (size_t)grid * stride, stride, grid, s);
        int flag = 0;
        HIPC(hipMemcpyAsync(phi_out, phi, sizeof(double) * npairs, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(answer_out, ans, sizeof(int) * npairs, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (flag & kSaalshOverflowBit) fail(RKMIPS_EDEVICE, "internal: SA-ALSH candidates overflowed");
    });
}

rkmips_status rkmips_saalsh_probe(rkmips_index* idx, const void* queries, const float* query_scales, int64_t nq,
                                  const int32_t* ks, const int64_t* pair_query, const int64_t* pair_user,
                                  int64_t npairs, float probe_frac, void* stream, double* phi_out, int32_t* answer_out)
{
    return qguard([&] {
        if (!idx) fail(RKMIPS_EINVAL, "index is NULL");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (nq < 1 || !queries || !ks) fail(RKMIPS_EINVAL, "queries/ks missing");
        if (npairs < 0 || (npairs > 0 && (!pair_query || !pair_user || !phi_out || !answer_out)))
            fail(RKMIPS_EINVAL, "pair arrays missing");
        if (!(probe_frac > 0.f && probe_frac <= 1.f)) fail(RKMIPS_EINVAL, "probe_frac must be in (0, 1]");
        const bool fp8 = x.dtype == RKMIPS_FP8_E4M3;
        if (fp8 != (query_scales != nullptr)) fail(RKMIPS_EINVAL, "scales are required exactly for FP8 data");
        for (int64_t i = 0; i < nq; i++)
            if (ks[i] < 1 || ks[i] > x.prm.k_max) fail(RKMIPS_ERANGE, "k outside [1, k_max]");
        std::vector<uint32_t> perm(x.m), inv(x.m);
        HIPC(hipMemcpy(perm.data(), x.user_perm.p, sizeof(uint32_t) * x.m, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < x.m; i++) inv[perm[i]] = (uint32_t)i;
        std::vector<unsigned long long> pairs(npairs);
        for (int64_t i = 0; i < npairs; i++) {
            if (pair_query[i] < 0 || pair_query[i] >= nq || pair_user[i] < 0 || pair_user[i] >= x.m)
                fail(RKMIPS_EINVAL, "pair index out of range");
            pairs[i] = ((unsigned long long)pair_query[i] << 32) | inv[pair_user[i]];
        }
        if (npairs == 0) return;
        hipStream_t s = (hipStream_t)stream;
        mem::StreamScope scope(s);
        DevBuf qpad, qsc, qk, dpairs, phi, ans, scratch, dflag;
        dflag.alloc(sizeof(int));
        HIPC(hipMemsetAsync(dflag.p, 0, sizeof(int), s));
        qpad.alloc((size_t)nq * x.ld * elt_bytes(x.dtype));
        if (fp8) qsc.alloc(sizeof(float) * nq);
        qk.alloc(sizeof(int) * nq);
        dpairs.alloc(sizeof(unsigned long long) * npairs);
        phi.alloc(sizeof(double) * npairs);
        ans.alloc(sizeof(int) * npairs);
        launch_gather_rows(x.dtype, queries, x.d, query_scales, nullptr, nq, x.d, qpad.p, x.ld, qsc.f(), s);
        HIPC(hipMemcpyAsync(qk.p, ks, sizeof(int) * nq, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(dpairs.p, pairs.data(), sizeof(unsigned long long) * npairs, hipMemcpyHostToDevice, s));
        const int grid = (int)std::min<int64_t>(npairs, 128);
        const int64_t stride = saalsh_scratch_stride(x, probe_frac);
        scratch.alloc(sizeof(double) * (size_t)grid * stride);
        SaQueryArgs sa = make_sa_args(x, qpad.p, qsc.f(), qk.i(), (const unsigned long long*)dpairs.p, npairs,
                                      probe_frac, phi.d(), ans.i());
        sa.overflow = dflag.i();
        launch_saalsh_query(sa, scratch.d(), scratch.bytes, stride, grid, s);
        int flag = 0;
        HIPC(hipMemcpyAsync(phi_out, phi.p, sizeof(double) * npairs, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(answer_out, ans.p, sizeof(int) * npairs, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(&flag, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (flag & kSaalshOverflowBit) fail(RKMIPS_EDEVICE, "internal: SA-ALSH candidates overflowed");
    });
}

rkmips_status rkmips_get_saalsh(const rkmips_index* idx, int64_t* part_start, float* centroid, float* radius,
                                uint32_t* item_codes, uint32_t* user_codes)
{
    return qguard([&] {
        if (!idx) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        const int W = x.prm.num_hash / 32;
        if (part_start) HIPC(hipMemcpy(part_start, x.part_start.p, sizeof(int64_t) * (x.t + 1), hipMemcpyDeviceToHost));
        if (centroid) {
            std::vector<float> c((size_t)x.t * x.ld);
            HIPC(hipMemcpy(c.data(), x.centroid.p, sizeof(float) * c.size(), hipMemcpyDeviceToHost));
            for (int j = 0; j < x.t; j++) std::memcpy(centroid + (int64_t)j * x.d, &c[(size_t)j * x.ld], sizeof(float) * x.d);
        }
        if (radius) HIPC(hipMemcpy(radius, x.radius.p, sizeof(float) * x.t, hipMemcpyDeviceToHost));
        if (item_codes) {
            std::vector<uint32_t> c((size_t)x.n * W), o(x.n);
            HIPC(hipMemcpy(c.data(), x.item_codes.p, sizeof(uint32_t) * c.size(), hipMemcpyDeviceToHost));
            HIPC(hipMemcpy(o.data(), x.item_order.p, sizeof(uint32_t) * x.n, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < x.n; i++) std::memcpy(item_codes + (int64_t)o[i] * W, &c[(size_t)i * W], 4 * W);
        }
        if (user_codes) {
            std::vector<uint32_t> c((size_t)x.m * W), o(x.m);
            HIPC(hipMemcpy(c.data(), x.user_codes.p, sizeof(uint32_t) * c.size(), hipMemcpyDeviceToHost));
            HIPC(hipMemcpy(o.data(), x.user_perm.p, sizeof(uint32_t) * x.m, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < x.m; i++) std::memcpy(user_codes + (int64_t)o[i] * W, &c[(size_t)i * W], 4 * W);
        }
    });
}

rkmips_status rkmips_get_blocks(const rkmips_index* idx, int32_t* leaf_users, int64_t* block_start, float* center,
                                float* cos_omega, float* sin_omega, float* cos_theta, float* sin_theta,
                                float* block_lb)
{
    return qguard([&] {
        if (!idx) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (leaf_users) {
            std::vector<uint32_t> o(x.m);
            HIPC(hipMemcpy(o.data(), x.user_perm.p, sizeof(uint32_t) * x.m, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < x.m; i++) leaf_users[i] = (int32_t)o[i];
        }
        if (block_start)
            HIPC(hipMemcpy(block_start, x.block_start.p, sizeof(int64_t) * (x.nblocks + 1), hipMemcpyDeviceToHost));
        if (center) {
            std::vector<float> c((size_t)x.nblocks * x.ld);
            HIPC(hipMemcpy(c.data(), x.center.p, sizeof(float) * c.size(), hipMemcpyDeviceToHost));
            for (int64_t b = 0; b < x.nblocks; b++) std::memcpy(center + b * x.d, &c[(size_t)b * x.ld], sizeof(float) * x.d);
        }
        if (cos_omega) HIPC(hipMemcpy(cos_omega, x.cos_w.p, sizeof(float) * x.nblocks, hipMemcpyDeviceToHost));
        if (sin_omega) HIPC(hipMemcpy(sin_omega, x.sin_w.p, sizeof(float) * x.nblocks, hipMemcpyDeviceToHost));
        if (cos_theta) HIPC(hipMemcpy(cos_theta, x.cos_t.p, sizeof(float) * x.m, hipMemcpyDeviceToHost));
        if (sin_theta) HIPC(hipMemcpy(sin_theta, x.sin_t.p, sizeof(float) * x.m, hipMemcpyDeviceToHost));
        if (block_lb) HIPC(hipMemcpy(block_lb, x.block_lb.p, sizeof(float) * x.nblocks * x.prm.k_max, hipMemcpyDeviceToHost));
    });
}

}  // extern "C"
