// C ABI of the exact RkMIPS library: argument validation, the index object and the
// orchestration of the build and query kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "index.h"
#include "internal.h"
#include "mem.h"
#include "query.h"

namespace rk {

static thread_local std::string g_last_error;

void fail(rkmips_status st, const std::string& msg) { throw Error{st, msg}; }

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) fail(RKMIPS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void host_wait(hipEvent_t e)
{
    for (;;) {
        const hipError_t r = hipEventQuery(e);
        if (r == hipSuccess) return;
        if (r != hipErrorNotReady) hip_check(r, "hipEventQuery");
    }
}

int elt_bytes(int dtype) { return dtype == RKMIPS_F32 ? 4 : dtype == RKMIPS_BF16 ? 2 : 1; }

int padded_dim(int d, int /*dtype*/)
{
    for (int p : {32, 64, 128, 256})
        if (d <= p) return p;
    return -1;
}

// ---------------------------------------------------------------- device buffers
DevBuf::~DevBuf() { reset(); }
void DevBuf::reset()
{
    if (p) mem::device_free(p, bytes);
    p = nullptr;
    bytes = 0;
}
void DevBuf::alloc(size_t b)
{
    reset();
    if (b == 0) b = 16;
    p = mem::device_alloc(b, nullptr);
    if (!p) fail(RKMIPS_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    bytes = b;
}

// Error bound of the fast scores relative to ||u|| ||x||: twice the classical
// gamma_{d+2} = (d+2)u / (1 - (d+2)u), u = 2^-24 (the factor 2 covers the matrix
// cores' unspecified summation order and rounding), plus the FP64 canonical form's own
// gamma_d at u = 2^-53.
double fast_err_rel(int d)
{
    const double u = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    const double g = (d + 2) * u / (1.0 - (d + 2) * u);
    const double g64 = d * u64 / (1.0 - d * u64);
    return 2.0 * g + g64;
}

// Split BF16 products for FP32 storage (items [h | l | h] against users [h | h | l]):
// the representation error of h.h + l.h + h.l against x.y is at most
// 3 * 2^-18 (1 + 2^-9)^2 |x_i y_i| per term, plus 2^-28 ||x|| ||y|| for the parts that
// fall below the BF16 subnormal range (non-zero norms are >= 1e-30 > 2^-100); the
// 3d BF16 products are exact in FP32 and their accumulation adds at most
// 2 gamma_{3d+2} times their absolute sum (<= (1 + 4 * 2^-9) sum |x_i y_i|); the FP64
// reference adds gamma64_d.  Relative to ||x|| ||y||.
double split_err_rel(int d)
{
    const double u = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53), b = std::ldexp(1.0, -9);
    const double rep = 3.0 * std::ldexp(1.0, -18) * (1.0 + b) * (1.0 + b) + std::ldexp(1.0, -28);
    const double n = 3.0 * d + 2.0;
    const double g = n * u / (1.0 - n * u);
    const double g64 = d * u64 / (1.0 - d * u64);
    return rep + 2.0 * g * (1.0 + 4.0 * b) + g64;
}

static float ev_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

struct Events {
    std::vector<hipEvent_t> ev;
    explicit Events(int k)
    {
        ev.resize(k, nullptr);
        for (auto& e : ev) HIPC(hipEventCreate(&e));
    }
    ~Events()
    {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------- build
void validate_params(const rkmips_params& p)
{
    if (p.k_max < 1 || p.k_max > 256) fail(RKMIPS_EINVAL, "k_max must be in [1, 256]");
    if (p.leaf_size < 1 || p.leaf_size > 64) fail(RKMIPS_EINVAL, "leaf_size must be in [1, 64]");
    if (p.num_hash < 32 || p.num_hash > 256 || p.num_hash % 32) fail(RKMIPS_EINVAL, "num_hash must be 32..256, a multiple of 32");
    if (p.topk_slack < 0 || p.topk_slack > 256) fail(RKMIPS_EINVAL, "topk_slack must be in [0, 256]");
    if (!(p.b > 0.f && p.b < 1.f)) fail(RKMIPS_EINVAL, "b must be in (0, 1)");
    if (!(p.probe_frac > 0.f && p.probe_frac <= 1.f)) fail(RKMIPS_EINVAL, "probe_frac must be in (0, 1]");
    if (p.mode != RKMIPS_MODE_EXACT && p.mode != RKMIPS_MODE_SAH && p.mode != RKMIPS_MODE_LAZY)
        fail(RKMIPS_EINVAL, "mode must be RKMIPS_MODE_EXACT, RKMIPS_MODE_SAH or RKMIPS_MODE_LAZY");
    if (p.sah_items < 0) fail(RKMIPS_EINVAL, "sah_items must be >= 0");
}

// Compute-unit count of a device (cached: the attribute query is not free).
static int device_cus(int dev)
{
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        cus = 256;
    }
    cache[dev] = cus;
    return cus;
}

// A second stream per device (default priority) for the build work that does not
// depend on lambda; it lives as long as the process.
static hipStream_t aux_stream(int dev)
{
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    std::lock_guard<std::mutex> g(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    HIPC(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams[dev] = st;
    return st;
}

// Operand form of the top-k passes: FP32 data as BF16 pairs [hi | lo] (three products
// per k-step on the matrix cores), otherwise the index's matrix-core form.
static int topk_dtype(const Index& x) { return x.mma_dtype; }
static int topk_ld(const Index& x) { return x.mma_ld; }

static void choose_topk(Index& x)
{
    const int C = x.prm.k_max + x.prm.topk_slack;
    x.C = C;
    if (C > 224) fail(RKMIPS_EINVAL, "k_max + topk_slack too large (at most 224)");
    // Seed pass: a stratified sample of ns items gives each user a threshold that about
    // target items of the whole set beat (the (2 TK_T)-th best of the sample scaled up),
    // so the main pass appends about target candidates per user and rarely compacts.
    const int64_t target = 4 * (int64_t)C;
    int64_t ns = (2 * TK_T * x.n_lam + target - 1) / target;
    x.ns = (x.n_lam >= 2048 && 4 * ns <= x.n_lam) ? ns : 0;
    int gpl = 2;
    if (x.ns > 0)
        while (gpl * 64 < 2 * target && gpl < 16) gpl *= 2;
    // each half-wave appends to its own half of a user's buffer; after a compaction the
    // C survivors sit in one half, which must still take a block's 16 appends
    while (gpl * 32 < C + 16) gpl *= 2;
    if (gpl > 16) fail(RKMIPS_EINVAL, "internal: candidate buffer too large");
    const int upb = topk_users_per_block(topk_dtype(x), topk_ld(x));
    const int64_t tiles = (x.m + upb - 1) / upb;
    // the buffers stay within a fixed share of the device memory
    while (gpl > 2 && gpl * 16 >= C + 16 && (double)x.m * gpl * 64 * 8 > 24e9) gpl /= 2;
    // Item segments (grid.y): the grid runs in rounds of the resident workgroups, so the
    // segment count is the one that fills its last round best (fewer on near ties).
    const int cus = x.num_cus;
    const int64_t slots = (int64_t)cus * topk_resident_blocks(topk_dtype(x), topk_ld(x), gpl * 64);
    int nmax = (int)std::min<int64_t>(std::max<int64_t>(1, x.n_lam / 1024), std::max(1, 2048 / (gpl * 64)));
    while (nmax > 1 && (double)x.m * nmax * gpl * 64 * 8 > 24e9) nmax--;
    int nmain = 1;
    double best = 0.0;
    for (int nm = 1; nm <= nmax; nm++) {
        const int64_t wgs = tiles * nm;
        const double eff = (double)wgs / (double)(((wgs + slots - 1) / slots) * slots);
        if (eff > best + 0.02) {
            best = eff;
            nmain = nm;
        }
    }
    int64_t seg_len = (x.n_lam + nmain - 1) / nmain;
    seg_len = std::max<int64_t>(64, (seg_len + 63) / 64 * 64);
    nmain = (int)((x.n_lam + seg_len - 1) / seg_len);
    x.nseg = nmain;
    x.seg_len = seg_len;
    x.G = gpl * 64;
}

// Items from which the main top-k pass waits for the build's second stream (see below).
static constexpr int64_t kMainWaitsItems = int64_t(1) << 18;

// Exact lambda table over the users in their ORIGINAL order (users_o: padded copy
// [m x ld], user_scales_o / user_n2_o in the same order); lambda rows and the raw
// candidates are indexed by original user.  Two stream-ordered halves without host
// synchronisation: the fused top-k passes, then the FP64 refine with the certificate.
struct LambdaBuild {
    DevBuf buf, cnt, tau, theta, fail_list, fail_count, errbits, spill, items3, users3, sel, sel_meta, sample,
        sample_sc, lb_rows;
    Events ev{4};   // start, after the main pass, after the refine, after the seed pass
};

static void lambda_topk(Index& x, LambdaBuild& L, const DevBuf& users_o, const float* user_scales_o,
                        hipStream_t s, const std::function<void()>& before_main)
{
    choose_topk(x);
    const int64_t m = x.m;
    L.buf.alloc(sizeof(uint2) * (size_t)m * x.nseg * x.G);
    L.cnt.alloc(sizeof(int) * (size_t)m * x.nseg * 2);
    L.tau.alloc(sizeof(float) * (size_t)m * x.nseg);
    L.fail_list.alloc(sizeof(int) * (size_t)m);
    L.fail_count.alloc(2 * sizeof(int));   // [0] certificate failures, [1] refine spills
    L.errbits.alloc(2 * kErrSlots * sizeof(unsigned long long));
    L.spill.alloc(sizeof(int) * (size_t)m);
    HIPC(hipMemsetAsync(L.fail_count.p, 0, 2 * sizeof(int), s));
    HIPC(hipMemsetAsync(L.errbits.p, 0, 2 * kErrSlots * sizeof(unsigned long long), s));
    x.lam64.alloc(sizeof(double) * (size_t)x.prm.k_max * m);
    x.lam32.alloc(sizeof(float) * (size_t)x.prm.k_max * m);

    // matrix-core operands: the stored rows, or their BF16 forms (split FP32, widened FP8)
    const void* mi = x.items.p;
    const void* mu = users_o.p;
    const int tdt = topk_dtype(x), tld = topk_ld(x);
    // FP8 rows of 256 codes: the seed pass below runs on the codes as they are (see there)
    const bool f8 = x.ns > 0 && x.dtype == RKMIPS_FP8_E4M3 && x.ld == 256;
    auto operands = [&] {
        if (tdt == DT_SPLIT) {
            launch_split_bf16((const float*)x.items.p, x.n_lam, x.ld, L.items3.u16(), 2, s);
            launch_split_bf16((const float*)users_o.p, m, x.ld, L.users3.u16(), 2, s);
        } else {
            launch_mma_operand(x.mma_dtype, x.dtype, x.items.p, x.n_lam, x.ld, L.items3.u16(), 0, s);
            launch_mma_operand(x.mma_dtype, x.dtype, users_o.p, m, x.ld, L.users3.u16(), 1, s);
        }
    };
    if (x.mma_dtype != x.dtype) {
        L.items3.alloc(sizeof(uint16_t) * (size_t)x.n_lam * tld);
        L.users3.alloc(sizeof(uint16_t) * (size_t)m * tld);
        if (!f8) operands();   // otherwise after the seed pass, which does not read them
        mi = L.items3.p;
        mu = L.users3.p;
    }
    TopkArgs ta{};
    ta.items = mi; ta.item_scales = x.item_scales.f(); ta.n = x.n_lam;
    ta.users = mu; ta.user_scales = user_scales_o; ta.m = m;
    ta.d = x.d; ta.ld = tld; ta.nseg_total = x.nseg; ta.C = x.C; ta.G = x.G;
    ta.buf = (uint2*)L.buf.p; ta.cnt = L.cnt.i(); ta.tau = L.tau.f();
    HIPC(hipEventRecord(L.ev.ev[0], s));
    if (x.ns > 0) {   // per-user threshold estimates from the item sample
        L.theta.alloc(sizeof(float) * (size_t)m);
        // FP8 rows of 256 codes: the estimate runs on the FP8 matrix cores with the codes as
        // they are (half the matrix-core time; the estimate needs no error bound, as the
        // certificate does not depend on it); otherwise on the main pass's operand form
        const int sdt = f8 ? DT_FP8 : tdt, sld = f8 ? x.ld : tld;
        // the sample's rows gathered first, so that the pass streams contiguous tiles
        L.sample.alloc((size_t)x.ns * topk_row_bytes(sdt, sld));
        if (x.item_scales.p) L.sample_sc.alloc(sizeof(float) * (size_t)x.ns);
        launch_gather_sample(sdt, f8 ? x.items.p : mi, x.item_scales.f(), x.n_lam, x.ns, sld, L.sample.p,
                             x.item_scales.p ? L.sample_sc.f() : nullptr, s);
        TopkArgs a0 = ta;
        if (f8) {
            a0.users = users_o.p;
            a0.ld = sld;
        }
        a0.items = L.sample.p;
        a0.item_scales = x.item_scales.p ? L.sample_sc.f() : nullptr;
        a0.n = x.ns;
        a0.ns = x.ns; a0.v0 = 0; a0.v1 = x.ns; a0.nseg = 1; a0.seg_base = 0; a0.seg_len = x.ns;
        a0.theta_out = L.theta.f();
        launch_topk_seed(sdt, a0, s);
    }
    if (f8 && x.mma_dtype != x.dtype) operands();
    before_main();
    HIPC(hipEventRecord(L.ev.ev[3], s));
    TopkArgs a1 = ta;
    a1.v0 = 0; a1.v1 = x.n_lam; a1.nseg = x.nseg; a1.seg_base = 0; a1.seg_len = x.seg_len;
    a1.theta_init = x.ns > 0 ? L.theta.f() : nullptr;
    a1.theta_stride = 1;
    launch_topk(tdt, a1, s);
    HIPC(hipEventRecord(L.ev.ev[1], s));
}

static void lambda_refine(Index& x, LambdaBuild& L, const DevBuf& users_o, const float* user_scales_o,
                          const double* user_n2_o, hipStream_t s)
{
    const int64_t m = x.m;
    RefineArgs ra{};
    ra.items = x.items.p; ra.item_scales = x.item_scales.f(); ra.n = x.n_lam;
    ra.users = users_o.p; ra.user_scales = user_scales_o; ra.m = m;
    ra.d = x.d; ra.ld = x.ld; ra.nseg = x.nseg; ra.C = x.C; ra.G = x.G; ra.k_max = x.prm.k_max;
    ra.buf = (const uint2*)L.buf.p; ra.cnt = L.cnt.i(); ra.tau = L.tau.f();
    ra.item_n2_sorted = x.item_n2.d(); ra.seg_len = x.seg_len; ra.user_n2 = user_n2_o;
    ra.force_fail = (x.prm.flags & RKMIPS_FLAG_NO_CERT) ? 1 : 0;
    ra.lam64 = x.lam64.d(); ra.lam32 = x.lam32.f();
    ra.fail_list = L.fail_list.i(); ra.fail_count = L.fail_count.i();
    ra.max_raw_err_bits = (unsigned long long*)L.errbits.p;
    ra.err_rel = x.err_fast;
    ra.spill = L.spill.i();
    ra.spill_count = L.fail_count.i() + 1;
    // lambda / ||u|| per user in Cone-Tree leaf order, for the block lower bounds
    L.lb_rows.alloc(sizeof(double) * (size_t)m * x.prm.k_max);
    ra.lb_rows = L.lb_rows.d();
    ra.leaf_of = x.user_inv.u32();
    {   // the select and rescoring kernels pass the kept candidates through memory
        L.sel.alloc(sizeof(uint2) * (size_t)m * x.C);
        L.sel_meta.alloc(sizeof(int) * 4 * (size_t)m);
        ra.sel = (uint2*)L.sel.p;
        ra.sel_meta = L.sel_meta.i();
    }
    launch_refine(x.dtype, ra, s);
    {
        // rows whose certificate failed: full FP64 rescoring (the count stays on the
        // device; with none the fallback workgroups exit at once).  One workgroup per
        // failed user at a time, up to 256 at once (one per compute unit) within 2 GB of
        // score rows (c5: 250 users at once; 32 had made 375 failures cost 4.3 s)
        const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(256, (int64_t)(2e9 / (8.0 * (double)x.n_lam))));
        DevBuf scratch;
        scratch.alloc(sizeof(double) * (size_t)rows * x.n_lam);
        launch_fallback(x.dtype, ra, scratch.d(), rows, s);
    }
    HIPC(hipEventRecord(L.ev.ev[2], s));
    // build statistics, read by the host after the build's final wait
    x.h_lam_stats.alloc(sizeof(unsigned long long) * (2 * kErrSlots + 1));
    unsigned long long* hs = (unsigned long long*)x.h_lam_stats.p;
    HIPC(hipMemcpyAsync(hs, L.errbits.p, 2 * kErrSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(hs + 2 * kErrSlots, L.fail_count.p, sizeof(int), hipMemcpyDeviceToHost, s));
    x.lam_ev.assign(4, nullptr);
    for (int i = 0; i < 4; i++) std::swap(x.lam_ev[i], L.ev.ev[i]);
    // keep the raw candidates for inspection (per original user)
    x.cand.swap(L.buf);
    x.cand_cnt.swap(L.cnt);
    x.cand_tau.swap(L.tau);
}

// Persistent host threads that queue a build's second-stream work (a thread started per
// build can take hundreds of microseconds to run).  One job at a time per thread; a
// build takes an idle one or starts another.  Never destroyed: the threads end with the
// process.
struct HostWorker {
    std::mutex mu;
    std::condition_variable cv;
    std::function<void()> job;
    bool busy = false;
    HostWorker()
    {
        std::thread([this] {
            for (;;) {
                std::function<void()> f;
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return (bool)job; });
                    f.swap(job);
                }
                f();   // jobs catch their own exceptions
                {
                    std::lock_guard<std::mutex> g(mu);
                    busy = false;
                }
                cv.notify_all();
            }
        }).detach();
    }
    void start(std::function<void()> f)
    {
        {
            std::lock_guard<std::mutex> g(mu);
            busy = true;
            job = std::move(f);
        }
        cv.notify_all();
    }
    void wait()
    {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return !busy; });
    }
};

// The idle workers (never destroyed).
struct WorkerPool {
    std::mutex mu;
    std::vector<HostWorker*> idle;
    HostWorker* take()
    {
        std::lock_guard<std::mutex> g(mu);
        if (idle.empty()) return new HostWorker;
        HostWorker* w = idle.back();
        idle.pop_back();
        return w;
    }
    void give(HostWorker* w)
    {
        w->wait();
        std::lock_guard<std::mutex> g(mu);
        idle.push_back(w);
    }
};

static WorkerPool& worker_pool()
{
    static WorkerPool* p = new WorkerPool;
    return *p;
}

static void build_index(Index& x, const void* items, const float* item_scales, const void* users,
                        const float* user_scales, const float* srp, hipStream_t s)
{
    const int64_t n = x.n, m = x.m;
    const int eb = elt_bytes(x.dtype);
    Events ev(9);
    HIPC(hipEventRecord(ev.ev[0], s));
    // ---- validation + canonical norms of the caller's arrays
    DevBuf nstats, n2_items_orig, n2_users_orig;
    nstats.alloc(sizeof(unsigned long long) * 4);
    n2_items_orig.alloc(sizeof(double) * n);
    n2_users_orig.alloc(sizeof(double) * m);
    unsigned long long* st = (unsigned long long*)nstats.p;
    launch_norm_stats_init(st, s);
    launch_norm2(x.dtype, users, user_scales, m, x.d, x.d, n2_users_orig.d(), st, 1, s);
    HIPC(hipEventRecord(ev.ev[8], s));   // the Cone-Tree build needs only the users and their norms
    const hipStream_t s2 = aux_stream(x.device);
    HIPC(hipStreamWaitEvent(s2, ev.ev[8], 0));
    launch_norm2(x.dtype, items, item_scales, n, x.d, x.d, n2_items_orig.d(), st, 0, s);
    PinBuf hst;
    hst.alloc(sizeof(unsigned long long) * 4);
    // read at the first host wait (inside the Cone-Tree build); until then the build
    // only runs bounded kernels whose results are discarded on a refusal
    HIPC(hipMemcpyAsync(hst.p, st, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost, s));

    // ---- item order (descending canonical norm, ties by index)
    int64_t cap = 2;
    while (cap < n) cap <<= 1;
    DevBuf keys, vals, tkeys, tvals;
    keys.alloc(sizeof(uint64_t) * cap);
    vals.alloc(sizeof(uint32_t) * cap);
    tkeys.alloc(sizeof(uint64_t) * cap);
    tvals.alloc(sizeof(uint32_t) * cap);
    launch_norm_keys(n2_items_orig.d(), n, cap, (uint64_t*)keys.p, (uint32_t*)vals.p, s);
    sort_pairs((uint64_t*)keys.p, (uint32_t*)vals.p, (uint64_t*)tkeys.p, (uint32_t*)tvals.p, n, cap, s);
    x.item_order.alloc(sizeof(uint32_t) * n);
    HIPC(hipMemcpyAsync(x.item_order.p, vals.p, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    x.item_n2.alloc(sizeof(double) * n);
    launch_permute_f64(n2_items_orig.d(), x.item_order.u32(), n, x.item_n2.d(), s);
    x.items.alloc((size_t)n * x.ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) x.item_scales.alloc(sizeof(float) * n);
    launch_gather_rows(x.dtype, items, x.d, item_scales, x.item_order.u32(), n, x.d, x.items.p, x.ld,
                       x.item_scales.f(), s);
    PinBuf hnp;
    hnp.alloc(sizeof(int));
    start_partitions(x, (int*)hnp.p, s);
    // padded copy of the users in their original order for the lambda build
    DevBuf users_o, uscales_o;
    users_o.alloc((size_t)m * x.ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) uscales_o.alloc(sizeof(float) * m);
    launch_gather_rows(x.dtype, users, x.d, user_scales, nullptr, m, x.d, users_o.p, x.ld, uscales_o.f(), s);
    HIPC(hipEventRecord(ev.ev[1], s));

    // The fused top-k passes (matrix-core bound) run on the caller's stream, followed by
    // the item side of SA-ALSH; the Cone-Tree (latency bound, host-checked) and the SA-ALSH
    // user codes run on a second stream, queued by a second host thread so that neither
    // stream waits for the other's launches.  The refine pass waits for the second stream:
    // enqueued earlier, its grid of one wave per user would hold the compute units the
    // second stream's kernels need.
    LambdaBuild L;
    ConeWork cone_work;
    struct Worker {
        HostWorker* hw = nullptr;
        std::mutex mu;
        std::condition_variable cv;
        bool srp_ready = false;
        bool side_queued = false;   // ev[7] recorded (or the worker failed)
        std::atomic<bool> cancel{false};
        std::exception_ptr err;
        hipStream_t s2 = nullptr;
        void ready()
        {
            {
                std::lock_guard<std::mutex> g(mu);
                srp_ready = true;
            }
            cv.notify_all();
        }
        void queued()
        {
            {
                std::lock_guard<std::mutex> g(mu);
                side_queued = true;
            }
            cv.notify_all();
        }
        void finish()
        {
            if (!hw) return;
            worker_pool().give(hw);   // waits for the job
            hw = nullptr;
        }
        ~Worker()
        {
            cancel = true;
            finish();
            if (err && s2) (void)hipStreamSynchronize(s2);   // its buffers are released next
        }
    } wk;
    wk.s2 = s2;
    wk.hw = worker_pool().take();
    wk.hw->start([&] {
        try {
            HIPC(hipSetDevice(x.device));
            mem::StreamScope scope2(s2);
            HIPC(hipEventRecord(ev.ev[2], s2));
            saalsh_projections(x, srp, s2);
            HIPC(hipEventRecord(ev.ev[6], s2));
            wk.ready();
            // ---- Cone-Tree over user directions; users are stored in leaf order.  With
            // many items it starts once the item order and the padded copies are done: its
            // row gathers would slow those copies several times over and delay the seed
            // pass (with few items the copies are short and the Cone-Tree sets the build).
            // After that wait the padded FP8 codes are complete, and the split products run
            // on them (half the bytes of BF16 unit rows).
            const bool after_copies = x.n_lam >= kMainWaitsItems;
            if (after_copies) HIPC(hipStreamWaitEvent(s2, ev.ev[1], 0));
            const bool codes = after_copies && x.dtype == RKMIPS_FP8_E4M3;
            build_cone(x, users, user_scales, n2_users_orig.d(), s2, nullptr, cone_work, &wk.cancel,
                       codes ? (const uint8_t*)users_o.p : nullptr);
            if (wk.cancel.load()) {
                wk.queued();
                return;
            }
            saalsh_users(x, s2);
            HIPC(hipEventRecord(ev.ev[7], s2));
            wk.queued();
        } catch (...) {
            wk.err = std::current_exception();
            wk.ready();
            wk.queued();
        }
    });
    // With many items the main pass is long (about 2n times the second stream's work per
    // user): it then waits for the second stream, whose kernels would otherwise be starved
    // by the main pass's workgroups and stretch across it, taking compute units from it the
    // whole time.  With few items the two overlap (their lengths are comparable).
    const bool main_waits = x.n_lam >= kMainWaitsItems;
    lambda_topk(x, L, users_o, uscales_o.f(), s, [&] {
        if (!main_waits) return;
        {
            std::unique_lock<std::mutex> lk(wk.mu);
            wk.cv.wait(lk, [&] { return wk.side_queued; });
        }
        if (!wk.err && !wk.cancel.load()) HIPC(hipStreamWaitEvent(s, ev.ev[7], 0));
    });
    // validation (the input statistics and the partition count were copied before ev1),
    // then the item side of SA-ALSH behind the top-k passes
    host_wait(ev.ev[1]);
    range_check(x, (const unsigned long long*)hst.p);
    x.t = *(const int*)hnp.p;
    {
        std::unique_lock<std::mutex> lk(wk.mu);
        wk.cv.wait(lk, [&] { return wk.srp_ready; });
    }
    if (!wk.err) {
        HIPC(hipStreamWaitEvent(s, ev.ev[6], 0));
        HIPC(hipEventRecord(ev.ev[4], s));
        saalsh_items(x, s);
        HIPC(hipEventRecord(ev.ev[5], s));
    }
    wk.finish();
    if (wk.err) std::rethrow_exception(wk.err);
    HIPC(hipStreamWaitEvent(s, ev.ev[7], 0));
    lambda_refine(x, L, users_o, uscales_o.f(), n2_users_orig.d(), s);

    // ---- per-block quantities that need lambda (L^j(B))
    finish_blocks(x, s, L.lb_rows.d());
    // ev[3] follows every kernel of the build: the second stream's work precedes ev[7],
    // which the caller's stream waited on.  No host wait here: the temporaries below go
    // back to the cache tagged with events on the caller's stream, and the caller can
    // queue its first query batch while the refine pass is still running.
    HIPC(hipEventRecord(ev.ev[3], s));
    x.build_ev.swap(ev.ev);
    x.ready_ev = x.build_ev[3];
}

// Build statistics, read once the build is complete (the timings need its events done).
static void take_build_stats(Index& x)
{
    const std::vector<hipEvent_t>& ev = x.build_ev;
    x.ms_saalsh = ev_ms(ev[4], ev[5]);
    const unsigned long long* hs = (const unsigned long long*)x.h_lam_stats.p;
    unsigned long long raw = 0, l32 = 0;   // non-negative doubles order like their bits
    for (int i = 0; i < kErrSlots; i++) {
        raw = std::max(raw, hs[i]);
        l32 = std::max(l32, hs[kErrSlots + i]);
    }
    std::memcpy(&x.max_rel_err_raw, &raw, 8);
    std::memcpy(&x.max_rel_err_l32, &l32, 8);
    x.cert_failures = (int64_t)*(const int*)(hs + 2 * kErrSlots);
    const std::vector<hipEvent_t>& le = x.lam_ev;
    x.ms_seed = ev_ms(le[0], le[3]);
    x.ms_topk = ev_ms(le[3], le[1]);
    x.ms_lambda = ev_ms(le[0], le[1]);
    x.ms_refine = ev_ms(le[1], le[2]);
    x.ms_norms = ev_ms(ev[0], ev[1]);
    x.ms_cone = ev_ms(ev[2], ev[7]);
    x.ms_total = ev_ms(ev[0], ev[3]);
}

// Item insertion (exact mode).  The new items' canonical scores enter the users' lambda
// rows (an item changes exactly the rows of the users it would be answered for as a
// query with k = k_max, ties aside), then the item side of the index is rebuilt as a build
// over the grown set would make it: norms, order, sorted rows, SA-ALSH partitions,
// centroids, radii and codes (same projections), and the block lower bounds.  The users,
// their blocks and codes do not change.
static void insert_items(Index& x, const void* items, const float* item_scales, int64_t n_new, hipStream_t s)
{
    x.wait_ready();
    const int64_t n0 = x.n, n1 = x.n + n_new;
    const int eb = elt_bytes(x.dtype);
    // validation and the range check against the users already in the index
    DevBuf nstats, n2new;
    nstats.alloc(sizeof(unsigned long long) * 4);
    n2new.alloc(sizeof(double) * n_new);
    unsigned long long* st = (unsigned long long*)nstats.p;
    launch_norm_stats_init(st, s);
    launch_norm2(x.dtype, items, item_scales, n_new, x.d, x.d, n2new.d(), st, 0, s);
    unsigned long long hst[4];
    HIPC(hipMemcpyAsync(hst, st, sizeof hst, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    double mi = 0.0;
    std::memcpy(&mi, &hst[0], 8);
    mi = std::max(mi, x.max_item_norm * x.max_item_norm);
    std::memcpy(&hst[0], &mi, 8);
    const double mu2 = x.max_user_norm * x.max_user_norm;
    std::memcpy(&hst[1], &mu2, 8);
    range_check(x, hst);   // also sets max_item_norm over the grown set
    // the new rows, padded; their scores enter the lambda rows
    DevBuf newrows, newsc, changed;
    newrows.alloc((size_t)n_new * x.ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) newsc.alloc(sizeof(float) * n_new);
    launch_gather_rows(x.dtype, items, x.d, item_scales, nullptr, n_new, x.d, newrows.p, x.ld, newsc.f(), s);
    changed.alloc(sizeof(unsigned long long));
    HIPC(hipMemsetAsync(changed.p, 0, sizeof(unsigned long long), s));
    launch_insert_lambda(x.dtype, x.users.p, x.user_scales.f(), x.user_perm.u32(), x.m, x.d, x.ld, newrows.p,
                         newsc.f(), n_new, x.lam64.d(), x.lam32.f(), x.prm.k_max, (unsigned long long*)changed.p, s);
    // every item in original order: the stored rows back at their ids, then the new ones
    std::vector<uint32_t> order(n0), inv(n0);
    HIPC(hipMemcpy(order.data(), x.item_order.p, sizeof(uint32_t) * n0, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n0; i++) inv[order[i]] = (uint32_t)i;
    DevBuf dinv, all, allsc, n2all, st2;
    dinv.alloc(sizeof(uint32_t) * n0);
    HIPC(hipMemcpy(dinv.p, inv.data(), sizeof(uint32_t) * n0, hipMemcpyHostToDevice));
    all.alloc((size_t)n1 * x.ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) allsc.alloc(sizeof(float) * n1);
    launch_gather_rows(x.dtype, x.items.p, x.ld, x.item_scales.f(), dinv.u32(), n0, x.d, all.p, x.ld, allsc.f(), s);
    HIPC(hipMemcpyAsync((char*)all.p + (size_t)n0 * x.ld * eb, newrows.p, (size_t)n_new * x.ld * eb,
                        hipMemcpyDeviceToDevice, s));
    if (x.dtype == RKMIPS_FP8_E4M3)
        HIPC(hipMemcpyAsync(allsc.f() + n0, newsc.p, sizeof(float) * n_new, hipMemcpyDeviceToDevice, s));
    // norms, order and sorted rows as in the build
    n2all.alloc(sizeof(double) * n1);
    st2.alloc(sizeof(unsigned long long) * 4);
    launch_norm_stats_init((unsigned long long*)st2.p, s);
    launch_norm2(x.dtype, all.p, allsc.f(), n1, x.d, x.ld, n2all.d(), (unsigned long long*)st2.p, 0, s);
    int64_t cap = 2;
    while (cap < n1) cap <<= 1;
    DevBuf keys, vals, tkeys, tvals;
    keys.alloc(sizeof(uint64_t) * cap);
    vals.alloc(sizeof(uint32_t) * cap);
    tkeys.alloc(sizeof(uint64_t) * cap);
    tvals.alloc(sizeof(uint32_t) * cap);
    launch_norm_keys(n2all.d(), n1, cap, (uint64_t*)keys.p, (uint32_t*)vals.p, s);
    sort_pairs((uint64_t*)keys.p, (uint32_t*)vals.p, (uint64_t*)tkeys.p, (uint32_t*)tvals.p, n1, cap, s);
    x.item_order.alloc(sizeof(uint32_t) * n1);
    HIPC(hipMemcpyAsync(x.item_order.p, vals.p, sizeof(uint32_t) * n1, hipMemcpyDeviceToDevice, s));
    x.item_n2.alloc(sizeof(double) * n1);
    launch_permute_f64(n2all.d(), x.item_order.u32(), n1, x.item_n2.d(), s);
    x.items.alloc((size_t)n1 * x.ld * eb);
    if (x.dtype == RKMIPS_FP8_E4M3) x.item_scales.alloc(sizeof(float) * n1);
    launch_gather_rows(x.dtype, all.p, x.ld, allsc.f(), x.item_order.u32(), n1, x.d, x.items.p, x.ld,
                       x.item_scales.f(), s);
    x.n = n1;
    x.n_lam = n1;
    // SA-ALSH item side over the grown set, then the block lower bounds
    PinBuf hnp;
    hnp.alloc(sizeof(int));
    start_partitions(x, (int*)hnp.p, s);
    HIPC(hipStreamSynchronize(s));
    x.t = *(int*)hnp.p;
    saalsh_items(x, s);
    finish_blocks(x, s);
    // the raw candidates describe the old item set
    x.cand.reset();
    x.cand_cnt.reset();
    x.cand_tau.reset();
    HIPC(hipStreamSynchronize(s));
}

void Index::wait_ready()
{
    if (!ready_ev) return;
    host_wait(ready_ev);
    std::call_once(stats_once, [this] { take_build_stats(*this); });
}

void Index::ready_on(hipStream_t s) const
{
    if (ready_ev) HIPC(hipStreamWaitEvent(s, ready_ev, 0));
}

// Refuse magnitudes where the FP32 fast path could overflow or lose the error model.
// Refuses non-finite inputs and magnitudes where the FP32 fast path could overflow or
// lose the error model.  st: max item n2, max user n2, min positive n2 (as bits), bad.
void range_check(Index& x, const unsigned long long* st)
{
    if (st[3]) fail(RKMIPS_EINVAL, "non-finite value (or NaN code / non-finite scale) in items or users");
    double mi, mu, lo;
    std::memcpy(&mi, &st[0], 8);
    std::memcpy(&mu, &st[1], 8);
    std::memcpy(&lo, &st[2], 8);
    if (st[2] == ~0ull) lo = INFINITY;
    if (std::sqrt(mi) * std::sqrt(mu) > 1e30) fail(RKMIPS_ERANGE, "max||u|| * max||p|| exceeds 1e30");
    if (lo < 1e-60) fail(RKMIPS_ERANGE, "a non-zero vector norm is below 1e-30");
    x.max_item_norm = std::sqrt(mi);
    x.max_user_norm = std::sqrt(mu);
}

Index::~Index()
{
    // every use of the index's buffers is complete: they go back to the cache as idle
    // blocks (the members are released after this body, the tail guard ends the scope)
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : lam_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : build_ev)
        if (e) (void)hipEventDestroy(e);
    mem::idle_enter();
}
IdleTail::~IdleTail() { mem::idle_leave(); }

}  // namespace rk

using namespace rk;

template <typename F>
static rkmips_status guarded(F&& f)
{
    try {
        g_last_error.clear();
        f();
        return RKMIPS_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return RKMIPS_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return RKMIPS_EDEVICE;
    }
}

namespace rk {
rkmips_status guarded_call(void (*fn)(void*), void* ctx)
{
    return guarded([&] { fn(ctx); });
}
}  // namespace rk

extern "C" {

void rkmips_default_params(rkmips_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);   // every field, including ones added later, starts at 0
    p->k_max = 50;
    p->leaf_size = 64;
    p->num_hash = 128;
    p->topk_slack = 14;
    p->b = 0.5f;
    p->probe_frac = 0.1f;
    p->seed = 221112751ull;
    p->mode = RKMIPS_MODE_EXACT;
    p->flags = 0;
    p->sah_items = 0;
}

const char* rkmips_last_error(void) { return g_last_error.c_str(); }

rkmips_status rkmips_diag_mma_probe(int32_t kind, const uint8_t* a_codes, const uint8_t* b_codes, int32_t k,
                                    float* c_out)
{
    return guarded([&] { mma_probe(kind, a_codes, b_codes, k, c_out); });
}

rkmips_status rkmips_diag_fp8_decode(const uint8_t* codes, int32_t n, float* out)
{
    return guarded([&] { fp8_decode(codes, n, out); });
}

rkmips_status rkmips_build_index(const void* items, const float* item_scales, int64_t n, const void* users,
                                 const float* user_scales, int64_t m, int32_t d, int32_t dtype,
                                 const float* srp_proj, const rkmips_params* p, void* stream,
                                 rkmips_index** out)
{
    return guarded([&] {
        if (!out) fail(RKMIPS_EINVAL, "out is NULL");
        *out = nullptr;
        if (!items || !users) fail(RKMIPS_EINVAL, "items/users is NULL");
        if (n < 1 || m < 1) fail(RKMIPS_EINVAL, "n and m must be >= 1");
        if (n > (int64_t)1 << 30 || m > (int64_t)1 << 30) fail(RKMIPS_EINVAL, "n and m must be <= 2^30");
        if (d < 1 || d > 256) fail(RKMIPS_EINVAL, "d must be in [1, 256]");
        if (dtype != RKMIPS_F32 && dtype != RKMIPS_BF16 && dtype != RKMIPS_FP8_E4M3)
            fail(RKMIPS_EINVAL, "unknown dtype");
        const bool fp8 = dtype == RKMIPS_FP8_E4M3;
        if (fp8 && (!item_scales || !user_scales)) fail(RKMIPS_EINVAL, "FP8 data needs item and user scales");
        if (!fp8 && (item_scales || user_scales)) fail(RKMIPS_EINVAL, "scales are only for FP8 data");
        rkmips_params prm;
        if (p) prm = *p;
        else rkmips_default_params(&prm);
        validate_params(prm);
        std::unique_ptr<Index> x(new Index());
        x->n = n; x->m = m; x->d = d; x->dtype = dtype; x->prm = prm;
        x->n_lam = n;
        if (prm.mode != RKMIPS_MODE_EXACT) {
            // Alg. 4: P' = the first O(k_max) items in norm order; the SA-ALSH index
            // needs at least one item outside it
            if (n < 2) fail(RKMIPS_EINVAL, "SAH mode needs n >= 2");
            const int64_t np = prm.sah_items > 0 ? prm.sah_items : std::min<int64_t>(2 * (int64_t)prm.k_max, n - 1);
            if (np >= n) fail(RKMIPS_EINVAL, "sah_items must be below n");
            x->n_lam = np;
            x->prm.sah_items = (int32_t)np;
            // the lazy mode scores every item of each partition Alg. 2 visits
            if (prm.mode == RKMIPS_MODE_LAZY) x->prm.probe_frac = 1.f;
        }
        x->ld = padded_dim(d, dtype);
        // FP32 storage is scored on the BF16 matrix cores as split products where the
        // tripled rows fit the kernels (ld <= 64), unless the caller asks for FP32 MFMA.
        // FP8 storage is widened to BF16 operands: the FP8 matrix cores' accumulation is
        // not within an FP32 rounding model (measured error up to 2^-10.6 of the sum of
        // |terms| per instruction), so no a-priori bound would hold for them.
        const bool split = dtype == RKMIPS_F32 && x->ld <= 64 && !(prm.flags & RKMIPS_FLAG_F32_MATRIX);
        x->mma_dtype = split ? DT_SPLIT : (dtype == RKMIPS_FP8_E4M3 ? DT_FP8B : dtype);
        x->mma_ld = split ? 2 * x->ld : x->ld;
        x->err_fast = split ? split_err_rel(d) : fast_err_rel(d);
        HIPC(hipGetDevice(&x->device));
        x->num_cus = device_cus(x->device);
        mem::StreamScope scope((hipStream_t)stream);
        build_index(*x, items, item_scales, users, user_scales, srp_proj, (hipStream_t)stream);
        *out = (rkmips_index*)x.release();
    });
}

void rkmips_index_free(rkmips_index* idx) { delete (Index*)idx; }

rkmips_status rkmips_insert_items(rkmips_index* idx, const void* items, const float* item_scales, int64_t n_new,
                                  void* stream)
{
    return guarded([&] {
        if (!idx || (n_new > 0 && !items)) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        if (n_new < 0) fail(RKMIPS_EINVAL, "n_new must be >= 0");
        if (x.prm.mode != RKMIPS_MODE_EXACT) fail(RKMIPS_EINVAL, "item insertion needs an exact-mode index");
        const bool fp8 = x.dtype == RKMIPS_FP8_E4M3;
        if (fp8 != (item_scales != nullptr)) fail(RKMIPS_EINVAL, "scales are required exactly for FP8 data");
        if (x.n + n_new > (int64_t)1 << 30) fail(RKMIPS_EINVAL, "n would exceed 2^30");
        if (n_new == 0) return;
        mem::StreamScope scope((hipStream_t)stream);
        insert_items(x, items, item_scales, n_new, (hipStream_t)stream);
    });
}

rkmips_status rkmips_index_wait(rkmips_index* idx)
{
    return guarded([&] {
        if (!idx) fail(RKMIPS_EINVAL, "NULL argument");
        ((Index*)idx)->wait_ready();
    });
}

rkmips_status rkmips_get_stats(const rkmips_index* idx, rkmips_stats* o)
{
    return guarded([&] {
        if (!idx || !o) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        std::memset(o, 0, sizeof *o);
        o->max_rel_err_raw = x.max_rel_err_raw;
        o->max_rel_err_lambda32 = x.max_rel_err_l32;
        o->cert_failures = x.cert_failures;
        o->fallback_rate = (double)x.cert_failures / (double)x.m;
        std::lock_guard<std::mutex> g(x.stats_mu);
        o->batches = x.n_batches;
        o->queries = x.n_queries;
        o->query = x.qsum;
        o->recheck_rate = x.qsum.pairs_scored > 0 ? (double)x.qsum.pairs_rechecked / (double)x.qsum.pairs_scored : 0.0;
    });
}

rkmips_status rkmips_get_info(const rkmips_index* idx, rkmips_index_info* o)
{
    return guarded([&] {
        if (!idx || !o) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        std::memset(o, 0, sizeof *o);
        o->n = x.n; o->m = x.m; o->d = x.d; o->dtype = x.dtype; o->k_max = x.prm.k_max;
        o->cand_per_user = x.G * x.nseg; o->num_hash = x.prm.num_hash; o->leaf_size = x.prm.leaf_size;
        o->num_partitions = x.t; o->num_blocks = x.nblocks; o->cert_failures = x.cert_failures;
        o->max_rel_err_raw = x.max_rel_err_raw; o->max_rel_err_lambda32 = x.max_rel_err_l32;
        o->ms_norms = x.ms_norms; o->ms_lambda = x.ms_lambda; o->ms_refine = x.ms_refine;
        o->ms_saalsh = x.ms_saalsh; o->ms_cone = x.ms_cone; o->ms_total = x.ms_total;
        o->ms_seed = x.ms_seed; o->ms_topk = x.ms_topk;
        o->mma_dtype = (x.mma_dtype == DT_FP8B || x.mma_dtype == DT_SPLIT) ? RKMIPS_BF16 : x.mma_dtype;
        o->mma_terms = x.mma_dtype == DT_SPLIT ? 3 : 1;
        o->err_fast = x.err_fast;
        o->mode = x.prm.mode;
        o->lambda_items = (int32_t)x.n_lam;
        o->device_bytes = x.device_bytes();
    });
}

rkmips_status rkmips_get_lambda(const rkmips_index* idx, int32_t k, double* out_m)
{
    return guarded([&] {
        if (!idx || !out_m) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (k < 1 || k > x.prm.k_max) fail(RKMIPS_ERANGE, "k outside [1, k_max]");
        HIPC(hipMemcpy(out_m, x.lam64.d() + (int64_t)(k - 1) * x.m, sizeof(double) * x.m, hipMemcpyDeviceToHost));
    });
}

rkmips_status rkmips_get_lambda32(const rkmips_index* idx, int32_t k, float* out_m)
{
    return guarded([&] {
        if (!idx || !out_m) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (k < 1 || k > x.prm.k_max) fail(RKMIPS_ERANGE, "k outside [1, k_max]");
        HIPC(hipMemcpy(out_m, x.lam32.f() + (int64_t)(k - 1) * x.m, sizeof(float) * x.m, hipMemcpyDeviceToHost));
    });
}

rkmips_status rkmips_get_item_order(const rkmips_index* idx, int64_t* order, double* norm2)
{
    return guarded([&] {
        if (!idx) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (order) {
            std::vector<uint32_t> o(x.n);
            HIPC(hipMemcpy(o.data(), x.item_order.p, sizeof(uint32_t) * x.n, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < x.n; i++) order[i] = o[i];
        }
        if (norm2) HIPC(hipMemcpy(norm2, x.item_n2.p, sizeof(double) * x.n, hipMemcpyDeviceToHost));
    });
}

rkmips_status rkmips_get_candidates(const rkmips_index* idx, int32_t* ids, float* scores, float* tau)
{
    return guarded([&] {
        if (!idx) fail(RKMIPS_EINVAL, "NULL argument");
        Index& x = *(Index*)idx;
        x.wait_ready();
        if (!x.cand.p) fail(RKMIPS_EINVAL, "candidates are not kept by this index");
        const int64_t per = (int64_t)x.nseg * x.G;
        std::vector<uint2> buf((size_t)x.m * per);
        std::vector<int> cnt((size_t)x.m * x.nseg * 2);
        std::vector<float> tt((size_t)x.m * x.nseg);
        std::vector<uint32_t> iorder(x.n);
        HIPC(hipMemcpy(buf.data(), x.cand.p, sizeof(uint2) * buf.size(), hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(cnt.data(), x.cand_cnt.p, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(tt.data(), x.cand_tau.p, sizeof(float) * tt.size(), hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(iorder.data(), x.item_order.p, sizeof(uint32_t) * x.n, hipMemcpyDeviceToHost));
        const int CP = x.G * x.nseg;
        for (int64_t u = 0; u < x.m; u++) {   // buffers are kept per original user
            const int64_t ou = u;
            int k = 0;
            float tmax = -INFINITY;
            for (int p = 0; p < 2 * x.nseg; p++) {
                const int s = p >> 1;
                const int c = cnt[(u * x.nseg + s) * 2 + (p & 1)];
                tmax = std::max(tmax, tt[u * x.nseg + s]);
                for (int i = 0; i < c; i++, k++) {
                    const uint2 e = buf[(u * x.nseg + s) * x.G + (p & 1) * (x.G / 2) + i];
                    float f;   // raw score bits
                    std::memcpy(&f, &e.x, 4);
                    if (ids) ids[ou * CP + k] = (int32_t)iorder[e.y];
                    if (scores) scores[ou * CP + k] = f;
                }
            }
            for (; k < CP; k++) {
                if (ids) ids[ou * CP + k] = -1;
                if (scores) scores[ou * CP + k] = -INFINITY;
            }
            if (tau) tau[ou] = tmax;
        }
    });
}

}  // extern "C"
