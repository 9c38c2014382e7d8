// The index object behind rkmips_index (host side; all arrays live in device memory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <functional>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/rkmips.h"

namespace rk {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void alloc(size_t b);
    void reset();
    void swap(DevBuf& o)
    {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
    float* f() const { return (float*)p; }
    double* d() const { return (double*)p; }
    int* i() const { return (int*)p; }
    uint32_t* u32() const { return (uint32_t*)p; }
    uint16_t* u16() const { return (uint16_t*)p; }
    int64_t* i64() const { return (int64_t*)p; }
};

struct PinBuf {
    void* p = nullptr;
    size_t bytes = 0;
    PinBuf() = default;
    PinBuf(const PinBuf&) = delete;
    PinBuf& operator=(const PinBuf&) = delete;
    ~PinBuf();
    void alloc(size_t b);
    void reset();
};

struct Workspace;

// Ends the idle-release scope that ~Index opens; declared first in Index so that it is
// destroyed after every buffer member.
struct IdleTail {
    IdleTail() = default;
    ~IdleTail();
};

struct Index {
    IdleTail idle_tail;
    int device = 0;
    int mma_dtype = 0, mma_ld = 0;   // matrix-core operand type (DT_*) and row length
    double err_fast = 0;             // error bound of its fast scores, relative to ||u|| ||p||
    int num_cus = 256;
    int64_t n = 0, m = 0;
    int64_t n_lam = 0;   // items the lambda table covers: n, or |P'| (the first in norm order) in SAH mode
    int d = 0, ld = 0, dtype = 0;
    rkmips_params prm{};

    // items, sorted by descending canonical norm (Alg. 4 / Alg. 1 first step)
    DevBuf items, item_scales;   // [n x ld] storage dtype, [n]
    DevBuf item_order;           // uint32 [n] sorted position -> original item
    DevBuf item_n2;              // double [n] canonical squared norms, sorted order
    double max_item_norm = 0, max_user_norm = 0;

    // users in Cone-Tree leaf order
    DevBuf users, user_scales;   // [m x ld], [m]
    DevBuf users_mma;            // matrix-core user rows (split FP32 or widened FP8), leaf order
    DevBuf user_perm;            // uint32 [m] leaf position -> original user
    DevBuf user_inv;             // uint32 [m] original user -> leaf position (derived)
    DevBuf user_n2;              // double [m] leaf order
    DevBuf unorm, cos_t, sin_t;  // float [m] leaf order
    DevBuf user_block;           // int [m]

    // blocks (Cone-Tree leaves)
    int64_t nblocks = 0;
    DevBuf block_start;          // int64 [nblocks+1]
    DevBuf center;               // float [nblocks x ld] unit centres
    DevBuf center_mma;           // BF16 pair rows [nblocks x 2 ld] = [hi | lo] of the centres
                                 // (matrix-core operand of the block angles; not for FP32 MFMA)
    DevBuf cos_w, sin_w, block_ok;
    DevBuf block_lb;             // float [k_max x nblocks]

    // exact lambda table (leaf order, k-major)
    DevBuf lam64, lam32;
    int C = 0, G = 0, nseg = 1;
    int64_t ns = 0;              // item sample of the threshold seed pass (0: none)
    int64_t seg_len = 0;
    DevBuf cand, cand_cnt, cand_tau;  // raw candidates of the lambda pass
    int64_t cert_failures = 0;
    double max_rel_err_raw = 0, max_rel_err_l32 = 0;

    // SA-ALSH (Alg. 1)
    int t = 0;
    DevBuf part_start;           // int64 [t+1] (room for n+2)
    DevBuf num_parts;            // int: t
    DevBuf centroid;             // float [t x ld]
    DevBuf radius;               // float [t]
    DevBuf srp;                  // float [(d+1) x K]
    DevBuf item_codes;           // uint32 [n x K/32] sorted order
    DevBuf user_codes;           // uint32 [m x K/32] leaf order

    // reusable query workspaces (one per in-flight batch)
    std::mutex ws_mu;
    std::vector<std::unique_ptr<Workspace>> ws_all;
    std::vector<Workspace*> ws_free;
    Workspace* take_ws();
    void give_ws(Workspace* w);
    ~Index();

    // counters of every batch completed so far (rkmips_get_stats)
    std::mutex stats_mu;
    int64_t n_batches = 0, n_queries = 0;
    rkmips_query_stats qsum{};
    void add_batch_stats(int64_t nq, const rkmips_query_stats& st)
    {
        std::lock_guard<std::mutex> g(stats_mu);
        n_batches++;
        n_queries += nq;
        qsum.pairs_total += st.pairs_total; qsum.pairs_block_pruned += st.pairs_block_pruned;
        qsum.pairs_vector_pruned += st.pairs_vector_pruned; qsum.pairs_scored += st.pairs_scored;
        qsum.pairs_rechecked += st.pairs_rechecked; qsum.saalsh_checked += st.saalsh_checked;
        qsum.saalsh_rejects += st.saalsh_rejects; qsum.results += st.results; qsum.ms_total += st.ms_total;
    }

    double ms_norms = 0, ms_lambda = 0, ms_refine = 0, ms_saalsh = 0, ms_cone = 0, ms_total = 0;
    double ms_seed = 0, ms_topk = 0;
    PinBuf h_lam_stats;               // lambda build statistics, read once the build is complete
    std::vector<hipEvent_t> lam_ev;   // seed / top-k / refine boundaries of the build
    std::vector<hipEvent_t> build_ev; // phase boundaries of the build
    // The build returns once its work is queued: ready_ev follows its last kernel on the
    // build stream.  Host reads of index data wait for it (wait_ready, which also takes the
    // build statistics); work on another stream waits for it on the device (ready_on).
    hipEvent_t ready_ev = nullptr;
    std::once_flag stats_once;
    void wait_ready();
    void ready_on(hipStream_t s) const;

    int64_t device_bytes() const
    {
        const DevBuf* all[] = {&items, &item_scales, &item_order, &item_n2, &users, &user_scales, &users_mma,
                               &user_perm, &user_inv, &user_n2, &unorm, &cos_t, &sin_t, &user_block,
                               &block_start, &center, &center_mma, &cos_w, &sin_w, &block_ok, &block_lb,
                               &lam64, &lam32, &cand, &cand_cnt, &cand_tau, &part_start, &num_parts,
                               &centroid, &radius, &srp, &item_codes, &user_codes};
        int64_t s = 0;
        for (auto* b : all) s += (int64_t)b->bytes;
        return s;
    }
};

double fast_err_rel(int d);
double split_err_rel(int d);
void range_check(Index& x, const unsigned long long* stats);
// Working buffers of the Cone-Tree build, owned by the caller so that their release
// (and its host cost) can wait until the rest of the build is on its streams.
struct ConeWork {
    DevBuf unit, perm_a, perm_b, seg_a, seg_b, dot_l, left, lrank, blk_cnt;
    DevBuf d_start[2], d_act[2], d_key1[2], d_key2[2], d_ctl, d_nleft, d_degen, d_next_index;
    PinBuf h_ctl;
};
// Cone-Tree over the user directions (users end in leaf order).  `enqueued` runs once on
// the host after the first batch of levels is on the stream, before the host's first
// wait for them (work for other streams can be enqueued there).
// `cancel` (optional) is checked after each host wait: once set, the build stops there.
// `codes_padded` (optional, FP8 data): the users' codes in original order with rows of
// x.ld bytes, complete on `s`; the split products then run on them instead of BF16 unit rows.
void build_cone(Index& x, const void* users, const float* user_scales, const double* user_n2_orig,
                hipStream_t s, const std::function<void()>& enqueued, ConeWork& cw,
                const std::atomic<bool>* cancel = nullptr, const uint8_t* codes_padded = nullptr);
// L^j(B) for every block; lb_rows (optional): the lambda refine's leaf-order rows of
// lambda_u^(j) / ||u|| ([m x k_max]), else gathered from the lambda table
void finish_blocks(Index& x, hipStream_t s, const double* lb_rows = nullptr);
// Matrix-core operand of the block centres (x.center_mma), from x.center.
void make_center_operand(Index& x, hipStream_t s);
// x.user_inv from x.user_perm.
void make_user_inverse(Index& x, hipStream_t s);
void start_partitions(Index& x, int* h_num_parts, hipStream_t s);
// SA-ALSH index (Alg. 1) in three stream-ordered parts: the random projections, the item
// side (partition centroids, radii, item codes; needs x.t) and the user codes (users in
// leaf order).
void saalsh_projections(Index& x, const float* srp, hipStream_t s);
void saalsh_items(Index& x, hipStream_t s);
void saalsh_users(Index& x, hipStream_t s);

}  // namespace rk
