// Query-batch workspaces and the host steps shared by rkmips_query_batch and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "index.h"
#include "internal.h"

namespace rk {


// A run of queries (in k order) sharing one table of at most 8 distinct k values.
struct Group {
    int64_t begin = 0, end = 0;
    int nslots = 0;
};

// Device and pinned host buffers of one in-flight batch.
struct Workspace {
    int64_t nq_cap = 0, pool_cap = 0, amb_cap = 0;
    DevBuf qpad, qsc, qnorm, offsets, pool, ids, amb, ctr;
    // per-query tables of a batch, packed for one host-to-device copy: k-sorted position ->
    // caller index [nq], k slot [nq], k [nq], then the groups' slot tables [8 x groups]
    DevBuf meta;
    PinBuf h_meta;
    uint32_t* qorig = nullptr; int* qslot = nullptr; int* qk = nullptr; int* slotk = nullptr;   // in meta
    int64_t meta_ints = 0;                  // ints of meta this batch uses
    bool device_tail = false;               // recheck and lists were enqueued with the batch
    // answer bits [nq_cap x bm_words] (one bit per caller query and original user) when
    // they fit the budget: the lists then come out sorted without a pool or a sort
    DevBuf bitmap;
    int64_t bm_words = 0;
    bool bm_mode = false;                   // this batch uses the bits
    DevBuf cphi;                            // [nblocks x nq] query-centre cosines
    DevBuf prune;                           // [nblocks x ceil(nq / 32)] Lemma 2 prune words
    DevBuf qsplit;                          // matrix-core query rows (split FP32 or widened FP8)
    DevBuf qcnt, ids2;                      // per-query counts, scatter target of the lists
    DevBuf sa_scratch, sa_answer, sa_phi;   // SA-ALSH stage
    DevBuf sah_pairs, sah_score;            // SAH mode: pairs left to Alg. 2 (capacity amb_cap)
    DevBuf sah_need, sah_slot, sah_user;    // SAH mode: per-user flags and slots [m]
    DevBuf sah_tab;                         // SAH mode: per-user Alg. 2 tables, one chunk
    int64_t sah_chunk = 0;
    int sah_kstar = 0;                      // largest k of the batch
    PinBuf h_offsets, h_ids, h_ctr;
    std::vector<Group> groups;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_ctr = nullptr;
    Workspace();
    ~Workspace();
    void ensure(const Index& x, int64_t nq, int64_t pool_cap_req, int64_t amb_cap_req);
    static int64_t bytes_for(const Index& x, int64_t nq, int64_t pool_cap, int64_t amb_cap);
};

void run_saalsh(const Index& x, Workspace& w, const QueryArgs& a, int64_t npairs, hipStream_t s);
void run_sah(const Index& x, Workspace& w, const QueryArgs& a, hipStream_t s);
SaQueryArgs make_sa_args(const Index& x, const void* queries, const float* qscales, const int* qk,
                         const unsigned long long* pairs, int64_t npairs, float beta, double* phi, int* answer);
int64_t saalsh_scratch_stride(const Index& x, float beta);
QueryArgs make_query_args(const Index& x, Workspace& w, int64_t nq, int flags);
void plan_batch(const Index& x, Workspace& w, const int32_t* ks, int64_t nq);
void enqueue_batch(const Index& x, Workspace& w, const void* queries, const float* qscales, int64_t nq,
                   int flags, hipStream_t s);
void finish_batch(Index& x, Workspace& w, const void* queries, const float* qscales, int64_t nq, int flags,
                  hipStream_t s, std::vector<int64_t>& offsets, std::vector<int32_t>& ids,
                  rkmips_query_stats& st);

}  // namespace rk

// Outputs of one query batch (owned by the caller through the C handle).
struct rkmips_result {
    rk::Index* idx = nullptr;
    rk::Workspace* ws = nullptr;
    hipStream_t s = nullptr;
    int64_t nq = 0;
    int flags = 0;
    const void* queries = nullptr;
    const float* qscales = nullptr;
    bool done = false;
    rkmips_status status = RKMIPS_OK;
    std::string err;
    std::vector<int64_t> offsets;
    std::vector<int32_t> ids;
    rkmips_query_stats st{};
};


namespace rk {
rkmips_status guarded_call(void (*fn)(void*), void* ctx);
}  // namespace rk
