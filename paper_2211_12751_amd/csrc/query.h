// Query-batch workspaces and the host steps shared by rkmips_query_batch and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "index.h"
#include "internal.h"

namespace rk {

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

// A run of queries (in k order) sharing one table of at most 8 distinct k values.
struct Group {
    int64_t begin = 0, end = 0;
    int nslots = 0;
};

// Device and pinned host buffers of one in-flight batch.
struct Workspace {
    int64_t nq_cap = 0, pool_cap = 0, amb_cap = 0;
    DevBuf qpad, qsc, qnorm, qslot, qorig, qk, slotk, offsets, pool, ids, amb, ctr;
    PinBuf h_qslot, h_qorig, h_qk, h_slotk, h_offsets, h_ids, h_ctr;
    std::vector<Group> groups;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_ctr = nullptr;
    Workspace();
    ~Workspace();
    void ensure(const Index& x, int64_t nq, int64_t pool_cap_req, int64_t amb_cap_req);
    static int64_t bytes_for(const Index& x, int64_t nq, int64_t pool_cap, int64_t amb_cap);
};

QueryArgs make_query_args(const Index& x, Workspace& w, int64_t nq, int flags);
void plan_batch(const Index& x, Workspace& w, const int32_t* ks, int64_t nq);
void enqueue_batch(const Index& x, Workspace& w, const void* queries, const float* qscales, int64_t nq,
                   int flags, hipStream_t s);
void finish_batch(Index& x, Workspace& w, const void* queries, const float* qscales, int64_t nq, int flags,
                  hipStream_t s, std::vector<int64_t>& offsets, std::vector<int32_t>& ids,
                  rkmips_query_stats& st);

}  // namespace rk
