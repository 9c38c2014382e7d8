// Continuous-batching server (replay of a timed request stream).
//
// A feeder thread releases each request at its arrival time into the arrival queue.
// The dispatcher forms a batch of up to max_batch arrived requests whenever one of
// the stream slots is free; the number of slots is admitted by the memory budget (each
// slot owns preallocated device and pinned buffers, so nothing is allocated while
// serving).  Each slot has its own stream and completion thread, so batches that are
// admitted while others are still on the GPU overlap on the device; the completion
// thread takes the batch's close calls again in canonical FP64, assembles the sorted
// answers and records each request's latency (arrival to host-visible answer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "index.h"
#include "internal.h"
#include "mem.h"
#include "query.h"

namespace rk {

using Clock = std::chrono::steady_clock;

namespace {

struct Slot {
    int id = 0;
    hipStream_t stream = nullptr;
    Workspace ws;
    DevBuf dq, dqs;        // batch queries on the device
    PinBuf hq, hqs, hks;   // pinned staging of the batch
    std::vector<int64_t> members;   // request indices of the running batch
    bool busy = false;
    bool has_work = false;
    std::thread thr;
};

struct Server {
    Index* x = nullptr;
    const uint8_t* queries = nullptr;
    const float* qscales = nullptr;
    const int32_t* ks = nullptr;
    const int64_t* arrival = nullptr;
    int64_t nq = 0;
    rkmips_serve_params sp{};
    int64_t row_bytes = 0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<int64_t> arrived;
    bool feeding_done = false;
    bool stop = false;
    int inflight = 0;
    int64_t max_inflight = 0, batches = 0;
    Clock::time_point t0;
    std::vector<double> t_arrive, t_done;
    std::vector<std::vector<int32_t>> answers;
    std::vector<std::unique_ptr<Slot>> slots;
    rkmips_status err = RKMIPS_OK;
    std::string errmsg;

    double now_us() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }

    void record_error(const Error& e)
    {
        std::lock_guard<std::mutex> g(mu);
        if (err == RKMIPS_OK) {
            err = e.st;
            errmsg = e.msg;
        }
        stop = true;
        cv.notify_all();
    }

    void feeder()
    {
        for (int64_t i = 0; i < nq; i++) {
            const auto due = t0 + std::chrono::microseconds(arrival[i]);
            std::this_thread::sleep_until(due);
            std::lock_guard<std::mutex> g(mu);
            if (stop) return;
            t_arrive[i] = now_us();
            arrived.push_back(i);
            cv.notify_all();
        }
        std::lock_guard<std::mutex> g(mu);
        feeding_done = true;
        cv.notify_all();
    }

    void completion(Slot* s)
    {
        HIPC(hipSetDevice(x->device));
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return s->has_work || stop; });
                if (!s->has_work) return;
            }
            try {
                mem::StreamScope scope(s->stream);
                const int64_t B = (int64_t)s->members.size();
                std::vector<int64_t> off;
                std::vector<int32_t> ids;
                rkmips_query_stats st{};
                finish_batch(*x, s->ws, s->dq.p, s->dqs.f(), B, sp.flags | x->prm.flags, s->stream, off, ids, st);
                const double t = now_us();
                std::lock_guard<std::mutex> g(mu);
                for (int64_t j = 0; j < B; j++) {
                    const int64_t r = s->members[j];
                    answers[r].assign(ids.begin() + off[j], ids.begin() + off[j + 1]);
                    t_done[r] = t;
                }
                s->has_work = false;
                s->busy = false;
                inflight--;
                cv.notify_all();
            } catch (const Error& e) {
                record_error(e);
                return;
            }
        }
    }

    void dispatch(Slot* s, std::vector<int64_t>& batch)
    {
        mem::StreamScope scope(s->stream);
        const int64_t B = (int64_t)batch.size();
        uint8_t* hq = (uint8_t*)s->hq.p;
        float* hqs = (float*)s->hqs.p;
        int32_t* hk = (int32_t*)s->hks.p;
        for (int64_t j = 0; j < B; j++) {
            const int64_t r = batch[j];
            std::memcpy(hq + j * row_bytes, queries + r * row_bytes, row_bytes);
            if (qscales) hqs[j] = qscales[r];
            hk[j] = ks[r];
        }
        HIPC(hipMemcpyAsync(s->dq.p, hq, row_bytes * B, hipMemcpyHostToDevice, s->stream));
        if (qscales) HIPC(hipMemcpyAsync(s->dqs.p, hqs, sizeof(float) * B, hipMemcpyHostToDevice, s->stream));
        plan_batch(*x, s->ws, hk, B);
        HIPC(hipEventRecord(s->ws.ev0, s->stream));
        enqueue_batch(*x, s->ws, s->dq.p, qscales ? s->dqs.f() : nullptr, B, sp.flags | x->prm.flags, s->stream);
    }

    void run()
    {
        std::thread feed(&Server::feeder, this);
        for (auto& s : slots) s->thr = std::thread(&Server::completion, this, s.get());
        std::vector<int64_t> batch;
        for (;;) {
            Slot* free_slot = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] {
                    if (stop) return true;
                    if (arrived.empty()) return feeding_done;
                    for (auto& s : slots)
                        if (!s->busy) return true;
                    return false;
                });
                if (stop || (arrived.empty() && feeding_done)) break;
                for (auto& s : slots)
                    if (!s->busy) { free_slot = s.get(); break; }
                batch.clear();
                while (!arrived.empty() && (int64_t)batch.size() < sp.max_batch) {
                    batch.push_back(arrived.front());
                    arrived.pop_front();
                }
                free_slot->busy = true;
                free_slot->members = batch;
                inflight++;
                max_inflight = std::max<int64_t>(max_inflight, inflight);
                batches++;
            }
            try {
                dispatch(free_slot, batch);
            } catch (const Error& e) {
                record_error(e);
                break;
            }
            std::lock_guard<std::mutex> g(mu);
            free_slot->has_work = true;
            cv.notify_all();
        }
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return inflight == 0 || stop; });
            stop = true;
            cv.notify_all();
        }
        feed.join();
        for (auto& s : slots) s->thr.join();
    }
};

}  // namespace
}  // namespace rk

using namespace rk;

template <typename F>
static rkmips_status sguard(F&& f)
{
    struct Ctx { F* f; } c{&f};
    return rk::guarded_call([](void* p) { (*((Ctx*)p)->f)(); }, &c);
}

extern "C" rkmips_status rkmips_serve_replay(rkmips_index* idx, const void* queries, const float* query_scales,
                                             int64_t nq, const int32_t* ks, const int64_t* arrival_us,
                                             const rkmips_serve_params* sp, double* latency_us,
                                             rkmips_serve_stats* stats, rkmips_result** out)
{
    return sguard([&] {
            const float* qs = query_scales;
            const int64_t* arr = arrival_us;
            double* lat = latency_us;
            if (!out) fail(RKMIPS_EINVAL, "out is NULL");
            *out = nullptr;
            if (!idx || !sp || !lat) fail(RKMIPS_EINVAL, "NULL argument");
            Index& x = *(Index*)idx;
            x.wait_ready();
            if (nq < 0) fail(RKMIPS_EINVAL, "nq < 0");
            if (nq > 0 && (!queries || !ks || !arr)) fail(RKMIPS_EINVAL, "queries/ks/arrival_us is NULL");
            const bool fp8 = x.dtype == RKMIPS_FP8_E4M3;
            if (nq > 0 && fp8 && !qs) fail(RKMIPS_EINVAL, "FP8 queries need scales");
            if (!fp8 && qs) fail(RKMIPS_EINVAL, "scales are only for FP8 data");
            if (sp->max_batch < 1 || sp->max_batch > 4096) fail(RKMIPS_EINVAL, "max_batch must be in [1, 4096]");
            if (sp->num_streams < 1 || sp->num_streams > 8) fail(RKMIPS_EINVAL, "num_streams must be in [1, 8]");
            for (int64_t i = 0; i < nq; i++) {
                if (ks[i] < 1 || ks[i] > x.prm.k_max) fail(RKMIPS_ERANGE, "k outside [1, k_max]");
                if (arr[i] < 0 || (i > 0 && arr[i] < arr[i - 1])) fail(RKMIPS_EINVAL, "arrival times must be non-negative and non-decreasing");
            }
            Server S;
            S.x = &x;
            S.queries = (const uint8_t*)queries;
            S.qscales = qs;
            S.ks = ks;
            S.arrival = arr;
            S.nq = nq;
            S.sp = *sp;
            S.row_bytes = (int64_t)x.d * elt_bytes(x.dtype);
            const int64_t B = sp->max_batch;
            const int64_t pool = std::max<int64_t>(1 << 16, 8 * B * x.prm.k_max);
            const int64_t amb = std::max<int64_t>(1 << 14, 4 * B);
            const int64_t slot_bytes = Workspace::bytes_for(x, B, pool, amb) + B * S.row_bytes + B * 4;
            int nslots = sp->num_streams;
            if (sp->mem_budget > 0) nslots = (int)std::min<int64_t>(nslots, sp->mem_budget / slot_bytes);
            if (nslots < 1) fail(RKMIPS_ENOMEM, "memory budget below one batch slot");
            HIPC(hipSetDevice(x.device));
            for (int i = 0; i < nslots; i++) {
                auto s = std::make_unique<Slot>();
                s->id = i;
                HIPC(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
                s->ws.ensure(x, B, pool, amb);
                s->dq.alloc(B * S.row_bytes);
                if (fp8) s->dqs.alloc(sizeof(float) * B);
                s->hq.alloc(B * S.row_bytes);
                s->hqs.alloc(sizeof(float) * B);
                s->hks.alloc(sizeof(int32_t) * B);
                S.slots.push_back(std::move(s));
            }
            S.t_arrive.assign(nq, 0.0);
            S.t_done.assign(nq, 0.0);
            S.answers.assign(nq, {});
            S.t0 = Clock::now();
            S.run();
            for (auto& s : S.slots)
                if (s->stream) (void)hipStreamSynchronize(s->stream);
            {
                // the slots' buffers are idle now: back to the cache for any stream
                mem::IdleScope idle;
                for (auto& s : S.slots) {
                    if (s->stream) (void)hipStreamDestroy(s->stream);
                    s->stream = nullptr;
                }
                S.slots.clear();
            }
            if (S.err != RKMIPS_OK) fail(S.err, S.errmsg);
            std::unique_ptr<rkmips_result> r(new rkmips_result());
            r->idx = &x;
            r->nq = nq;
            r->done = true;
            r->offsets.assign(nq + 1, 0);
            for (int64_t i = 0; i < nq; i++) r->offsets[i + 1] = r->offsets[i] + (int64_t)S.answers[i].size();
            r->ids.reserve(r->offsets[nq]);
            for (int64_t i = 0; i < nq; i++) r->ids.insert(r->ids.end(), S.answers[i].begin(), S.answers[i].end());
            std::vector<double> l(nq);
            double wall = 0.0;
            for (int64_t i = 0; i < nq; i++) {
                l[i] = S.t_done[i] - S.t_arrive[i];
                lat[i] = l[i];
                wall = std::max(wall, S.t_done[i]);
            }
            r->st.results = r->offsets[nq];
            if (stats) {
                std::memset(stats, 0, sizeof *stats);
                stats->batches = S.batches;
                stats->max_inflight = S.max_inflight;
                stats->slots = nslots;
                stats->wall_ms = (wall - (nq ? S.t_arrive[0] : 0.0)) * 1e-3;
                if (nq) {
                    std::vector<double> sl = l;
                    std::sort(sl.begin(), sl.end());
                    auto pct = [&](double p) { return sl[std::min<int64_t>(nq - 1, (int64_t)(p * (nq - 1) + 0.5))]; };
                    stats->p50_us = pct(0.50);
                    stats->p99_us = pct(0.99);
                    double sum = 0;
                    for (double v : sl) sum += v;
                    stats->mean_us = sum / nq;
                }
            }
            *out = r.release();
    });
}
