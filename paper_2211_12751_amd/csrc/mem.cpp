// Caching allocator: see mem.h.
#include "mem.h"

#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

namespace rk::mem {

namespace {

struct Block {
    void* p;
    size_t bytes;
    hipStream_t stream;
    hipEvent_t ev;     // null: free for any stream
    uint64_t seq;
};

struct Cache {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, Block> dev;   // (device, class) -> block
    std::multimap<size_t, void*> host;
    std::vector<hipEvent_t> events;
    std::map<int, size_t> dev_cached, dev_cap;
    size_t host_cached = 0;
    uint64_t seq = 0;
};

// never destroyed: blocks outlive static destruction, the runtime reclaims them
Cache& cache()
{
    static Cache* c = new Cache;
    return *c;
}

thread_local hipStream_t t_stream = nullptr;
thread_local bool t_stream_set = false;
thread_local int t_idle = 0;

constexpr size_t kHostCap = size_t(1) << 30;

size_t size_class(size_t b)
{
    if (b <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)b);
    const size_t step = size_t(1) << (e - 3);
    return (b + step - 1) / step * step;
}

size_t device_cap(Cache& c, int dev)
{
    auto it = c.dev_cap.find(dev);
    if (it != c.dev_cap.end()) return it->second;
    // an index build over a million items and a few million users cycles through about
    // 40 GB of buffers: below that, every build would give blocks back with hipFree and
    // allocate them again
    size_t cap = size_t(64) << 30;
    if (const char* s = std::getenv("RKMIPS_CACHE_MB")) {
        cap = (size_t)std::strtoull(s, nullptr, 10) << 20;
    } else {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
            if (tot / 4 < cap) cap = tot / 4;
        } else {
            (void)hipGetLastError();
        }
    }
    c.dev_cap[dev] = cap;
    return cap;
}

hipEvent_t take_event(Cache& c)
{
    if (!c.events.empty()) {
        hipEvent_t e = c.events.back();
        c.events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Returns a cached block to the runtime (its last use has to be complete).
void release_block(Cache& c, Block& b)
{
    if (b.ev) {
        (void)hipEventSynchronize(b.ev);
        c.events.push_back(b.ev);
    }
    (void)hipFree(b.p);
}

void evict_locked(Cache& c, int dev, size_t cap)
{
    while (c.dev_cached[dev] > cap) {
        auto oldest = c.dev.end();
        for (auto it = c.dev.begin(); it != c.dev.end(); ++it)
            if (it->first.first == dev && (oldest == c.dev.end() || it->second.seq < oldest->second.seq)) oldest = it;
        if (oldest == c.dev.end()) break;
        c.dev_cached[dev] -= oldest->second.bytes;
        release_block(c, oldest->second);
        c.dev.erase(oldest);
    }
}

void trim_device_locked(Cache& c)
{
    for (auto& kv : c.dev) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (kv.first.first != cur) (void)hipSetDevice(kv.first.first);
        release_block(c, kv.second);
        if (kv.first.first != cur) (void)hipSetDevice(cur);
    }
    c.dev.clear();
    c.dev_cached.clear();
}

}  // namespace

void* device_alloc(size_t bytes, size_t* granted)
{
    Cache& c = cache();
    const hipStream_t stream = t_stream;
    const size_t cls = size_class(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto range = c.dev.equal_range({dev, cls});
        auto pick = c.dev.end();
        for (auto it = range.first; it != range.second; ++it) {
            if (pick == c.dev.end()) pick = it;
            if (!it->second.ev || it->second.stream == stream) { pick = it; break; }
        }
        if (pick != c.dev.end()) {
            Block b = pick->second;
            c.dev.erase(pick);
            c.dev_cached[dev] -= cls;
            if (b.ev) {
                // a block last used on another stream is ready once that stream passes
                // the release point
                if (b.stream != stream || !t_stream_set) {
                    // with no scope the block may be used on any stream: wait on the host
                    if (!t_stream_set || hipStreamWaitEvent(stream, b.ev, 0) != hipSuccess) {
                        (void)hipGetLastError();
                        (void)hipEventSynchronize(b.ev);
                    }
                }
                c.events.push_back(b.ev);
            }
            if (granted) *granted = cls;
            return b.p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, cls) != hipSuccess) {
        (void)hipGetLastError();
        trim();
        if (hipMalloc(&p, cls) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    if (granted) *granted = cls;
    return p;
}

void device_free(void* p, size_t bytes)
{
    if (!p) return;
    Cache& c = cache();
    const size_t cls = size_class(bytes);
    if (!t_idle && !t_stream_set) {
        (void)hipFree(p);
        return;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(c.mu);
    Block b{p, cls, t_stream, nullptr, ++c.seq};
    if (!t_idle) {
        b.ev = take_event(c);
        if (!b.ev || hipEventRecord(b.ev, t_stream) != hipSuccess) {
            (void)hipGetLastError();
            if (b.ev) c.events.push_back(b.ev);
            (void)hipStreamSynchronize(t_stream);
            b.ev = nullptr;
        }
    }
    c.dev.emplace(std::make_pair(dev, cls), b);
    c.dev_cached[dev] += cls;
    evict_locked(c, dev, device_cap(c, dev));
}

void* host_alloc(size_t bytes, size_t* granted)
{
    Cache& c = cache();
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.host.find(cls);
        if (it != c.host.end()) {
            void* p = it->second;
            c.host.erase(it);
            c.host_cached -= cls;
            if (granted) *granted = cls;
            return p;
        }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (granted) *granted = cls;
    return p;
}

void host_free(void* p, size_t bytes)
{
    if (!p) return;
    Cache& c = cache();
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> g(c.mu);
    if (c.host_cached + cls > kHostCap) {
        (void)hipHostFree(p);
        return;
    }
    c.host.emplace(cls, p);
    c.host_cached += cls;
}

void trim()
{
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    trim_device_locked(c);
    for (auto& kv : c.host) (void)hipHostFree(kv.second);
    c.host.clear();
    c.host_cached = 0;
}

StreamScope::StreamScope(hipStream_t s) : prev_(t_stream), prev_set_(t_stream_set)
{
    t_stream = s;
    t_stream_set = true;
}

StreamScope::~StreamScope()
{
    t_stream = prev_;
    t_stream_set = prev_set_;
}

IdleScope::IdleScope() { ++t_idle; }
IdleScope::~IdleScope() { --t_idle; }
void idle_enter() { ++t_idle; }
void idle_leave() { --t_idle; }

hipStream_t current_stream(bool* set)
{
    if (set) *set = t_stream_set;
    return t_stream;
}

bool idle() { return t_idle > 0; }

}  // namespace rk::mem
