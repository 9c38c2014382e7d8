// Caching allocator for the library's device and pinned host buffers.
//
// Building an index and answering a batch need a few dozen buffers each; hipMalloc /
// hipFree of them (hipFree also waits for the whole device) cost milliseconds per call
// sequence.  Released blocks are kept per device in size classes (eight per power of
// two) and handed out again:
//   * a block released by code running under a StreamScope carries an event recorded
//     on that stream at release time; handing it out on another stream makes that
//     stream wait for the event on the device (the host never blocks);
//   * a block released inside an IdleScope (the device was synchronised first) is free
//     for any stream at once.
// Blocks released with no scope at all are returned to the runtime with hipFree.
// Cached bytes are capped (RKMIPS_CACHE_MB, default 1/4 of the device memory, at most
// 64 GiB); the oldest blocks are returned first, after their event has completed.  An
// allocation that fails empties the cache and is tried once more.
//
// Pinned host blocks are cached the same way, without events: they are released only
// when no copy that uses them can be pending.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rk::mem {

// Device block of at least `bytes`, for use on the current scope's stream.
void* device_alloc(size_t bytes, size_t* granted);
// Returns a block of `bytes` (the size it was requested with) to the cache.
void device_free(void* p, size_t bytes);

void* host_alloc(size_t bytes, size_t* granted);
void host_free(void* p, size_t bytes);

// Empties both caches (device work is waited for first).
void trim();

// The stream that buffers allocated and released on this thread belong to.
struct StreamScope {
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
    StreamScope(const StreamScope&) = delete;
    StreamScope& operator=(const StreamScope&) = delete;
private:
    hipStream_t prev_;
    bool prev_set_;
};

// Releases on this thread happen after a device synchronisation.
struct IdleScope {
    IdleScope();
    ~IdleScope();
    IdleScope(const IdleScope&) = delete;
    IdleScope& operator=(const IdleScope&) = delete;
};

// IdleScope without the RAII shape, for objects that release members after their
// destructor body has run.
void idle_enter();
void idle_leave();

hipStream_t current_stream(bool* set);
bool idle();

}  // namespace rk::mem
