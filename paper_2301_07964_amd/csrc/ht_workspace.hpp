// ht_workspace.hpp -- per (device, stream) device workspace cache.
//
// A call takes one contiguous device buffer.  The cache keeps the largest
// buffer requested so far for each (device, stream) pair; growing it first
// synchronises that stream (work already enqueued may still use the old
// buffer), then frees and reallocates.  Buffers live until
// ht_release_workspace() or process exit.
#pragma once
#include <hip/hip_runtime.h>
#include <map>
#include <mutex>
#include <utility>

namespace ht {

struct WsEntry { void *ptr = nullptr; size_t size = 0; };

inline std::mutex &ws_mutex() { static std::mutex m; return m; }
inline std::map<std::pair<int, hipStream_t>, WsEntry> &ws_map()
{
    static std::map<std::pair<int, hipStream_t>, WsEntry> m;
    return m;
}

// Returns a device pointer of at least `bytes` bytes, or nullptr with *rc set.
inline void *workspace_get(size_t bytes, hipStream_t st, int *rc)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { *rc = 1; return nullptr; }
    std::lock_guard<std::mutex> lk(ws_mutex());
    WsEntry &e = ws_map()[{dev, st}];
    if (e.size >= bytes && e.ptr) return e.ptr;
    if (e.ptr) {
        if (hipStreamSynchronize(st) != hipSuccess) { *rc = 1; return nullptr; }
        (void)hipFree(e.ptr);
        e.ptr = nullptr; e.size = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) { (void)hipGetLastError(); *rc = 2; return nullptr; }
    e.ptr = p; e.size = bytes;
    return p;
}

// Grows the (current device, stream) buffer to at least `bytes` now, so that
// later calls on that stream whose workspace fits never allocate or synchronise.
inline int workspace_reserve(size_t bytes, hipStream_t st)
{
    int rc = 0;
    return workspace_get(bytes, st, &rc) ? 0 : rc;
}

// Pinned host staging per (device, stream) for small host-to-device copies
// (batched descriptors).  Before the buffer is rewritten, the host waits for
// the copy that last read it (an event on that stream), not for the stream.
struct PinnedEntry { void *ptr = nullptr; size_t size = 0; hipEvent_t done = nullptr; bool pending = false; };

inline std::map<std::pair<int, hipStream_t>, PinnedEntry> &pinned_map()
{
    static std::map<std::pair<int, hipStream_t>, PinnedEntry> m;
    return m;
}

// Returns the staging buffer (>= bytes) with its last copy finished, or nullptr.
inline PinnedEntry *pinned_get(size_t bytes, hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(ws_mutex());
    PinnedEntry &e = pinned_map()[{dev, st}];
    if (!e.done && hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (e.pending) {
        if (hipEventSynchronize(e.done) != hipSuccess) return nullptr;
        e.pending = false;
    }
    if (e.size < bytes) {
        if (e.ptr) (void)hipHostFree(e.ptr);
        e.ptr = nullptr; e.size = 0;
        if (hipHostMalloc(&e.ptr, bytes, hipHostMallocDefault) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        e.size = bytes;
    }
    return &e;
}

inline void workspace_release_all_current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(ws_mutex());
    auto &m = ws_map();
    for (auto it = m.begin(); it != m.end();) {
        if (it->first.first == dev) {
            if (it->second.ptr) {
                (void)hipStreamSynchronize(it->first.second);
                (void)hipFree(it->second.ptr);
            }
            it = m.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace ht


