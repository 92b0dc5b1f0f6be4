// ht_workspace.hpp -- per (device, stream) device workspace cache.
//
// A call takes one contiguous device buffer.  The cache keeps the largest
// buffer requested so far for each (device, stream) pair; growing it first
// synchronises that stream (work already enqueued may still use the old
// buffer), then frees and reallocates.  Buffers live until
// ht_release_workspace() or process exit.
#pragma once
#include <hip/hip_runtime.h>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>

namespace ht {

// ------------------------------------------------------------------ knobs
// Process-wide settings (ht_set_knob / ht_get_knob).  Index = HT_KNOB_* - 1.
constexpr int kNumKnobs = 3;
inline std::atomic<int64_t> *knobs()
{
    static std::atomic<int64_t> k[kNumKnobs] = {
        {int64_t(1) << 22},   // HT_KNOB_WAIT_POLLS: polls before a device-side wait gives up
        {0},                  // HT_KNOB_UPDATE_TILE_ROWS: 0 automatic, 1 or 2 tiles of 16 rows per wavefront
        {1},                  // HT_KNOB_LOOKAHEAD: 0 never, 1 from n = 1024 on, 2 always
    };
    return k;
}
inline int64_t knob(int id) { return knobs()[id - 1].load(std::memory_order_relaxed); }

// ------------------------------------------------------------ status word
// One device int per (device, stream): kernels OR failure bits into it (a
// bounded wait that gave up); ht_stream_status() reads and clears it.  Also a
// pinned host int that receives the value.
struct StatusEntry { int *dev = nullptr; int *host = nullptr; };

inline std::map<std::pair<int, hipStream_t>, StatusEntry> &status_map()
{
    static std::map<std::pair<int, hipStream_t>, StatusEntry> m;
    return m;
}

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

// The status word of (current device, stream), created (zeroed, stream
// ordered) on first use; nullptr on failure.
inline StatusEntry *status_get(hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(ws_mutex());
    StatusEntry &e = status_map()[{dev, st}];
    if (e.dev) return &e;
    if (hipMalloc(&e.dev, 256) != hipSuccess) { (void)hipGetLastError(); e.dev = nullptr; return nullptr; }
    if (hipHostMalloc(&e.host, 256, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError(); (void)hipFree(e.dev); e.dev = nullptr; e.host = nullptr; return nullptr;
    }
    *e.host = 0;
    if (hipMemcpyAsync(e.dev, e.host, sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipFree(e.dev); (void)hipHostFree(e.host); e.dev = nullptr; e.host = nullptr; return nullptr;
    }
    return &e;
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


