// Caching device-memory arena of one context: planning scratch and library-
// owned outputs are served from blocks kept after earlier calls, so that a
// query in a serving loop pays no allocator round trips once warm. Blocks
// come from, and go back to, the device's stream-ordered memory pool.
//
// Blocks are handed out with stream-ordered semantics: a block given back on
// stream S may be reused by later work on S at once; reuse by another stream
// waits (hipStreamWaitEvent) for an event recorded on S when the block was
// given back. Blocks given back as idle (no pending device work) carry no
// event. Thread-safe.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace slg {

class Arena {
  public:
    Arena(int device, uint64_t cache_limit);
    ~Arena();
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;

    // A block of at least `bytes` usable by work on `st`.
    hipError_t get(void **p, size_t bytes, hipStream_t st);
    // Gives blocks back after the work already queued on `st` (one event
    // for the whole set); st == nullptr with idle == true: no pending work.
    void put(const std::vector<void *> &blocks, hipStream_t st, bool idle = false);
    // Frees every cached block (waiting for their events first).
    void trim();
    uint64_t cached_bytes();

  private:
    struct Event {
        hipEvent_t e = nullptr;
        ~Event();
    };
    struct Free {
        void *p;
        size_t size;
        hipStream_t st;
        bool idle;
        std::shared_ptr<Event> ev;
    };
    static size_t size_class(size_t bytes);
    void release_locked(std::multimap<size_t, Free>::iterator it);
    void shrink_locked(uint64_t target);

    std::mutex mu_;
    int device_;
    hipStream_t free_st_ = nullptr;  // frees of cached blocks (made at the first)
    uint64_t limit_;
    uint64_t cached_ = 0;
    std::multimap<size_t, Free> free_;
    std::unordered_map<void *, size_t> live_;
};

}  // namespace slg
