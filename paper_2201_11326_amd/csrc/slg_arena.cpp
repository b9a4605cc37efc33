#include "slg_arena.h"

#include <algorithm>

namespace slg {

Arena::Event::~Event() {
    if (e) (void)hipEventDestroy(e);
}

Arena::Arena(int device, uint64_t cache_limit) : device_(device), limit_(cache_limit) {}

Arena::~Arena() {
    trim();
    if (free_st_) {
        (void)hipStreamSynchronize(free_st_);
        (void)hipStreamDestroy(free_st_);
    }
    (void)hipGetLastError();  // nothing of the teardown reaches a later call's error check
}

// 256 B granules up to 4 KiB, then four classes per power of two (at most
// 25% slack).
size_t Arena::size_class(size_t bytes) {
    if (bytes <= 4096) return std::max<size_t>((bytes + 255) & ~size_t(255), 256);
    size_t p = 4096;
    while (p * 2 < bytes) p *= 2;  // p < bytes <= 2p
    const size_t q = p / 4;
    return ((bytes + q - 1) / q) * q;
}

hipError_t Arena::get(void **p, size_t bytes, hipStream_t st) {
    *p = nullptr;
    const size_t want = size_class(bytes ? bytes : 1);
    {
        std::lock_guard<std::mutex> lk(mu_);
        // smallest cached block that fits without wasting more than half
        auto lo = free_.lower_bound(want), hi = free_.upper_bound(want * 2);
        auto pick = free_.end();
        for (auto it = lo; it != hi; ++it) {
            if (it->second.idle || it->second.st == st) {  // no wait needed
                pick = it;
                break;
            }
            if (pick == free_.end()) pick = it;
        }
        if (pick != free_.end()) {
            Free f = pick->second;
            free_.erase(pick);
            cached_ -= f.size;
            live_[f.p] = f.size;
            if (!f.idle && f.st != st && f.ev) {
                hipError_t e = hipStreamWaitEvent(st, f.ev->e, 0);
                if (e != hipSuccess) return e;
            }
            *p = f.p;
            return hipSuccess;
        }
    }
    // blocks come from the device's stream-ordered pool (it keeps freed
    // memory, so giving a block back and allocating again costs no device
    // synchronisation and no new mapping)
    hipError_t e = hipMallocAsync(p, want, st);
    if (e == hipErrorOutOfMemory) {  // give the cache back and try once more
        (void)hipGetLastError();
        trim();
        e = hipMallocAsync(p, want, st);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    std::lock_guard<std::mutex> lk(mu_);
    live_[*p] = want;
    return hipSuccess;
}

void Arena::put(const std::vector<void *> &blocks, hipStream_t st, bool idle) {
    if (blocks.empty()) return;
    std::shared_ptr<Event> ev;
    if (!idle) {
        ev = std::make_shared<Event>();
        if (hipEventCreateWithFlags(&ev->e, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev->e, st) != hipSuccess) {
            // cannot mark the point in the stream: wait for it instead
            (void)hipStreamSynchronize(st);
            (void)hipGetLastError();
            idle = true;
            ev.reset();
        }
    }
    std::lock_guard<std::mutex> lk(mu_);
    for (void *p : blocks) {
        auto it = live_.find(p);
        if (it == live_.end()) continue;  // not ours
        const size_t size = it->second;
        live_.erase(it);
        free_.insert({size, Free{p, size, st, idle, ev}});
        cached_ += size;
    }
    if (cached_ > limit_) shrink_locked(limit_ / 4 * 3);  // some room below the limit, not a full flush
}

// The block's own pending work is waited for on the host (its event, not the
// whole device), then it goes back to the pool on the arena's own stream
// (the stream it was given back on may be gone by now, and the legacy null
// stream would order the free after every other stream's work). Errors are
// dropped here and cleared, so that they do not surface in a later,
// unrelated launch check; a block whose free fails is freed synchronously.
void Arena::release_locked(std::multimap<size_t, Free>::iterator it) {
    if (it->second.ev) (void)hipEventSynchronize(it->second.ev->e);
    if (!free_st_ && hipStreamCreateWithFlags(&free_st_, hipStreamNonBlocking) != hipSuccess) free_st_ = nullptr;
    if (hipFreeAsync(it->second.p, free_st_) != hipSuccess) (void)hipFree(it->second.p);
    (void)hipGetLastError();
    cached_ -= it->second.size;
    free_.erase(it);
}

// Frees the largest cached blocks until at most `target` bytes stay cached.
void Arena::shrink_locked(uint64_t target) {
    (void)hipSetDevice(device_);
    while (cached_ > target && !free_.empty()) release_locked(std::prev(free_.end()));
}

void Arena::trim() {
    std::lock_guard<std::mutex> lk(mu_);
    shrink_locked(0);
}

uint64_t Arena::cached_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return cached_;
}

}  // namespace slg
