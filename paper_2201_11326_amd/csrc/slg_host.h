// Host-side internals shared by the API (slg_api.cpp) and the request
// server (slg_server.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <functional>
#include <memory>
#include <mutex>

#include "slg.h"

namespace slg {

class Arena;

// Device-memory ledger of one server. Results handed to the caller keep it
// (and the arena their buffers came from) alive, so that they can be freed
// after the server.
struct ServeCore {
    std::mutex mu;
    std::condition_variable cv;  // memory released / request state changed
    uint64_t budget = 0;         // 0 = no limit
    uint64_t used = 0, peak = 0;
    uint64_t held_by_results = 0;

    void release(uint64_t bytes, bool from_result) {
        std::lock_guard<std::mutex> lk(mu);
        used -= bytes;
        if (from_result) held_by_results -= bytes;
        cv.notify_all();
    }
};

// Grants `bytes` of device memory (true) or refuses them (false); the
// caller keeps the reason for a refusal.
using ReserveFn = std::function<bool(uint64_t bytes)>;

// One query of the served form: plans `g` for the s-set on `st` with the
// worker context `wctx`, calling `reserve` with the device bytes of each
// allocation phase before it is made (planning scratch in two phases, then
// the outputs), emits, releases the planning scratch and waits for `st`.
// On success *out owns the outputs, which are accounted to `core`;
// *scratch_bytes is what the planning phases reserved (now free again),
// *output_bytes what the result holds. A refused reservation ends the query
// with SLG_ERR_OUT_OF_MEMORY. Any error leaves nothing allocated; the
// reservations granted so far are reported in *scratch_bytes /
// *output_bytes for the caller to give back.
slg_status serve_query(slg_context *wctx, slg_graph *g, const int32_t *s, int32_t num_s, hipStream_t st,
                       const ReserveFn &reserve, const std::shared_ptr<ServeCore> &core, slg_result **out,
                       uint64_t *scratch_bytes, uint64_t *output_bytes);

// Device of a context / a registered graph's context.
int context_device(const slg_context *ctx);
const slg_context *graph_context(const slg_graph *g);
slg_status set_error(slg_context *ctx, slg_status code, const char *msg);
// slg_context_create, with the choice of the context's second stream (on
// which a large plan's light counting pass runs beside the heavy tier's
// planning). A server's slots go without it: they already overlap whole
// queries, and a second stream per slot only adds streams to share the
// hardware queues.
slg_status create_context(int device, uint64_t mem_budget_bytes, const slg_allocator *alloc, bool second_stream,
                          slg_context **out);
// Copies the plan-shape tuning (slg_context_set_tuning) of `src` to `dst`.
void copy_tuning(slg_context *dst, const slg_context *src);
// Makes `ctx` take its scratch and outputs from `arena` (shared by a
// server's slots).
void share_arena(slg_context *ctx, const std::shared_ptr<Arena> &arena);

}  // namespace slg
