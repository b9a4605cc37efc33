// Host side of the C ABI declared in include/slg.h: contexts, graph
// registration and validation, the plan (prune -> work estimate -> count ->
// prefix sums), the emit pass and the one-shot result object.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "slg.h"
#include "slg_arena.h"
#include "slg_host.h"
#include "slg_internal.h"

using namespace slg;

namespace {
enum Stage {
    kStPrune, kStRowPlan, kStPlanScans, kStSlots, kStBounds, kStCountLight, kStCountHeavy,
    kStCountHeavyWide, kStCountDense, kStCountScans, kStEmitLight, kStEmitHeavy, kStEmitHeavyWide, kStEmitDense,
    kStRowPtr, kNumStages
};
const char *const kStageNames[kNumStages] = {
    "prune", "row_plan", "plan_scans", "slots", "bounds", "count_light", "count_heavy",
    "count_heavy_wide", "count_dense", "count_scans", "emit_light", "emit_heavy", "emit_heavy_wide", "emit_dense",
    "row_ptr"};
struct PendingTime {
    int stage;
    hipEvent_t start, stop;
};
// Work counters of a context, summed over every counting pass (whole plans
// and row blocks) since the last reset.
enum Work {
    kWkBlocks, kWkTwoPaths, kWkHeavyTwoPaths, kWkDenseTwoPaths, kWkEdges, kWkHeavyEdges, kWkDenseEdges,
    kWkDenseSlots, kWkDenseStored, kWkDenseRewalk, kNumWork
};
}  // namespace

struct slg_context {
    int device = 0;
    int heavy_resident = 0;  // persistent workgroups of the heavy tier
    bool timing = false;
    std::vector<PendingTime> pending;
    std::vector<hipEvent_t> event_pool;
    int64_t stage_launches[kNumStages] = {};
    double stage_ms[kNumStages] = {};
    int64_t work[kNumWork] = {};  // work counters since the last reset (slg_context_get_work)
    bool capturing = false;  // a hipGraph capture is recording: no event timing
    int32_t light_max = kLightMax;
    int64_t slot_work = kSlotWork;
    int heavy_grid = 0;
    int dense_resident = 0;  // persistent workgroups of the dense tier
    int32_t dense_ratio = kDenseRatio;  // the dense tier's rule (ratio 0: off)
    int32_t dense_min = kDenseMinRange;
    int64_t store_limit = int64_t(32) << 30;  // largest count store a plan keeps (0: none)
    int64_t store_min = int64_t(1) << 24;     // fewest heavy 2-paths for which a plan keeps one
    int64_t list_shortfall = 0;  // error-path tests: heavy lists planned this much short
    uint64_t budget = 0;
    bool has_alloc = false;
    slg_allocator alloc{};
    std::string last_error;
    int64_t *pinned = nullptr;  // host staging for readbacks
    // second stream: the light tier's counting pass beside the heavy
    // planning, made at the first plan large enough to fork
    bool aux_allowed = true;
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    std::shared_ptr<slg::Arena> arena;  // scratch and library-owned outputs
    void *noalloc = nullptr;            // this device's fixed scratch array (slg_components_noalloc)
    hipError_t noalloc_err = hipSuccess;
};

struct slg_graph {
    slg_context *ctx = nullptr;
    slg_incidence inc{};
    std::vector<void *> owned;  // SLG_COPY: the graph's own copies of the CSRs
};

namespace {

constexpr int kPinnedSlots = 96;

// Layout of the plan's small device counter block (int64 entries).
constexpr int kCntClass = 0;                    // kNumLists: rows / slots per tier list
constexpr int kCntErr = kCntClass + kNumLists;  // malformed-input flag (low 32 bits)
constexpr int kCntFill = kCntErr + 1;           // kNumLists: append cursors of the tier lists
constexpr int kCntHeavyWork = kCntFill + kNumLists;  // 2-paths in heavy rows
constexpr int kCntPieces = kCntHeavyWork + 1;     // large-row pieces of row planning
constexpr int kCntDenseWork = kCntPieces + 1;     // 2-paths in dense rows
constexpr int kCntTotal = kCntDenseWork + 1;
static_assert(kCntTotal <= 32, "counter block");
// Host staging slots for readbacks.
constexpr int kHbSlots = kCntTotal;      // slot table size, then 2-paths, boundary entries
constexpr int kHbEdges = 40;             // SLG_MAX_S edge totals
constexpr int kHbHeavyEdges = kHbEdges + SLG_MAX_S;
constexpr int kHbRange = kHbHeavyEdges + 7;  // a chunk's heavy list ranges (2 per list)
static_assert(kHbSlots + 3 <= kHbEdges && kHbRange + 2 * kNumHeavyLists <= kPinnedSlots, "pinned staging layout");
// Device counters of a plan (int64 entries of `tickets`).
constexpr int kTkCount = 0;       // kNumHeavyLists: slot tickets of the counting passes
constexpr int kTkEmit = 3;        // kNumHeavyLists: slot tickets of the emit passes
constexpr int kTkHeavyEdges = 6;  // edges of heavy and heavy-wide slots
constexpr int kTkStored = 7;      // entries of the heavy count store
constexpr int kTkDenseCursor = 8; // room taken from the dense store (in chunks)
constexpr int kTkDenseAsked = 9;  // survivors the dense slots asked the store to keep
constexpr int kTkDenseKept = 10;  // ... and those it kept (fewer: some slots walk again)
constexpr int kTkDenseEdges = 11; // edges of dense slots
constexpr int kTkRange = 12;      // 2 per heavy list: a chunk's part of it
constexpr int kTkTotal = kTkRange + 2 * kNumHeavyLists;
static_assert(kTkHeavyEdges + 1 == kTkStored && kTkStored + 1 == kTkDenseCursor &&
                  kTkDenseCursor + 1 == kTkDenseAsked && kTkDenseAsked + 1 == kTkDenseKept &&
                  kTkDenseKept + 1 == kTkDenseEdges,
              "plan counters read back together; the dense kernel takes cursor, asked, kept in a row");

// Freed device blocks a context keeps for reuse unless told otherwise.
constexpr uint64_t kDefaultCacheMin = uint64_t(16) << 30;  // default block cache: half of the
                                                           // device's memory, at least this

slg_status fail(slg_context *ctx, slg_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return st;
}

#define SLG_HIP(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            return fail((ctx), e_ == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE, \
                        "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__);     \
        }                                                                                        \
    } while (0)

// Stream-ordered scratch owned by a plan.
struct Scratch {
    hipStream_t st = nullptr;
    slg::Arena *arena = nullptr;
    std::vector<void *> ptrs;
    Scratch() = default;
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    ~Scratch() { release(); }  // an early error return gives the blocks back too
    hipError_t get(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 8;
        hipError_t e = arena->get(p, bytes, st);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    template <typename T>
    hipError_t get(T **p, size_t count) {
        return get(reinterpret_cast<void **>(p), count * sizeof(T));
    }
    void release() {  // after the work already queued on st
        if (arena) arena->put(ptrs, st);
        ptrs.clear();
    }
};

// Allocations of one planning phase, summed before any is made so that a
// budget can be asked for them at once.
struct AllocList {
    std::vector<std::pair<void **, size_t>> items;
    uint64_t bytes = 0;
    template <typename T>
    void add(T **p, size_t count) {
        const size_t b = std::max<size_t>(count * sizeof(T), 8);
        items.push_back({reinterpret_cast<void **>(p), b});
        bytes += b;
    }
};

// Brackets the launches of one stage with events on their stream when the
// context's timing is on.
struct StageTimer {
    slg_context *ctx;
    int stage;
    hipStream_t st;
    hipEvent_t start = nullptr, stop = nullptr;
    StageTimer(slg_context *c, int sg, hipStream_t s) : ctx(c), stage(sg), st(s) {
        if (!ctx || !ctx->timing || ctx->capturing) return;
        start = take();
        stop = take();
        if (start && stop) (void)hipEventRecord(start, st);
    }
    ~StageTimer() {
        if (start && stop) {
            (void)hipEventRecord(stop, st);
            ctx->pending.push_back({stage, start, stop});
        }
    }
    hipEvent_t take() {
        if (!ctx->event_pool.empty()) {
            hipEvent_t e = ctx->event_pool.back();
            ctx->event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
};

bool valid_s(const int32_t *s, int32_t k) {
    if (!s || k < 1 || k > SLG_MAX_S || s[0] < 1) return false;
    for (int32_t t = 1; t < k; ++t)
        if (s[t] <= s[t - 1]) return false;
    return true;
}

// Stable sort of n int32 keys in [0, 2^key_bits) with up to two payloads
// (b only with a), from the *_in arrays into the *_out arrays (which may be
// caller memory), through scratch from `sc` when more than one digit pass is
// needed. With key_bits = 0 the inputs are copied. With `in_scratch`, the
// outputs are not given: the last pass writes scratch too (two buffers per
// array in all) and *_out receive where the sorted arrays are.
hipError_t sort_pairs(Scratch &sc, const int32_t *key_in, const int32_t *a_in, const int32_t *b_in, int64_t n,
                      int key_bits, int32_t *key_out, int32_t *a_out, int32_t *b_out, hipStream_t st,
                      const int32_t **in_scratch = nullptr) {
    if (n <= 0) return hipSuccess;
    const int passes = sort_passes(key_bits);
    hipError_t e;
    if (in_scratch && passes == 0) {  // already in order: the inputs themselves
        in_scratch[0] = key_in;
        in_scratch[1] = a_in;
        in_scratch[2] = b_in;
        return hipSuccess;
    }
    if (passes == 0) {
        const int32_t *src[3] = {key_in, a_in, b_in};
        int32_t *dst[3] = {key_out, a_out, b_out};
        for (int t = 0; t < 3; ++t)
            if (src[t] && dst[t] && src[t] != dst[t] &&
                (e = hipMemcpyAsync(dst[t], src[t], n * sizeof(int32_t), hipMemcpyDeviceToDevice, st)) != hipSuccess)
                return e;
        return hipSuccess;
    }
    const int digit = (key_bits + passes - 1) / passes;
    const int64_t hist_n = (int64_t(1) << digit) * sort_chunks(n);
    int32_t *hist = nullptr, *tmp[2][3] = {};
    int64_t *off = nullptr, *part = nullptr;
    if ((e = sc.get(&hist, hist_n)) != hipSuccess || (e = sc.get(&off, hist_n + 1)) != hipSuccess ||
        (e = sc.get(&part, scan_partials_size(hist_n))) != hipSuccess)
        return e;
    const int arrays = b_in ? 3 : (a_in ? 2 : 1);
    // pass p writes tmp[p & 1] except the last, which writes the outputs
    // (or tmp as well, with in_scratch)
    const int bufs = in_scratch ? (passes > 1 ? 2 : 1) : (passes > 2 ? 2 : passes - 1);
    for (int h = 0; h < bufs; ++h)
        for (int t = 0; t < arrays; ++t)
            if ((e = sc.get(&tmp[h][t], n)) != hipSuccess) return e;
    const int32_t *k = key_in, *a = a_in, *b = b_in;
    for (int p = 0; p < passes; ++p) {
        const bool last = p + 1 == passes && !in_scratch;
        int32_t *ko = last ? key_out : tmp[p & 1][0];
        int32_t *ao = a_in ? (last ? a_out : tmp[p & 1][1]) : nullptr;
        int32_t *bo = b_in ? (last ? b_out : tmp[p & 1][2]) : nullptr;
        const int shift = p * digit;
        if ((e = launch_sort_pass(k, a, b, n, shift, std::min(digit, key_bits - shift), hist, off, part, ko, ao, bo,
                                  st)) != hipSuccess)
            return e;
        k = ko;
        a = ao;
        b = bo;
    }
    if (in_scratch) {
        in_scratch[0] = k;
        in_scratch[1] = a;
        in_scratch[2] = b;
    }
    return hipSuccess;
}

int bits_for(int64_t values) {  // bits of the largest value below `values`
    int b = 0;
    while ((int64_t(1) << b) < values) ++b;
    return b;
}

}  // namespace

// Device buffers of a plan, kept so the planning launches can be replayed.
struct PlanBufs {
    uint8_t *flag = nullptr;
    int64_t *pos = nullptr, *part_nnz = nullptr, *vs_ptr = nullptr;
    int32_t *vs_idx = nullptr;
    int32_t *tail_beg = nullptr, *jmax = nullptr, *nslots = nullptr, *slot_row = nullptr;
    int64_t *work = nullptr, *work_pre = nullptr, *counters = nullptr, *part_m = nullptr;
    int64_t *bsize = nullptr, *bbase = nullptr, *hat = nullptr, *part_s = nullptr;
    int32_t *hcnt = nullptr;
    int64_t *pieces = nullptr;
    uint8_t *rclass = nullptr;
    int32_t *nslots_all = nullptr;  // row blocks: every row's slots, class and boundary
    uint8_t *rclass_all = nullptr;  // entries, kept while each block masks the
    int64_t *bsize_all = nullptr;   // others out
    uint8_t *keep = nullptr;     // E_s positions (dense tier): kept-row flags,
    int64_t *kpre = nullptr;     // their exclusive scan,
    int32_t *cid = nullptr, *cid_row = nullptr, *vs_cid = nullptr;  // ranks, rows of ranks, lists in ranks
    uint16_t *vs_win = nullptr;  // the lists' ranks modulo the dense window
};

struct slg_plan {
    slg_context *ctx = nullptr;
    slg_graph *g = nullptr;
    hipStream_t st = nullptr;
    EmitParams prm{};
    Pruned pr{};
    Scratch scratch;   // the rows phase: kept for the plan's life
    Scratch scratch2;  // a row block's slot tables, lists, stores (released per block)
    PlanBufs b;
    bool blocks = false;           // planned block by block (the rows phase keeps every row's facts)
    uint32_t *dstore_fixed = nullptr;  // row blocks: one dense store for every block
    int64_t dstore_fixed_cap = 0;
    int64_t row_lo = 0, row_hi = 0;  // the rows of the current block
    bool prune = false;            // vertex lists are compacted to E_{s_min}
    int32_t s_min = 1;
    int32_t light_max = kLightMax; // tuning: wavefront-sort tier bound
    int64_t slot_work = kSlotWork; // tuning: 2-paths per heavy slot
    int heavy_grid = 0;            // tuning: persistent heavy workgroups
    int64_t *slot_base = nullptr;  // [m+1]
    int64_t S = 0;                 // number of slots
    Slots slots{};
    int32_t *bounds = nullptr;
    int64_t *tickets = nullptr;    // work counters of the persistent heavy launches
    HeavyDesc *heavy[kNumHeavyLists] = {};  // heavy, heavy-wide and dense slot descriptors
    int32_t *lists[kNumLists] = {};
    int64_t list_count[kNumLists] = {};
    int64_t *slot_cnt = nullptr;   // [K][S]
    int64_t *slot_off = nullptr;   // [K][S+1]
    bool dense = false;            // rows may take the dense tier (E_s positions computed)
    int32_t dense_ratio = 0, dense_min = 0;
    int dense_grid = 0;
    bool use_dstore = false;       // dense slots keep their survivors for the emit pass
    CountStore dstore{};
    int64_t dstore_cap = 0;        // entries of the dense store
    int64_t dense_two_paths = 0;
    int64_t dense_edges = 0;
    int64_t dense_stored = 0;      // survivors the dense slots asked the store to keep
    int64_t dense_kept = 0;        // ... and those it kept (fewer: some slots walk again)
    bool use_store = false;        // the counting pass keeps the heavy overlaps for the emit pass
    CountStore store{};
    bool use_lstore = false;       // ... and the light rows' overlaps
    LightStore lstore{};
    int32_t *lwork = nullptr;      // [m]: 2-paths of the light rows
    int32_t *dorder = nullptr;     // [dense slots]: the counting pass's order (window-major)
    int64_t kept_rows = 0;         // |E_{s_min}|
    int64_t *store_work = nullptr; // [heavy slots]: 2-paths per slot
    int64_t store_limit = 0;
    int64_t store_min = 0;
    int64_t list_shortfall = 0;
    int64_t plan_lo = 0, plan_hi = -1;  // rows the rows phase plans (-1: to the last)
    int64_t stored_ranks = 0;
    int64_t two_paths = 0;
    int64_t heavy_two_paths = 0;
    int64_t heavy_edges = 0;
    int64_t nbounds = 0;
    int64_t num_edges[SLG_MAX_S] = {};
    const slg::ReserveFn *reserve = nullptr;  // asked before each planning allocation phase
    uint64_t reserved = 0;                    // bytes granted by `reserve`
};

struct slg_batch {
    slg_context *ctx = nullptr;
    hipStream_t st = nullptr;        // stream the batch was built on
    int32_t n = 0;
    std::vector<int64_t> m_off, m_g;  // per graph (m_off has n + 1 entries)
    std::vector<int64_t> edge_off;    // n + 1 global edge offsets
    slg_graph ug;                     // the disjoint union
    slg_plan *p = nullptr;
    int64_t *row_ptr = nullptr;
    int32_t *row = nullptr, *col = nullptr, *w = nullptr;
    int64_t edges = 0;
    std::vector<void *> owned;        // union arrays and outputs (hipMallocAsync)
    hipStream_t cap = nullptr;        // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct slg_result {
    slg_context *ctx = nullptr;
    hipStream_t st = nullptr;
    int32_t k = 0;
    int64_t m = 0;
    int64_t two_paths = 0;
    int64_t num_edges[SLG_MAX_S] = {};
    int64_t *row_ptr[SLG_MAX_S] = {};
    int32_t *row[SLG_MAX_S] = {};
    int32_t *col[SLG_MAX_S] = {};
    int32_t *w[SLG_MAX_S] = {};
    std::vector<void *> owned;
    std::shared_ptr<slg::Arena> arena;     // owner of `owned` unless the context's allocator made them
    std::shared_ptr<slg::ServeCore> core;  // served results: ledger the outputs are accounted to
    uint64_t bytes = 0;                    // device bytes accounted to `core`
};

namespace slg {
slg_status create_context(int device, uint64_t mem_budget_bytes, const slg_allocator *alloc, bool second_stream,
                          slg_context **out) {
    if (!out) return SLG_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return SLG_ERR_DEVICE;
    slg_context *ctx = new (std::nothrow) slg_context();
    if (!ctx) return SLG_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    ctx->budget = mem_budget_bytes;
    if (alloc && alloc->alloc && alloc->release) {
        ctx->has_alloc = true;
        ctx->alloc = *alloc;
    }
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&ctx->pinned), kPinnedSlots * sizeof(int64_t),
                      hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return SLG_ERR_DEVICE;
    }
    ctx->heavy_resident = heavy_resident(device);
    ctx->dense_resident = dense_resident(device);
    // the fixed scratch of the no-allocation entry point: its address on
    // this device, looked up once per device with the device current
    ctx->noalloc_err = noalloc_scratch(device, &ctx->noalloc);
    if (ctx->noalloc_err != hipSuccess) (void)hipGetLastError();
    ctx->aux_allowed = second_stream;
    uint64_t cache = mem_budget_bytes;
    if (!cache) {
        size_t free_b = 0, total_b = 0;
        cache = hipMemGetInfo(&free_b, &total_b) == hipSuccess ? total_b / 2 : 0;
        if (cache < kDefaultCacheMin) cache = kDefaultCacheMin;
    }
    ctx->arena = std::make_shared<slg::Arena>(device, cache);
    // keep freed scratch in the stream-ordered pool between calls
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    *out = ctx;
    return SLG_OK;
}
}  // namespace slg

extern "C" {

const char *slg_version(void) { return "slg 0.1.0 (gfx950)"; }

slg_status slg_context_create(int device, uint64_t mem_budget_bytes, const slg_allocator *alloc,
                              slg_context **out) {
    return slg::create_context(device, mem_budget_bytes, alloc, true, out);
}

slg_status slg_context_destroy(slg_context *ctx) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    for (const PendingTime &pt : ctx->pending) {
        (void)hipEventSynchronize(pt.stop);
        ctx->event_pool.push_back(pt.start);
        ctx->event_pool.push_back(pt.stop);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    (void)hipGetLastError();  // teardown errors stay out of later calls' launch checks
    return SLG_OK;
}

const char *slg_last_error(const slg_context *ctx) {
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

slg_status slg_graph_register(slg_context *ctx, const slg_incidence *inc, uint32_t flags,
                              void *stream, slg_graph **out) {
    if (!ctx || !inc || !out) return fail(ctx, SLG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const int64_t m = inc->num_hyperedges, n = inc->num_vertices, nnz = inc->nnz;
    if (m < 0 || n < 0 || nnz < 0) return fail(ctx, SLG_ERR_INVALID_ARG, "negative size");
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31))
        return fail(ctx, SLG_ERR_OVERFLOW, "m, n and nnz must be below 2^31");
    if (!inc->he_ptr || !inc->v_ptr || (nnz > 0 && (!inc->he_idx || !inc->v_idx)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "null CSR array");
    if (flags & ~(SLG_VALIDATE | SLG_COPY)) return fail(ctx, SLG_ERR_INVALID_ARG, "unknown flags");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // SLG_COPY: the library's own copies (from host or device memory); the
    // caller's arrays are free again when the call returns
    slg_incidence copy = *inc;
    std::vector<void *> owned;
    if (flags & SLG_COPY) {
        auto drop = [&](slg_status code, const char *msg) {
            (void)hipStreamSynchronize(st);
            for (void *q : owned) (void)hipFree(q);
            return fail(ctx, code, "%s", msg);
        };
        const void *src[4] = {inc->he_ptr, inc->he_idx, inc->v_ptr, inc->v_idx};
        const size_t bytes[4] = {size_t(m + 1) * 8, size_t(nnz) * 4, size_t(n + 1) * 8, size_t(nnz) * 4};
        void *dst[4] = {};
        for (int t = 0; t < 4; ++t) {
            if (hipMalloc(&dst[t], bytes[t] ? bytes[t] : 8) != hipSuccess) {
                (void)hipGetLastError();
                return drop(SLG_ERR_OUT_OF_MEMORY, "no device memory for the graph's copy");
            }
            owned.push_back(dst[t]);
            if (bytes[t] && hipMemcpyAsync(dst[t], src[t], bytes[t], hipMemcpyDefault, st) != hipSuccess) {
                (void)hipGetLastError();
                return drop(SLG_ERR_DEVICE, "copying the incidence failed");
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            return drop(SLG_ERR_DEVICE, "copying the incidence failed");
        }
        copy.he_ptr = static_cast<const int64_t *>(dst[0]);
        copy.he_idx = static_cast<const int32_t *>(dst[1]);
        copy.v_ptr = static_cast<const int64_t *>(dst[2]);
        copy.v_idx = static_cast<const int32_t *>(dst[3]);
        inc = &copy;
    }
    auto drop_owned = [&]() {
        for (void *q : owned) (void)hipFree(q);
        owned.clear();
    };
    if (flags & SLG_VALIDATE) {
        Scratch sc;
        sc.st = st;
        sc.arena = ctx->arena.get();
        int64_t *err = nullptr;
        SLG_HIP(ctx, sc.get(&err, 1));
        SLG_HIP(ctx, launch_fill_i64(err, 1, 0, st));
        int *e32 = reinterpret_cast<int *>(err);
        SLG_HIP(ctx, launch_validate_ptr(inc->he_ptr, m, nnz, e32, st));
        SLG_HIP(ctx, launch_validate_ptr(inc->v_ptr, n, nnz, e32, st));
        SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        SLG_HIP(ctx, hipStreamSynchronize(st));
        int64_t code = ctx->pinned[0];
        if (!code) {  // pointers are sound: rows may be read
            SLG_HIP(ctx, launch_validate_rows(inc->he_ptr, inc->he_idx, m, n, e32, st));
            SLG_HIP(ctx, launch_validate_rows(inc->v_ptr, inc->v_idx, n, m, e32, st));
            SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            SLG_HIP(ctx, hipStreamSynchronize(st));
            code = ctx->pinned[0];
        }
        if (!code) {  // ids in range: check the transpose
            SLG_HIP(ctx, launch_validate_transpose(inc->he_ptr, inc->he_idx, m, inc->v_ptr, inc->v_idx,
                                                   n, e32, st));
            SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            SLG_HIP(ctx, hipStreamSynchronize(st));
            code = ctx->pinned[0];
        }
        sc.release();
        if (code) drop_owned();
        if (code & 2) return fail(ctx, SLG_ERR_INVALID_GRAPH, "CSR pointer array malformed");
        if (code & 4) return fail(ctx, SLG_ERR_INVALID_GRAPH, "CSR row holds an out-of-range or repeated id");
        if (code & 8) return fail(ctx, SLG_ERR_INVALID_GRAPH, "vertex CSR is not the transpose");
    }
    slg_graph *g = new (std::nothrow) slg_graph();
    if (!g) {
        drop_owned();
        return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    g->ctx = ctx;
    g->owned = owned;
    g->inc = *inc;
    *out = g;
    return SLG_OK;
}

slg_status slg_graph_release(slg_graph *g) {
    if (!g) return SLG_ERR_INVALID_ARG;
    if (!g->owned.empty()) {
        (void)hipSetDevice(g->ctx->device);
        (void)hipDeviceSynchronize();  // work still reading the copies
        for (void *q : g->owned) (void)hipFree(q);
        (void)hipGetLastError();
    }
    delete g;
    return SLG_OK;
}

namespace {

// Planning launches up to the tier sizes: pruning, per-row plan, scans.
hipError_t enqueue_rows(slg_plan *p, hipStream_t st) {
    slg_context *ctx = p->ctx;
    const slg_incidence &inc = p->g->inc;
    const int64_t m = inc.num_hyperedges, n = inc.num_vertices, nnz = inc.nnz;
    PlanBufs &b = p->b;
    hipError_t e;
    if ((e = launch_fill_i64(b.counters, 32, 0, st)) != hipSuccess) return e;
    if (p->prune) {
        StageTimer tm(ctx, kStPrune, st);
        if ((e = launch_keep_incidence(nnz, inc.v_idx, inc.he_ptr, m, p->s_min, p->pr.row_s, b.flag, st)) !=
            hipSuccess)
            return e;
        if ((e = launch_exclusive_scan_u8(b.flag, nnz, b.pos, b.part_nnz, st)) != hipSuccess) return e;
        if ((e = launch_compact_vertex_lists(n, nnz, inc.v_ptr, inc.v_idx, b.flag, b.pos, b.vs_ptr, b.vs_idx,
                                             st)) != hipSuccess)
            return e;
    }
    if (p->dense) {  // E_s positions: ranks of the kept rows, and the pruned lists in ranks
        StageTimer tm(ctx, kStPrune, st);
        if ((e = launch_row_keep(m, inc.he_ptr, p->s_min, p->pr.row_s, b.keep, st)) != hipSuccess) return e;
        if ((e = launch_exclusive_scan_u8(b.keep, m, b.kpre, b.part_m, st)) != hipSuccess) return e;
        if ((e = launch_cid(m, b.keep, b.kpre, b.cid, b.cid_row, st)) != hipSuccess) return e;
        if ((e = launch_vs_cid(n, m, nnz, p->pr.vs_ptr, p->pr.vs_idx, b.cid, b.vs_cid, b.vs_win, st)) != hipSuccess) return e;
    }
    {
        StageTimer tm(ctx, kStRowPlan, st);
        if ((e = launch_row_plan(p->pr, p->s_min, p->light_max, p->slot_work, p->plan_lo,
                                 p->plan_hi < 0 ? m : p->plan_hi, p->dense ? p->dense_ratio : 0,
                                 p->dense_min, b.tail_beg, b.work, b.jmax, b.nslots, b.rclass, b.bsize,
                                 reinterpret_cast<unsigned long long *>(b.counters + kCntClass),
                                 reinterpret_cast<int *>(b.counters + kCntErr),
                                 reinterpret_cast<unsigned long long *>(b.counters + kCntHeavyWork),
                                 reinterpret_cast<unsigned long long *>(b.counters + kCntDenseWork), b.pieces,
                                 reinterpret_cast<unsigned long long *>(b.counters + kCntPieces), st)) !=
            hipSuccess)
            return e;
    }
    StageTimer tm(ctx, kStPlanScans, st);
    if ((e = launch_exclusive_scan_i32(b.nslots, m, p->slot_base, b.part_m, st)) != hipSuccess) return e;
    if ((e = launch_exclusive_scan_i64(b.work, m, b.work_pre, b.part_m, st)) != hipSuccess) return e;
    return launch_exclusive_scan_i64(b.bsize, m, b.bbase, b.part_m, st);
}

// Slot table, tier lists, boundary table, counting pass and its scans.
// Plans with fewer 2-paths stay on one stream: their light counting pass is
// short, and an extra stream per context, even idle, has measured slower
// when several contexts serve concurrent queries (more streams share the
// process's hardware queues).
constexpr int64_t kForkMinTwoPaths = int64_t(1) << 28;

// Makes the context's second stream and its events; false when the context
// goes without, creation fails, or a HIP-graph capture is recording (a
// captured path never forks, even on a context that already has the
// stream).
bool ensure_aux(slg_context *ctx) {
    if (ctx->capturing) return false;
    if (ctx->aux) return true;
    if (!ctx->aux_allowed) return false;
    if (hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) == hipSuccess)
        return true;
    (void)hipGetLastError();  // run everything on the caller's stream instead
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    ctx->aux = nullptr;
    ctx->fork_ev = ctx->join_ev = nullptr;
    ctx->aux_allowed = false;
    return false;
}

// Work forked onto the context's second stream after what `st` holds so far,
// and joined back into `st` when the guard ends (on every path out). Without
// the second stream, the work stays on `st`.
struct AuxFork {
    slg_context *ctx;
    hipStream_t st;
    bool on = false;
    AuxFork(slg_context *c, hipStream_t s) : ctx(c), st(s) {}
    hipStream_t begin(bool want, hipError_t *e) {
        *e = hipSuccess;
        if (!want || !ensure_aux(ctx)) return st;
        if ((*e = hipEventRecord(ctx->fork_ev, st)) != hipSuccess) return st;
        if ((*e = hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0)) != hipSuccess) return st;
        on = true;
        return ctx->aux;
    }
    hipError_t join() {
        if (!on) return hipSuccess;
        on = false;
        const hipError_t e = hipEventRecord(ctx->join_ev, ctx->aux);
        return e != hipSuccess ? e : hipStreamWaitEvent(st, ctx->join_ev, 0);
    }
    ~AuxFork() { (void)join(); }
};

hipError_t enqueue_slots_count(slg_plan *p, hipStream_t st) {
    slg_context *ctx = p->ctx;
    const int64_t m = p->pr.m;
    PlanBufs &b = p->b;
    hipError_t e;
    // lists start zeroed: an entry the fill kernels refuse to write (list
    // overflow, flagged in err) names slot 0 / an empty descriptor
    for (int c = 0; c < kLightClasses; ++c)
        if ((e = launch_fill_i32(p->lists[c], p->list_count[c], 0, st)) != hipSuccess) return e;
    for (int h = 0; h < kNumHeavyLists; ++h)
        if ((e = launch_fill_i64(reinterpret_cast<int64_t *>(p->heavy[h]),
                                 p->list_count[kLightClasses + h] * (int64_t)(sizeof(HeavyDesc) / 8), 0, st)) !=
            hipSuccess)
            return e;
    {
        StageTimer tm(ctx, kStSlots, st);
        // room of every list as planned (less the error-path tests' shortfall
        // on the heavy lists: appends past it are refused and flagged)
        int64_t caps[kNumLists];
        for (int c = 0; c < kNumLists; ++c)
            caps[c] = c < kLightClasses ? p->list_count[c] : std::max<int64_t>(0, p->list_count[c] - p->list_shortfall);
        if ((e = launch_fill_slots(m, p->pr.he_ptr, p->slot_base, b.nslots, b.jmax, b.rclass, b.bbase, b.cid,
                                   b.hat, b.hcnt, b.part_m, b.slot_row, p->lists, p->heavy, caps,
                                   reinterpret_cast<unsigned long long *>(b.counters + kCntFill),
                                   reinterpret_cast<int *>(b.counters + kCntErr), st)) != hipSuccess)
            return e;
    }
    // the light tier's counting pass runs on the context's second stream,
    // beside the boundary table: it reads the light lists and writes the
    // light slots' counts (and the light store), which nothing on the
    // caller's stream touches before the join
    AuxFork fork(ctx, st);
    const hipStream_t lst = fork.begin(p->two_paths >= kForkMinTwoPaths, &e);
    if (e != hipSuccess) return e;
    {
        StageTimer tm(ctx, kStCountLight, lst);
        if (p->use_lstore) {  // the light store's layout
            if ((e = launch_light_work(m, b.rclass, b.work, p->lwork, lst)) != hipSuccess) return e;
            if ((e = launch_exclusive_scan_i32(p->lwork, m, p->lstore.off, b.part_m, lst)) != hipSuccess) return e;
        }
        for (int c = 0; c < kLightClasses; ++c)
            if ((e = launch_light(c, false, p->lists[c], p->list_count[c], p->slots, p->pr, p->prm, p->slot_cnt,
                                  nullptr, (p->use_lstore && c > 0) ? &p->lstore : nullptr, lst)) != hipSuccess)
                return e;
    }
    {
        StageTimer tm(ctx, kStBounds, st);
        for (int h = 0; h < kNumHeavyLists; ++h) {
            // dense slots bound their members' tails by E_s position
            Pruned pg = p->pr;
            if (h == 2) pg.vs_idx = b.vs_cid;
            if ((e = launch_bounds(pg, p->heavy[h], p->list_count[kLightClasses + h], p->bounds, st)) != hipSuccess)
                return e;
        }
    }
    if (p->use_store) {  // the store's layout: each heavy slot's 2-paths bound its partners
        StageTimer tm(ctx, kStBounds, st);
        const int64_t nh = p->list_count[kLightClasses];
        if ((e = launch_slot_work(p->heavy[0], nh, p->bounds, p->store_work, st)) != hipSuccess) return e;
        if ((e = launch_exclusive_scan_i64(p->store_work, nh, p->store.off, b.part_s, st)) != hipSuccess) return e;
    }
    // joined before the heavy counting pass: its persistent grid fills every
    // CU, and light workgroups still resident would hold some of it back
    if ((e = fork.join()) != hipSuccess) return e;
    if ((e = launch_fill_i64(p->tickets, kTkTotal, 0, st)) != hipSuccess) return e;
    for (int wide = 0; wide < 2; ++wide) {
        if (p->list_count[kLightClasses + wide] <= 0) continue;
        StageTimer tm(ctx, wide ? kStCountHeavyWide : kStCountHeavy, st);
        if ((e = launch_heavy(false, wide, p->heavy[wide], p->list_count[kLightClasses + wide], p->S, p->bounds,
                              p->pr, p->prm, p->slot_cnt, nullptr, p->tickets + kTkCount + wide, p->heavy_grid,
                              (p->use_store && !wide) ? &p->store : nullptr, st)) != hipSuccess)
            return e;
    }
    const int64_t nd = p->list_count[kLightClasses + 2];
    if (nd > 0) {
        // window-major order: the workgroups in flight count the same
        // window of E_s for many rows, so the vertex-list segments of that
        // window are read from L2 instead of HBM (stable: rows stay in order)
        const int32_t *order = nullptr;
        if (nd > 1 && p->dorder) {
            StageTimer tm(ctx, kStSlots, st);
            int32_t *key = nullptr, *id = nullptr, *skey = nullptr;
            if ((e = p->scratch2.get(&key, nd)) != hipSuccess || (e = p->scratch2.get(&id, nd)) != hipSuccess ||
                (e = p->scratch2.get(&skey, nd)) != hipSuccess)
                return e;
            if ((e = launch_dense_keys(p->heavy[2], nd, key, id, st)) != hipSuccess) return e;
            const int64_t windows = (p->kept_rows >> kDenseBits) + 1;
            if ((e = sort_pairs(p->scratch2, key, id, nullptr, nd, bits_for(windows), skey, p->dorder, nullptr, st)) !=
                hipSuccess)
                return e;
            order = p->dorder;
        }
        StageTimer tm(ctx, kStCountDense, st);
        if ((e = launch_dense(false, p->heavy[2], nd, order, p->S, p->bounds, p->pr, p->prm, p->slot_cnt, nullptr,
                              p->tickets + kTkCount + 2, p->dense_grid, p->use_dstore ? &p->dstore : nullptr,
                              p->tickets + kTkDenseCursor, p->dstore_cap, st)) != hipSuccess)
            return e;
    }
    StageTimer tm(ctx, kStCountScans, st);
    for (int k = 0; k < p->prm.k; ++k)
        if ((e = launch_exclusive_scan_i64(p->slot_cnt + (size_t)k * p->S, p->S,
                                           p->slot_off + (size_t)k * (p->S + 1), b.part_s, st)) != hipSuccess)
            return e;
    return hipSuccess;
}

#define BUILD_HIP(call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(ctx, e_ == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE,     \
                        "%s: %s", #call, hipGetErrorString(e_));                                   \
    } while (0)

// The rows phase of a plan: pruning, E_s positions, the per-row work
// estimate and tiers, and their scans over every row, with the readback
// that sizes a plan of all rows.
// Workgroups of the dense tier's launches, at most (each may leave one
// store chunk partly unused).
int64_t dense_workgroups(const slg_plan *p) { return p->dense_grid > 0 ? p->dense_grid : 512; }

slg_status plan_rows(slg_plan *p) {
    slg_context *ctx = p->ctx;
    const slg_incidence &inc = p->g->inc;
    const int64_t m = inc.num_hyperedges, n = inc.num_vertices, nnz = inc.nnz;
    hipStream_t st = p->st;
    Scratch &sc = p->scratch;
    PlanBufs &b = p->b;
    Pruned &pr = p->pr;
    pr.m = m;
    pr.n = n;
    pr.nnz = nnz;
    pr.he_ptr = inc.he_ptr;
    pr.he_idx = inc.he_idx;
    p->prune = (p->s_min > 1 || pr.row_s) && nnz > 0;
    // the dense tier works in E_s positions; the batched form (a threshold
    // per row) keeps to the other tiers
    p->dense = p->dense_ratio > 0 && !pr.row_s && nnz > 0 && m > 0;
    AllocList phase1;
    if (p->prune) {
        phase1.add(&b.flag, nnz);
        phase1.add(&b.pos, nnz + 1);
        phase1.add(&b.part_nnz, scan_partials_size(nnz));
        phase1.add(&b.vs_ptr, n + 1);
        phase1.add(&b.vs_idx, nnz);
    }
    phase1.add(&b.tail_beg, nnz);
    phase1.add(&b.work, m);
    phase1.add(&b.work_pre, m + 1);
    phase1.add(&b.jmax, m);
    phase1.add(&b.nslots, m);
    phase1.add(&b.rclass, m);
    phase1.add(&b.bsize, m);
    phase1.add(&b.bbase, m + 1);
    phase1.add(&b.hat, kNumHeavyLists * (m + 1));
    phase1.add(&b.hcnt, kNumHeavyLists * m);
    if (p->dense) {
        phase1.add(&b.keep, m);
        phase1.add(&b.kpre, m + 1);
        phase1.add(&b.cid, m);
        phase1.add(&b.cid_row, m);
        phase1.add(&b.vs_cid, nnz + kDensePad);
        phase1.add(&b.vs_win, nnz + kDensePad);  // the dense walk may load (not count) past the end
    }
    if (p->blocks) {
        phase1.add(&b.nslots_all, m);
        phase1.add(&b.rclass_all, m);
        phase1.add(&b.bsize_all, m);
    }
    phase1.add(&b.counters, 32);
    phase1.add(&b.pieces, 3 * plan_pieces_cap(nnz));
    phase1.add(&b.part_m, scan_partials_size(m));
    phase1.add(&p->slot_base, m + 1);
    if (p->reserve) {
        if (!(*p->reserve)(phase1.bytes)) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "device-memory budget refused");
        p->reserved += phase1.bytes;
    }
    for (const auto &a : phase1.items) BUILD_HIP(sc.get(a.first, a.second));
    if (p->prune) {
        pr.vs_ptr = b.vs_ptr;
        pr.vs_idx = b.vs_idx;
    } else {
        pr.vs_ptr = inc.v_ptr;
        pr.vs_idx = inc.v_idx;
    }
    pr.tail_beg = b.tail_beg;
    pr.cid = b.cid;
    pr.cid_row = b.cid_row;
    pr.vs_cid = b.vs_cid;
    pr.vs_win = b.vs_win;
    BUILD_HIP(enqueue_rows(p, st));
    if (p->blocks && m > 0) {
        BUILD_HIP(hipMemcpyAsync(b.nslots_all, b.nslots, m * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        BUILD_HIP(hipMemcpyAsync(b.rclass_all, b.rclass, m, hipMemcpyDeviceToDevice, st));
        BUILD_HIP(hipMemcpyAsync(b.bsize_all, b.bsize, m * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    }
    int64_t *hb = ctx->pinned;
    BUILD_HIP(hipMemcpyAsync(hb, b.counters, kCntTotal * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BUILD_HIP(hipMemcpyAsync(hb + kHbSlots, p->slot_base + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BUILD_HIP(hipMemcpyAsync(hb + kHbSlots + 1, b.work_pre + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BUILD_HIP(hipMemcpyAsync(hb + kHbSlots + 2, b.bbase + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (p->dense) BUILD_HIP(hipMemcpyAsync(hb + kHbRange + 1, b.kpre + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BUILD_HIP(hipStreamSynchronize(st));
    p->kept_rows = p->dense ? hb[kHbRange + 1] : 0;
    if (hb[kCntErr] & 0xffffffff)
        return fail(ctx, SLG_ERR_INVALID_GRAPH,
                    "malformed incidence (bad pointer, id out of range, or vertex CSR not the transpose)");
    for (int c = 0; c < kNumLists; ++c) p->list_count[c] = hb[kCntClass + c];
    p->S = hb[kHbSlots];
    p->two_paths = hb[kHbSlots + 1];
    p->nbounds = hb[kHbSlots + 2];
    p->heavy_two_paths = hb[kCntHeavyWork];
    p->dense_two_paths = hb[kCntDenseWork];
    p->row_lo = 0;
    p->row_hi = m;
    return SLG_OK;
}

// The block phase: the slot table, tier lists, boundary table, stores and
// the counting pass of rows [r0, r1) (all rows: [0, m), sized by the rows
// phase; a part of them: the other rows are masked out first). Its
// allocations come from scratch2, released by the next block or the plan's
// end.
slg_status plan_block(slg_plan *p, int64_t r0, int64_t r1) {
    slg_context *ctx = p->ctx;
    const int64_t m = p->pr.m;
    hipStream_t st = p->st;
    Scratch &sc = p->scratch2;
    PlanBufs &b = p->b;
    int64_t *hb = ctx->pinned;
    sc.release();
    if (r0 > 0 || r1 < m) {
        if (!p->blocks) return fail(ctx, SLG_ERR_INVALID_ARG, "internal error: a row block of a whole plan");
        BUILD_HIP(launch_fill_i64(b.counters, 32, 0, st));
        BUILD_HIP(launch_block_mask(m, r0, r1, b.nslots_all, b.rclass_all, b.bsize_all, b.work, b.nslots, b.rclass,
                                    b.bsize, reinterpret_cast<unsigned long long *>(b.counters + kCntClass),
                                    reinterpret_cast<unsigned long long *>(b.counters + kCntHeavyWork),
                                    reinterpret_cast<unsigned long long *>(b.counters + kCntDenseWork), st));
        BUILD_HIP(launch_exclusive_scan_i32(b.nslots, m, p->slot_base, b.part_m, st));
        BUILD_HIP(launch_exclusive_scan_i64(b.bsize, m, b.bbase, b.part_m, st));
        BUILD_HIP(hipMemcpyAsync(hb, b.counters, kCntTotal * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BUILD_HIP(hipMemcpyAsync(hb + kHbSlots, p->slot_base + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BUILD_HIP(hipMemcpyAsync(hb + kHbSlots + 1, b.work_pre + r0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BUILD_HIP(hipMemcpyAsync(hb + kHbSlots + 2, b.bbase + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BUILD_HIP(hipMemcpyAsync(hb + kHbRange, b.work_pre + r1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BUILD_HIP(hipStreamSynchronize(st));
        for (int c = 0; c < kNumLists; ++c) p->list_count[c] = hb[kCntClass + c];
        p->S = hb[kHbSlots];
        p->two_paths = hb[kHbRange] - hb[kHbSlots + 1];
        p->nbounds = hb[kHbSlots + 2];
        p->heavy_two_paths = hb[kCntHeavyWork];
        p->dense_two_paths = hb[kCntDenseWork];
    } else if (p->blocks && (p->row_lo != 0 || p->row_hi != m)) {
        return fail(ctx, SLG_ERR_INVALID_ARG, "internal error: all rows after a row block");
    }
    p->row_lo = r0;
    p->row_hi = r1;
    if (p->S >= (int64_t(1) << 31)) return fail(ctx, SLG_ERR_OVERFLOW, "more than 2^31 output slots");
    if (p->nbounds >= (int64_t(1) << 40)) return fail(ctx, SLG_ERR_OVERFLOW, "boundary table too large");

    const int K = p->prm.k;
    AllocList phase2;
    phase2.add(&b.slot_row, p->S);
    phase2.add(&p->bounds, p->nbounds);
    phase2.add(&p->tickets, kTkTotal);
    for (int c = 0; c < kLightClasses; ++c) phase2.add(&p->lists[c], p->list_count[c]);
    for (int h = 0; h < kNumHeavyLists; ++h) phase2.add(&p->heavy[h], p->list_count[kLightClasses + h]);
    static_assert(sizeof(HeavyDesc) % 8 == 0, "HeavyDesc is filled as int64 words");
    phase2.add(&p->slot_cnt, (size_t)K * p->S);
    phase2.add(&p->slot_off, (size_t)K * (p->S + 1));
    phase2.add(&b.part_s, scan_partials_size(p->S));
    {  // the count store, when it fits the context's limit
        const int64_t nh = p->list_count[kLightClasses];
        // below store_min (a batch of small graphs) the store's extra
        // launches cost more than the walk they save
        const int64_t bytes = p->heavy_two_paths * 4 + nh * 20 + 16;
        p->use_store = nh > 0 && p->store_limit > 0 && bytes <= p->store_limit &&
                       p->heavy_two_paths >= p->store_min;
        // the light rows' pairs: at most their 2-paths (all but the heavy and dense ones)
        const int64_t lcap = p->two_paths - p->heavy_two_paths - p->dense_two_paths;
        const int64_t lbytes = lcap * 6 + m * 16 + 16;
        p->use_lstore = p->store_limit > 0 && lcap > 0 && p->two_paths >= p->store_min &&
                        (p->use_store ? bytes : 0) + lbytes <= p->store_limit;
        if (p->use_lstore) {
            phase2.add(&p->lstore.key, lcap);
            phase2.add(&p->lstore.cnt, lcap);
            phase2.add(&p->lstore.off, m + 1);
            phase2.add(&p->lstore.n, m);
            phase2.add(&p->lwork, m);
        }
        if (p->use_store) {
            phase2.add(&p->store.ent, p->heavy_two_paths);
            phase2.add(&p->store.off, nh + 1);
            phase2.add(&p->store.n, nh);
            phase2.add(&p->store_work, nh);
        }
        // the dense slots' survivors: at most one per s_min of their 2-paths,
        // in what the limit leaves (slots that find it full walk again)
        const int64_t nd = p->list_count[kLightClasses + 2];
        const int64_t left = p->store_limit - (p->use_store ? bytes : 0) - (p->use_lstore ? lbytes : 0) -
                             nd * 12 - 16;
        // (room is handed out in chunks: each persistent workgroup may leave one unfilled)
        p->dstore_cap = std::min<int64_t>(
            p->dense_two_paths / std::max(p->s_min, 1) + 1 + (int64_t)dense_workgroups(p) * kDenseChunk, left / 4);
        if (p->dstore_fixed) p->dstore_cap = p->dstore_fixed_cap;  // row blocks share one store of fixed size
        p->use_dstore = nd > 0 && p->dstore_cap > 0;
        if (nd > 1) phase2.add(&p->dorder, nd);
        if (p->use_dstore) {
            if (!p->dstore_fixed) phase2.add(&p->dstore.ent, p->dstore_cap);
            phase2.add(&p->dstore.off, nd);
            phase2.add(&p->dstore.n, nd);
        } else {
            p->dstore_cap = 0;
        }
    }
    if (p->reserve) {
        if (!(*p->reserve)(phase2.bytes)) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "device-memory budget refused");
        p->reserved += phase2.bytes;
    }
    for (const auto &a : phase2.items) BUILD_HIP(sc.get(a.first, a.second));
    if (p->dstore_fixed && p->use_dstore) p->dstore.ent = p->dstore_fixed;
    p->slots.count = p->S;
    p->slots.row = b.slot_row;
    BUILD_HIP(enqueue_slots_count(p, st));
    for (int k = 0; k < K; ++k)
        BUILD_HIP(hipMemcpyAsync(hb + kHbEdges + k, p->slot_off + (size_t)k * (p->S + 1) + p->S, sizeof(int64_t),
                                 hipMemcpyDeviceToHost, st));
    for (int h = 0; h < 2; ++h)
        BUILD_HIP(launch_heavy_edges(p->heavy[h], p->list_count[kLightClasses + h], p->slot_cnt, p->S, K,
                                     p->tickets + kTkHeavyEdges, st));
    BUILD_HIP(launch_heavy_edges(p->heavy[2], p->list_count[kLightClasses + 2], p->slot_cnt, p->S, K,
                                 p->tickets + kTkDenseEdges, st));
    if (p->use_store)
        BUILD_HIP(launch_sum_i32(p->store.n, p->list_count[kLightClasses], p->tickets + kTkStored, st));
    BUILD_HIP(hipMemcpyAsync(hb + kHbHeavyEdges, p->tickets + kTkHeavyEdges, 6 * sizeof(int64_t),
                             hipMemcpyDeviceToHost, st));  // heavy edges, stored, dense room, asked, kept, edges
    BUILD_HIP(hipMemcpyAsync(hb + kHbHeavyEdges + 6, b.counters + kCntErr, sizeof(int64_t),
                             hipMemcpyDeviceToHost, st));
    BUILD_HIP(hipStreamSynchronize(st));
    if (hb[kHbHeavyEdges + 6] & 0xffffffff)
        return fail(ctx, SLG_ERR_DEVICE, "internal error: a tier list overflowed its planned size");
    for (int k = 0; k < K; ++k) p->num_edges[k] = hb[kHbEdges + k];
    p->heavy_edges = hb[kHbHeavyEdges];
    p->stored_ranks = hb[kHbHeavyEdges + 1];
    p->dense_stored = hb[kHbHeavyEdges + 3];
    p->dense_kept = hb[kHbHeavyEdges + 4];
    p->dense_edges = hb[kHbHeavyEdges + 5];
    int64_t *wk = ctx->work;
    wk[kWkBlocks] += 1;
    wk[kWkTwoPaths] += p->two_paths;
    wk[kWkHeavyTwoPaths] += p->heavy_two_paths;
    wk[kWkDenseTwoPaths] += p->dense_two_paths;
    for (int k = 0; k < K; ++k) wk[kWkEdges] += p->num_edges[k];
    wk[kWkHeavyEdges] += p->heavy_edges;
    wk[kWkDenseEdges] += p->dense_edges;
    wk[kWkDenseSlots] += p->list_count[kLightClasses + 2];
    wk[kWkDenseStored] += p->dense_kept;
    wk[kWkDenseRewalk] += (p->list_count[kLightClasses + 2] > 0 && p->dense_stored > p->dense_kept) ? 1 : 0;
    return SLG_OK;
}

// Builds a plan of all rows.
slg_status plan_build(slg_plan *p) {
    slg_status rc = plan_rows(p);
    return rc != SLG_OK ? rc : plan_block(p, 0, p->pr.m);
}
#undef BUILD_HIP

slg_plan *plan_new(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s, hipStream_t st) {
    slg_plan *p = new (std::nothrow) slg_plan();
    if (!p) return nullptr;
    p->ctx = ctx;
    p->g = g;
    p->st = st;
    p->scratch.st = st;
    p->scratch.arena = ctx->arena.get();
    p->scratch2.st = st;
    p->scratch2.arena = ctx->arena.get();
    p->prm.k = num_s;
    for (int t = 0; t < num_s; ++t) p->prm.s[t] = s[t];
    p->s_min = s[0];
    p->light_max = ctx->light_max;
    p->slot_work = ctx->slot_work;
    p->heavy_grid = ctx->heavy_grid > 0 ? ctx->heavy_grid : ctx->heavy_resident;
    p->dense_ratio = ctx->dense_ratio;
    p->dense_min = ctx->dense_min;
    p->dense_grid = ctx->dense_resident;
    p->store_limit = ctx->store_limit;
    p->store_min = ctx->store_min;
    p->list_shortfall = ctx->list_shortfall;
    return p;
}

void plan_free(slg_plan *p) {
    p->scratch2.release();
    p->scratch.release();
    (void)hipStreamSynchronize(p->st);
    (void)hipGetLastError();
    delete p;
}
}  // namespace

slg_status slg_plan_create(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                           void *stream, slg_plan **out) {
    if (!ctx || !g || !out) return fail(ctx, SLG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (!valid_s(s, num_s))
        return fail(ctx, SLG_ERR_INVALID_ARG, "s must be strictly increasing, s[0] >= 1, 1 <= num_s <= %d",
                    SLG_MAX_S);
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    slg_plan *p = plan_new(ctx, g, s, num_s, static_cast<hipStream_t>(stream));
    if (!p) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    slg_status rc = plan_build(p);
    if (rc != SLG_OK) {
        plan_free(p);
        return rc;
    }
    *out = p;
    return SLG_OK;
}

slg_status slg_plan_info(const slg_plan *p, int32_t k, int64_t *num_edges, int64_t *two_paths) {
    if (!p || k < 0 || k >= p->prm.k) return SLG_ERR_INVALID_ARG;
    if (num_edges) *num_edges = p->num_edges[k];
    if (two_paths) *two_paths = p->two_paths;
    return SLG_OK;
}

namespace {
// Emit rows [r0, r1) (slots [s0, s1)) of every threshold into buffers whose
// first entry is global edge offset base[k]; row_ptr[k] gets r1 - r0 + 1
// entries relative to base[k].
// lists (optional, host): the chunk's part [lists[2h], lists[2h+1]) of
// heavy list h, known beforehand; else found on the device and read back.
slg_status emit_range(slg_plan *p, int64_t r0, int64_t r1, int64_t s0, int64_t s1, const int64_t *base,
                      int64_t *const *row_ptr, int32_t *const *row, int32_t *const *col, int32_t *const *w,
                      hipStream_t st, const int64_t *lists = nullptr) {
    slg_context *ctx = p->ctx;
    const int K = p->prm.k;
    EmitParams prm = p->prm;
    prm.slot_lo = (int32_t)s0;
    prm.slot_hi = (int32_t)s1;
    for (int k = 0; k < K; ++k) {
        prm.row_ptr[k] = row_ptr[k];
        prm.row[k] = row ? row[k] : nullptr;
        prm.col[k] = col[k];
        prm.w[k] = w[k];
        prm.out_base[k] = base[k];
    }
    {
        StageTimer tm(ctx, kStEmitLight, st);
        for (int c = 0; c < kLightClasses; ++c) {
            if (p->use_lstore && c > 0)
                SLG_HIP(ctx, launch_light_store_emit(p->lists[c], p->list_count[c], p->slots, p->lstore, prm,
                                                     p->slot_off, st));
            else
                SLG_HIP(ctx, launch_light(c, true, p->lists[c], p->list_count[c], p->slots, p->pr, prm, nullptr,
                                          p->slot_off, nullptr, st));
        }
    }
    SLG_HIP(ctx, launch_fill_i64(p->tickets + kTkEmit, kNumHeavyLists, 0, st));
    // a chunk's heavy slots: a contiguous part of each heavy list (all are
    // in slot order), found on the device and read back
    int64_t lo[kNumHeavyLists] = {}, hi[kNumHeavyLists];
    for (int h = 0; h < kNumHeavyLists; ++h) hi[h] = p->list_count[kLightClasses + h];
    if (lists) {
        for (int h = 0; h < kNumHeavyLists; ++h) {
            lo[h] = lists[2 * h];
            hi[h] = lists[2 * h + 1];
        }
    } else if (s0 > 0 || s1 < p->S) {
        int64_t *hb = ctx->pinned + kHbRange;
        for (int h = 0; h < kNumHeavyLists; ++h) {
            if (hi[h] <= 0) continue;
            SLG_HIP(ctx, launch_heavy_range(p->heavy[h], hi[h], s0, s1, p->tickets + kTkRange + 2 * h, st));
            SLG_HIP(ctx, hipMemcpyAsync(hb + 2 * h, p->tickets + kTkRange + 2 * h, 2 * sizeof(int64_t),
                                        hipMemcpyDeviceToHost, st));
        }
        SLG_HIP(ctx, hipStreamSynchronize(st));
        for (int h = 0; h < kNumHeavyLists; ++h)
            if (hi[h] > 0) {
                lo[h] = hb[2 * h];
                hi[h] = hb[2 * h + 1];
            }
    }
    for (int wide = 0; wide < 2; ++wide) {
        const int64_t cnt = hi[wide] - lo[wide];
        if (cnt <= 0) continue;
        StageTimer tm(ctx, wide ? kStEmitHeavyWide : kStEmitHeavy, st);
        if (p->use_store && !wide) {
            const CountStore part{p->store.ent, p->store.off + lo[0], p->store.n + lo[0]};
            SLG_HIP(ctx, launch_heavy_store_emit(p->heavy[0] + lo[0], cnt, p->S, part, prm, p->slot_off, nullptr, st));
        } else {
            SLG_HIP(ctx, launch_heavy(true, wide, p->heavy[wide] + lo[wide], cnt, p->S, p->bounds, p->pr, prm,
                                      nullptr, p->slot_off, p->tickets + kTkEmit + wide, p->heavy_grid, nullptr,
                                      st));
        }
    }
    if (hi[2] > lo[2]) {  // dense slots: from their store, then any the store could not hold
        StageTimer tm(ctx, kStEmitDense, st);
        const int64_t cnt = hi[2] - lo[2];
        const CountStore part{p->dstore.ent, p->dstore.off + lo[2], p->dstore.n + lo[2]};
        if (p->use_dstore)
            SLG_HIP(ctx, launch_heavy_store_emit(p->heavy[2] + lo[2], cnt, p->S, part, prm, p->slot_off,
                                                 p->pr.cid_row, st));
        if (!p->use_dstore || p->dense_stored > p->dense_kept)
            SLG_HIP(ctx, launch_dense(true, p->heavy[2] + lo[2], cnt, nullptr, p->S, p->bounds, p->pr, prm, nullptr,
                                      p->slot_off, p->tickets + kTkEmit + 2, p->dense_grid,
                                      p->use_dstore ? &part : nullptr, nullptr, 0, st));
    }
    {
        StageTimer tm(ctx, kStRowPtr, st);
        SLG_HIP(ctx, launch_row_ptr(r0, r1, p->slot_base, p->slot_off, p->S, prm, st));
    }
    return SLG_OK;
}

slg_status order_after(slg_context *ctx, hipStream_t later, hipStream_t earlier) {
    if (later == earlier) return SLG_OK;
    hipEvent_t ev;
    SLG_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    SLG_HIP(ctx, hipEventRecord(ev, earlier));
    SLG_HIP(ctx, hipStreamWaitEvent(later, ev, 0));
    SLG_HIP(ctx, hipEventDestroy(ev));
    return SLG_OK;
}
}  // namespace

slg_status slg_plan_emit(slg_plan *p, int64_t *const *row_ptr, int32_t *const *row,
                         int32_t *const *col, int32_t *const *w, void *stream) {
    if (!p || !row_ptr || !col || !w) return fail(p ? p->ctx : nullptr, SLG_ERR_INVALID_ARG, "null argument");
    slg_context *ctx = p->ctx;
    const int K = p->prm.k;
    for (int k = 0; k < K; ++k) {
        if (!row_ptr[k]) return fail(ctx, SLG_ERR_INVALID_ARG, "null row_ptr[%d]", k);
        if (p->num_edges[k] > 0 && (!col[k] || !w[k]))
            return fail(ctx, SLG_ERR_INVALID_ARG, "null col/w for threshold %d", k);
    }
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    slg_status rc = order_after(ctx, st, p->st);  // after the plan's own work
    if (rc != SLG_OK) return rc;
    const int64_t zero[SLG_MAX_S] = {};
    rc = emit_range(p, 0, p->pr.m, 0, p->S, zero, row_ptr, row, col, w, st);
    if (rc != SLG_OK) return rc;
    return order_after(ctx, p->st, st);  // scratch is freed on the plan's stream
}

namespace {
// Rows [row_begin, row_end) of every L_s of the s-set, handed to `fn` in
// chunks. The rows phase runs once for the whole graph; the rest is planned
// and counted one row block at a time, so that the slot tables, boundary
// table and stores are bounded by the block, not by the graph: a block
// takes rows while its estimated scratch fits the count-store limit (the
// dense tier's survivors per 2-path are estimated from the blocks before).
// Inside a block, chunks are row ranges whose output fits chunk_bytes. Two
// sets of chunk buffers alternate: chunk c + 1 is emitted on `st` while the
// callback consumes chunk c on the consumer stream (the context's second
// stream when it has one), which waits for chunk c alone; a buffer set is
// written again only after the consumer's work on it.
slg_status stream_rows(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s, int64_t row_begin,
                       int64_t row_end, int64_t chunk_bytes, slg_chunk_fn fn, void *user, hipStream_t st) {
    if (!valid_s(s, num_s))
        return fail(ctx, SLG_ERR_INVALID_ARG, "s must be strictly increasing, s[0] >= 1, 1 <= num_s <= %d",
                    SLG_MAX_S);
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    slg_plan *p = plan_new(ctx, g, s, num_s, st);
    if (!p) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->blocks = true;
    const int K = num_s;
    const int64_t m = g->inc.num_hyperedges;
    Scratch bufs;  // chunk-cut scratch of the call
    bufs.st = st;
    bufs.arena = ctx->arena.get();
    hipEvent_t done[2] = {}, used[2] = {};  // chunk written / consumer finished, per buffer set
    hipStream_t cst = st;
    auto cleanup = [&](slg_status code) {
        if (cst != st) {  // the consumer's last work before the buffers go back
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
                (void)hipEventRecord(ev, cst);
                (void)hipStreamWaitEvent(st, ev, 0);
                (void)hipEventDestroy(ev);
            }
        }
        (void)hipStreamSynchronize(st);
        bufs.release();
        plan_free(p);
        for (int t = 0; t < 2; ++t) {
            if (done[t]) (void)hipEventDestroy(done[t]);
            if (used[t]) (void)hipEventDestroy(used[t]);
        }
        (void)hipGetLastError();  // the status returned is `code`
        return code;
    };
#define STREAM_HIP(call)                                                                            \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return cleanup(fail(ctx, e_ == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE, \
                                "%s: %s", #call, hipGetErrorString(e_)));                           \
    } while (0)
    // the rows phase plans the call's rows only (the E_s positions still
    // cover every row: partners lie anywhere after a row)
    p->plan_lo = row_begin;
    p->plan_hi = row_end;
    slg_status rc = plan_rows(p);
    if (rc != SLG_OK) return cleanup(rc);
    for (int t = 0; t < 2; ++t) {
        STREAM_HIP(hipEventCreateWithFlags(&done[t], hipEventDisableTiming));
        STREAM_HIP(hipEventCreateWithFlags(&used[t], hipEventDisableTiming));
    }
    if (ensure_aux(ctx)) cst = ctx->aux;
    const int64_t nr = row_end - row_begin;
    if (nr <= 0) return cleanup(SLG_OK);
    // every row's facts, to cut the blocks
    std::vector<int64_t> work(nr), bsz(nr);
    std::vector<int32_t> nsl(nr);
    std::vector<uint8_t> cls(nr);
    STREAM_HIP(hipMemcpyAsync(work.data(), p->b.work + row_begin, nr * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    STREAM_HIP(hipMemcpyAsync(bsz.data(), p->b.bsize_all + row_begin, nr * sizeof(int64_t), hipMemcpyDeviceToHost,
                              st));
    STREAM_HIP(hipMemcpyAsync(nsl.data(), p->b.nslots_all + row_begin, nr * sizeof(int32_t), hipMemcpyDeviceToHost,
                              st));
    STREAM_HIP(hipMemcpyAsync(cls.data(), p->b.rclass_all + row_begin, nr, hipMemcpyDeviceToHost, st));
    STREAM_HIP(hipStreamSynchronize(st));
    // block scratch: one dense store of fixed size for every block (half the
    // count-store limit; blocks are cut so that their survivors fit it), and
    // at most a quarter of the limit for the rest of a block's tables and
    // stores; sizes that repeat from block to block keep the block cache
    // from giving memory back and taking it again
    const int64_t budget = p->store_limit > 0 ? p->store_limit : (int64_t(8) << 30);
    bool any_dense = false;
    for (int64_t r = 0; r < nr && !any_dense; ++r) any_dense = cls[r] == kDense;
    if (any_dense && p->store_limit > 0) {
        p->dstore_fixed_cap = budget / 2 / 4;
        STREAM_HIP(p->scratch.get(&p->dstore_fixed, p->dstore_fixed_cap));
    }
    double dense_ratio = 0.125;  // survivors per dense 2-path, until a block has measured it
    int64_t base[SLG_MAX_S] = {};  // edges of the call before the current block
    int64_t *rp[2][SLG_MAX_S] = {};
    int32_t *ri[2][SLG_MAX_S] = {}, *rj[2][SLG_MAX_S] = {}, *rw[2][SLG_MAX_S] = {};
    int64_t cap_rows = -1, cap_e[SLG_MAX_S] = {};  // room of the chunk buffers
    int pending = -1;           // buffer set of a chunk emitted but not yet handed over
    int64_t pr0 = 0, pr1 = 0;   // its rows
    int64_t pe0[SLG_MAX_S] = {}, pne[SLG_MAX_S] = {};
    auto hand_over = [&]() -> slg_status {  // the pending chunk to the callback, on the consumer stream
        const int t = pending;
        pending = -1;
        if (hipEventSynchronize(done[t]) != hipSuccess ||
            (cst != st && hipStreamWaitEvent(cst, done[t], 0) != hipSuccess))
            return fail(ctx, SLG_ERR_DEVICE, "waiting for a chunk failed");
        for (int k = 0; k < K; ++k)
            if (fn(user, k, s[k], pr0, pr1, pe0[k], pne[k], rp[t][k], ri[t][k], rj[t][k], rw[t][k], cst) != 0)
                return fail(ctx, SLG_ERR_CANCELLED, "chunk callback stopped the stream at row %lld",
                            (long long)pr0);
        if (hipEventRecord(used[t], cst) != hipSuccess) return fail(ctx, SLG_ERR_DEVICE, "event record failed");
        return SLG_OK;
    };
    int64_t b0 = 0;
    int next_set = 0;
    while (b0 < nr) {
        // the block: rows while the estimated scratch fits
        const double per_dense = dense_ratio * 1.25;  // store entries per dense 2-path, with room
        // (less what the workgroups' unfilled chunks may take)
        const double dense_room =
            std::max(0.0, (double)p->dstore_fixed_cap - (double)dense_workgroups(p) * (double)kDenseChunk);
        double bytes = 0, entries = 0;
        int64_t b1 = b0;
        while (b1 < nr) {
            const int c = cls[b1];
            double r = (double)nsl[b1] * (24.0 + 16.0 * K) + 4.0 * (double)bsz[b1], d = 0;
            if (c == kHeavy || c == kHeavyWide) r += 4.0 * (double)work[b1];
            else if (c == kDense) d = per_dense * (double)work[b1];
            else if (c != kNone) r += 6.0 * (double)work[b1];
            if (b1 > b0 && (bytes + r > 0.25 * (double)budget || (dense_room > 0 && entries + d > dense_room)))
                break;
            bytes += r;
            entries += d;
            ++b1;
        }
        const int64_t R0 = row_begin + b0, R1 = row_begin + b1;
        // the consumer's use of both buffer sets ends before the block's
        // scratch (and the buffers in it) goes back
        if (pending >= 0 && (rc = hand_over()) != SLG_OK) return cleanup(rc);
        for (int t = 0; t < 2; ++t) STREAM_HIP(hipStreamWaitEvent(st, used[t], 0));
        rc = plan_block(p, R0, R1);
        if (rc != SLG_OK) return cleanup(rc);
        if (p->dense_two_paths > 0 && p->use_dstore)  // the room asked for, whether or not it fitted
            dense_ratio = std::max(1e-4, (double)p->dense_stored / (double)p->dense_two_paths);
        // output bytes before every row of the block; chunks are greedy row ranges
        const int64_t nb = R1 - R0;
        int64_t *dbytes;
        STREAM_HIP(p->scratch2.get(&dbytes, m + 1));
        STREAM_HIP(launch_row_bytes(m, p->slot_base, p->slot_off, p->S, K, dbytes, st));
        std::vector<int64_t> rbytes(nb + 1);
        STREAM_HIP(hipMemcpyAsync(rbytes.data(), dbytes + R0, (nb + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                                  st));
        STREAM_HIP(hipStreamSynchronize(st));
        std::vector<int64_t> cuts{R0};
        while (cuts.back() < R1) {
            const int64_t r0 = cuts.back();
            const int64_t limit = rbytes[r0 - R0] + chunk_bytes - 8 * K;  // room for the closing row_ptr entry
            int64_t r1 = R0 + (int64_t)(std::upper_bound(rbytes.begin() + (r0 - R0) + 1, rbytes.end(), limit) -
                                        rbytes.begin()) - 1;
            if (r1 <= r0)
                return cleanup(fail(ctx, SLG_ERR_OUT_OF_MEMORY,
                                    "row %lld alone needs %lld bytes, more than chunk_bytes", (long long)r0,
                                    (long long)(rbytes[r0 - R0 + 1] - rbytes[r0 - R0] + 8 * K)));
            cuts.push_back(r1);
        }
        // slot offsets of every threshold at every cut
        const int64_t nc = (int64_t)cuts.size();
        int64_t *dcuts, *doffs;
        STREAM_HIP(p->scratch2.get(&dcuts, nc));
        STREAM_HIP(p->scratch2.get(&doffs, nc * K));
        STREAM_HIP(hipMemcpyAsync(dcuts, cuts.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice, st));
        STREAM_HIP(launch_gather_offsets(dcuts, nc, p->slot_base, p->slot_off, p->S, K, doffs, st));
        std::vector<int64_t> offs(nc * K), sb(nc), parts(kNumHeavyLists * nc);
        // first slot of every cut row, then where each heavy list reaches it
        int64_t *dsb, *dparts;
        STREAM_HIP(p->scratch2.get(&dsb, nc));
        STREAM_HIP(p->scratch2.get(&dparts, kNumHeavyLists * nc));
        STREAM_HIP(launch_gather_i64(p->slot_base, dcuts, nc, dsb, st));
        for (int h = 0; h < kNumHeavyLists; ++h)
            STREAM_HIP(launch_list_cuts(p->heavy[h], p->list_count[kLightClasses + h], dsb, nc, dparts + h * nc, st));
        STREAM_HIP(hipMemcpyAsync(offs.data(), doffs, nc * K * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        STREAM_HIP(hipMemcpyAsync(sb.data(), dsb, nc * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        STREAM_HIP(hipMemcpyAsync(parts.data(), dparts, kNumHeavyLists * nc * sizeof(int64_t), hipMemcpyDeviceToHost,
                                  st));
        STREAM_HIP(hipStreamSynchronize(st));
        // two buffer sets for the largest chunk of every threshold so far:
        // they grow when a block needs more, and are kept otherwise
        int64_t max_rows = 0, max_e[SLG_MAX_S] = {};
        for (int64_t c = 0; c + 1 < nc; ++c) {
            max_rows = std::max(max_rows, cuts[c + 1] - cuts[c]);
            for (int k = 0; k < K; ++k) max_e[k] = std::max(max_e[k], offs[(c + 1) * K + k] - offs[c * K + k]);
        }
        bool grow = max_rows > cap_rows;
        for (int k = 0; k < K; ++k) grow |= max_e[k] > cap_e[k];
        if (grow) {
            bufs.release();  // after the work queued on st (which waited for the consumer)
            cap_rows = std::max(cap_rows, max_rows + max_rows / 4);
            for (int t = 0; t < 2; ++t)
                for (int k = 0; k < K; ++k) {
                    if (t == 0) cap_e[k] = std::max(cap_e[k], std::max<int64_t>(max_e[k] + max_e[k] / 4, 1));
                    STREAM_HIP(bufs.get(&rp[t][k], cap_rows + 1));
                    void *q[3];
                    for (int u = 0; u < 3; ++u) STREAM_HIP(bufs.get(&q[u], cap_e[k] * sizeof(int32_t)));
                    ri[t][k] = static_cast<int32_t *>(q[0]);
                    rj[t][k] = static_cast<int32_t *>(q[1]);
                    rw[t][k] = static_cast<int32_t *>(q[2]);
                }
        }
        for (int64_t c = 0; c + 1 < nc; ++c) {
            const int t = next_set;
            next_set ^= 1;
            STREAM_HIP(hipStreamWaitEvent(st, used[t], 0));  // the consumer is done with this set
            int64_t *rpk[SLG_MAX_S];
            int32_t *rik[SLG_MAX_S], *rjk[SLG_MAX_S], *rwk[SLG_MAX_S];
            for (int k = 0; k < K; ++k) {
                rpk[k] = rp[t][k];
                rik[k] = ri[t][k];
                rjk[k] = rj[t][k];
                rwk[k] = rw[t][k];
            }
            int64_t lists[2 * kNumHeavyLists];
            for (int h = 0; h < kNumHeavyLists; ++h) {
                lists[2 * h] = parts[h * nc + c];
                lists[2 * h + 1] = parts[h * nc + c + 1];
            }
            rc = emit_range(p, cuts[c], cuts[c + 1], sb[c], sb[c + 1], &offs[c * K], rpk, rik, rjk, rwk, st, lists);
            if (rc != SLG_OK) return cleanup(rc);
            STREAM_HIP(hipEventRecord(done[t], st));
            if (pending >= 0 && (rc = hand_over()) != SLG_OK) return cleanup(rc);
            pending = t;
            pr0 = cuts[c];
            pr1 = cuts[c + 1];
            for (int k = 0; k < K; ++k) {
                pe0[k] = base[k] + offs[c * K + k];
                pne[k] = offs[(c + 1) * K + k] - offs[c * K + k];
            }
        }
        for (int k = 0; k < K; ++k) base[k] += offs[(nc - 1) * K + k] - offs[k];
        b0 = b1;
    }
    if (pending >= 0 && (rc = hand_over()) != SLG_OK) return cleanup(rc);
#undef STREAM_HIP
    return cleanup(SLG_OK);
}
}  // namespace

slg_status slg_line_graph_stream(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                                 int64_t chunk_bytes, slg_chunk_fn fn, void *user, void *stream) {
    if (!ctx || !g || !fn || chunk_bytes <= 0) return fail(ctx, SLG_ERR_INVALID_ARG, "bad stream arguments");
    return stream_rows(ctx, g, s, num_s, 0, g->inc.num_hyperedges, chunk_bytes, fn, user,
                       static_cast<hipStream_t>(stream));
}

slg_status slg_line_graph_stream_rows(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                                      int64_t row_begin, int64_t row_end, int64_t chunk_bytes, slg_chunk_fn fn,
                                      void *user, void *stream) {
    if (!ctx || !g || !fn || chunk_bytes <= 0) return fail(ctx, SLG_ERR_INVALID_ARG, "bad stream arguments");
    if (row_begin < 0 || row_end < row_begin || row_end > g->inc.num_hyperedges)
        return fail(ctx, SLG_ERR_INVALID_ARG, "rows [%lld, %lld) outside [0, m)", (long long)row_begin,
                    (long long)row_end);
    return stream_rows(ctx, g, s, num_s, row_begin, row_end, chunk_bytes, fn, user,
                       static_cast<hipStream_t>(stream));
}

slg_status slg_work_prefix(slg_context *ctx, slg_graph *g, int32_t s_min, int64_t *prefix, void *stream) {
    if (!ctx || !g || !prefix || s_min < 1) return fail(ctx, SLG_ERR_INVALID_ARG, "bad work prefix arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    slg_plan *p = plan_new(ctx, g, &s_min, 1, st);
    if (!p) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    slg_status rc = plan_rows(p);
    if (rc == SLG_OK) {
        const int64_t m = g->inc.num_hyperedges;
        if (hipMemcpyAsync(prefix, p->b.work_pre, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = fail(ctx, SLG_ERR_DEVICE, "copying the work prefix failed");
    }
    plan_free(p);
    return rc;
}

slg_status slg_plan_stats(const slg_plan *p, int64_t *out, int32_t cap, int32_t *count) {
    if (!p || (!out && cap > 0) || cap < 0) return SLG_ERR_INVALID_ARG;
    int64_t vals[20];
    vals[0] = p->S;
    for (int c = 0; c < kLightClasses; ++c) vals[1 + c] = p->list_count[c];
    vals[8] = p->list_count[kLightClasses];
    vals[9] = p->list_count[kLightClasses + 1];
    vals[10] = p->two_paths;
    vals[11] = p->heavy_two_paths;
    vals[12] = p->nbounds;
    vals[13] = p->heavy_edges;
    vals[14] = p->stored_ranks;
    vals[15] = p->list_count[kLightClasses + 2];
    vals[16] = p->dense_two_paths;
    vals[17] = p->dense_edges;
    vals[18] = p->dense_kept;
    vals[19] = p->dense_stored > p->dense_kept ? 1 : 0;
    static_assert(kLightClasses == 7, "plan stats layout");
    int32_t n = cap < 20 ? cap : 20;
    for (int32_t t = 0; t < n; ++t) out[t] = vals[t];
    if (count) *count = n;
    return SLG_OK;
}

slg_status slg_context_set_timing(slg_context *ctx, int enable) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    ctx->timing = enable != 0;
    return SLG_OK;
}

slg_status slg_context_get_timing(slg_context *ctx, slg_stage_time *out, int32_t cap, int32_t *count) {
    if (!ctx || cap < 0 || (cap > 0 && !out)) return fail(ctx, SLG_ERR_INVALID_ARG, "bad timing query");
    for (const PendingTime &pt : ctx->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(pt.stop) == hipSuccess && hipEventElapsedTime(&ms, pt.start, pt.stop) == hipSuccess) {
            ctx->stage_ms[pt.stage] += ms;
            ctx->stage_launches[pt.stage] += 1;
        }
        ctx->event_pool.push_back(pt.start);
        ctx->event_pool.push_back(pt.stop);
    }
    ctx->pending.clear();
    int32_t n = 0;
    for (int sg = 0; sg < kNumStages; ++sg) {
        if (!ctx->stage_launches[sg]) continue;
        if (n < cap) {
            out[n].name = kStageNames[sg];
            out[n].launches = ctx->stage_launches[sg];
            out[n].milliseconds = ctx->stage_ms[sg];
        }
        ++n;
    }
    if (count) *count = n < cap ? n : cap;
    return SLG_OK;
}

slg_status slg_context_reset_timing(slg_context *ctx) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    int32_t n = 0;
    (void)slg_context_get_timing(ctx, nullptr, 0, &n);  // drain pending events
    for (int sg = 0; sg < kNumStages; ++sg) {
        ctx->stage_launches[sg] = 0;
        ctx->stage_ms[sg] = 0.0;
    }
    for (int t = 0; t < kNumWork; ++t) ctx->work[t] = 0;
    return SLG_OK;
}

slg_status slg_context_get_work(const slg_context *ctx, int64_t *out, int32_t cap, int32_t *count) {
    if (!ctx || cap < 0 || (cap > 0 && !out)) return SLG_ERR_INVALID_ARG;
    const int32_t n = cap < kNumWork ? cap : kNumWork;
    for (int32_t t = 0; t < n; ++t) out[t] = ctx->work[t];
    if (count) *count = n;
    return SLG_OK;
}

slg_status slg_plan_destroy(slg_plan *p) {
    if (!p) return SLG_ERR_INVALID_ARG;
    p->scratch2.release();
    p->scratch.release();
    delete p;
    return SLG_OK;
}

slg_status slg_context_set_count_store(slg_context *ctx, int64_t max_bytes, int64_t min_two_paths) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    if (max_bytes < 0 || min_two_paths < 0)
        return fail(ctx, SLG_ERR_INVALID_ARG, "max_bytes and min_two_paths must be >= 0");
    ctx->store_limit = max_bytes;
    ctx->store_min = min_two_paths;
    return SLG_OK;
}

slg_status slg_context_set_dense(slg_context *ctx, int32_t min_ratio, int32_t min_range) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    if (min_ratio < 0 || min_range < 0) return fail(ctx, SLG_ERR_INVALID_ARG, "min_ratio and min_range must be >= 0");
    ctx->dense_ratio = min_ratio;
    ctx->dense_min = min_range > 0 ? min_range : kDenseMinRange;
    return SLG_OK;
}

slg_status slg_context_set_list_shortfall(slg_context *ctx, int64_t entries) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    if (entries < 0) return fail(ctx, SLG_ERR_INVALID_ARG, "entries must be >= 0");
    ctx->list_shortfall = entries;
    return SLG_OK;
}

slg_status slg_context_set_tuning(slg_context *ctx, int32_t light_max, int64_t slot_work, int32_t heavy_grid) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    if (light_max < 0 || light_max > kLightMax || slot_work < 0 || heavy_grid < 0)
        return fail(ctx, SLG_ERR_INVALID_ARG, "tuning out of range (light_max <= %d)", kLightMax);
    ctx->light_max = light_max > 0 ? light_max : kLightMax;
    ctx->slot_work = slot_work > 0 ? slot_work : kSlotWork;
    ctx->heavy_grid = heavy_grid;
    return SLG_OK;
}


namespace {
slg_status batch_enqueue(slg_batch *b, hipStream_t st) {
    slg_plan *p = b->p;
    slg_context *ctx = b->ctx;
    SLG_HIP(ctx, enqueue_rows(p, st));
    SLG_HIP(ctx, enqueue_slots_count(p, st));
    const int64_t zero[SLG_MAX_S] = {};
    int64_t *rp[1] = {b->row_ptr};
    int32_t *ri[1] = {b->row}, *rj[1] = {b->col}, *rw[1] = {b->w};
    return emit_range(p, 0, p->pr.m, 0, p->S, zero, rp, ri, rj, rw, st);
}

void batch_free(slg_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->p) plan_free(b->p);
    for (void *q : b->owned) (void)hipFreeAsync(q, b->st);
    (void)hipStreamSynchronize(b->st);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    (void)hipGetLastError();
    delete b;
}
}  // namespace

slg_status slg_batch_create(slg_context *ctx, slg_graph *const *graphs, const int32_t *s, int32_t n,
                            void *stream, slg_batch **out) {
    if (!ctx || !graphs || !s || !out || n < 1 || n > 65535)
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad batch arguments (1 <= n <= 65535)");
    *out = nullptr;
    int32_t smin = INT32_MAX;
    for (int32_t g = 0; g < n; ++g) {
        if (!graphs[g] || s[g] < 1) return fail(ctx, SLG_ERR_INVALID_ARG, "graph %d: null or s < 1", g);
        smin = std::min(smin, s[g]);
    }
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    slg_batch *b = new (std::nothrow) slg_batch();
    if (!b) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->ctx = ctx;
    b->st = static_cast<hipStream_t>(stream);
    b->n = n;
    auto bail = [&](slg_status code) {
        batch_free(b);
        return code;
    };
#define BATCH_HIP(call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bail(fail(ctx, e_ == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE, \
                             "%s: %s", #call, hipGetErrorString(e_)));                              \
    } while (0)
    hipStream_t st = b->st;
    std::vector<UnionPart> parts(n);
    int64_t M = 0, N = 0, NNZ = 0, max_elems = 0;
    b->m_off.resize(n + 1);
    b->m_g.resize(n);
    for (int32_t g = 0; g < n; ++g) {
        const slg_incidence &gi = graphs[g]->inc;
        UnionPart &u = parts[g];
        u.he_ptr = gi.he_ptr;
        u.v_ptr = gi.v_ptr;
        u.he_idx = gi.he_idx;
        u.v_idx = gi.v_idx;
        u.m = gi.num_hyperedges;
        u.n = gi.num_vertices;
        u.nnz = gi.nnz;
        u.m_off = M;
        u.n_off = N;
        u.nnz_off = NNZ;
        u.s = s[g];
        u.pad_ = 0;
        b->m_off[g] = M;
        b->m_g[g] = u.m;
        M += u.m;
        N += u.n;
        NNZ += u.nnz;
        max_elems = std::max(max_elems, std::max(std::max(u.m + 1, u.n + 1), u.nnz));
    }
    b->m_off[n] = M;
    if (M >= (int64_t(1) << 31) || N >= (int64_t(1) << 31) || NNZ >= (int64_t(1) << 31))
        return bail(fail(ctx, SLG_ERR_OVERFLOW, "batch totals must stay below 2^31"));
    auto get = [&](void **q, size_t bytes) -> hipError_t {
        hipError_t e = hipMallocAsync(q, bytes ? bytes : 8, st);
        if (e == hipSuccess) b->owned.push_back(*q);
        return e;
    };
    int64_t *he_ptr, *v_ptr;
    int32_t *he_idx, *v_idx, *row_s, *row_base;
    UnionPart *dparts;
    BATCH_HIP(get(reinterpret_cast<void **>(&he_ptr), (M + 1) * sizeof(int64_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&v_ptr), (N + 1) * sizeof(int64_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&he_idx), NNZ * sizeof(int32_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&v_idx), NNZ * sizeof(int32_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&row_s), M * sizeof(int32_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&row_base), M * sizeof(int32_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&dparts), n * sizeof(UnionPart)));
    BATCH_HIP(hipMemcpyAsync(dparts, parts.data(), n * sizeof(UnionPart), hipMemcpyHostToDevice, st));
    BATCH_HIP(launch_union(dparts, n, max_elems, he_ptr, he_idx, v_ptr, v_idx, row_s, row_base, st));
    BATCH_HIP(hipStreamSynchronize(st));  // `parts` leaves scope; union ready
    b->ug.ctx = ctx;
    b->ug.inc = {N, M, NNZ, he_ptr, he_idx, v_ptr, v_idx};
    b->p = plan_new(ctx, &b->ug, &smin, 1, st);
    if (!b->p) return bail(fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed"));
    b->p->pr.row_s = row_s;
    b->p->prm.row_s = row_s;
    b->p->prm.row_base = row_base;
    slg_status rc = plan_build(b->p);
    if (rc != SLG_OK) return bail(rc);
    b->edges = b->p->num_edges[0];
    BATCH_HIP(get(reinterpret_cast<void **>(&b->row_ptr), (M + 1) * sizeof(int64_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&b->row), b->edges * sizeof(int32_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&b->col), b->edges * sizeof(int32_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&b->w), b->edges * sizeof(int32_t)));
    const int64_t zero[SLG_MAX_S] = {};
    int64_t *rp[1] = {b->row_ptr};
    int32_t *ri[1] = {b->row}, *rj[1] = {b->col}, *rw[1] = {b->w};
    rc = emit_range(b->p, 0, M, 0, b->p->S, zero, rp, ri, rj, rw, st);
    if (rc != SLG_OK) return bail(rc);
    // global edge offset of every graph's first row
    int64_t *didx, *doff;
    BATCH_HIP(get(reinterpret_cast<void **>(&didx), (n + 1) * sizeof(int64_t)));
    BATCH_HIP(get(reinterpret_cast<void **>(&doff), (n + 1) * sizeof(int64_t)));
    BATCH_HIP(hipMemcpyAsync(didx, b->m_off.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    BATCH_HIP(launch_gather_i64(b->row_ptr, didx, n + 1, doff, st));
    b->edge_off.resize(n + 1);
    BATCH_HIP(hipMemcpyAsync(b->edge_off.data(), doff, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BATCH_HIP(hipStreamSynchronize(st));
    BATCH_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
#undef BATCH_HIP
    *out = b;
    return SLG_OK;
}

slg_status slg_batch_run(slg_batch *b, int32_t use_graph, void *stream) {
    if (!b) return SLG_ERR_INVALID_ARG;
    slg_context *ctx = b->ctx;
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!use_graph) return batch_enqueue(b, st);
    if (!b->exec) {  // capture the whole device path once
        slg_status rc = order_after(ctx, b->cap, b->st);
        if (rc != SLG_OK) return rc;
        SLG_HIP(ctx, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        ctx->capturing = true;
        rc = batch_enqueue(b, b->cap);
        ctx->capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap, &graph);
        if (rc != SLG_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(ctx, SLG_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        b->graph = graph;
        SLG_HIP(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    SLG_HIP(ctx, hipGraphLaunch(b->exec, st));
    return SLG_OK;
}

slg_status slg_batch_info(const slg_batch *b, int64_t *num_edges, int64_t *two_paths, int64_t *rows) {
    if (!b) return SLG_ERR_INVALID_ARG;
    if (num_edges) *num_edges = b->edges;
    if (two_paths) *two_paths = b->p->two_paths;
    if (rows) *rows = b->m_off[b->n];
    return SLG_OK;
}

slg_status slg_batch_result(const slg_batch *b, int32_t g, int64_t *edge_begin, int64_t *num_edges,
                            const int64_t **row_ptr, const int32_t **row, const int32_t **col,
                            const int32_t **w) {
    if (!b || g < 0 || g >= b->n) return SLG_ERR_INVALID_ARG;
    const int64_t e0 = b->edge_off[g];
    if (edge_begin) *edge_begin = e0;
    if (num_edges) *num_edges = b->edge_off[g + 1] - e0;
    if (row_ptr) *row_ptr = b->row_ptr + b->m_off[g];
    if (row) *row = b->row + e0;
    if (col) *col = b->col + e0;
    if (w) *w = b->w + e0;
    return SLG_OK;
}

slg_status slg_batch_destroy(slg_batch *b) {
    if (!b) return SLG_ERR_INVALID_ARG;
    batch_free(b);
    return SLG_OK;
}

slg_status slg_line_graph(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                          void *stream, slg_result **out) {
    if (!ctx || !out) return fail(ctx, SLG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    slg_plan *p = nullptr;
    slg_status rc = slg_plan_create(ctx, g, s, num_s, stream, &p);
    if (rc != SLG_OK) return rc;
    slg_result *r = new (std::nothrow) slg_result();
    if (!r) {
        slg_plan_destroy(p);
        return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    r->ctx = ctx;
    r->st = static_cast<hipStream_t>(stream);
    if (!ctx->has_alloc) r->arena = ctx->arena;
    r->k = num_s;
    r->m = g->inc.num_hyperedges;
    r->two_paths = p->two_paths;
    auto get = [&](void **ptr, size_t bytes) -> bool {
        if (bytes == 0) bytes = 8;
        if (ctx->has_alloc) {
            *ptr = ctx->alloc.alloc(ctx->alloc.user, bytes, stream);
        } else if (ctx->arena->get(ptr, bytes, r->st) != hipSuccess) {
            *ptr = nullptr;
        }
        if (*ptr) r->owned.push_back(*ptr);
        return *ptr != nullptr;
    };
    bool ok = true;
    for (int k = 0; k < num_s && ok; ++k) {
        const int64_t e = p->num_edges[k];
        r->num_edges[k] = e;
        ok = get(reinterpret_cast<void **>(&r->row_ptr[k]), (r->m + 1) * sizeof(int64_t)) &&
             get(reinterpret_cast<void **>(&r->row[k]), e * sizeof(int32_t)) &&
             get(reinterpret_cast<void **>(&r->col[k]), e * sizeof(int32_t)) &&
             get(reinterpret_cast<void **>(&r->w[k]), e * sizeof(int32_t));
    }
    if (ok) rc = slg_plan_emit(p, r->row_ptr, r->row, r->col, r->w, stream);
    slg_plan_destroy(p);
    if (!ok || rc != SLG_OK) {
        slg_result_free(r);
        return ok ? rc : fail(ctx, SLG_ERR_OUT_OF_MEMORY, "result allocation failed");
    }
    *out = r;
    return SLG_OK;
}

}  // extern "C"

namespace slg {

int context_device(const slg_context *ctx) { return ctx->device; }
const slg_context *graph_context(const slg_graph *g) { return g->ctx; }
slg_status set_error(slg_context *ctx, slg_status code, const char *msg) { return fail(ctx, code, "%s", msg); }

void share_arena(slg_context *ctx, const std::shared_ptr<Arena> &arena) { ctx->arena = arena; }

void copy_tuning(slg_context *dst, const slg_context *src) {
    dst->light_max = src->light_max;
    dst->slot_work = src->slot_work;
    dst->heavy_grid = src->heavy_grid;
    dst->store_limit = src->store_limit;
    dst->store_min = src->store_min;
    dst->dense_ratio = src->dense_ratio;
    dst->dense_min = src->dense_min;
}

slg_status serve_query(slg_context *wctx, slg_graph *g, const int32_t *s, int32_t num_s, hipStream_t st,
                       const ReserveFn &reserve, const std::shared_ptr<ServeCore> &core, slg_result **out,
                       uint64_t *scratch_bytes, uint64_t *output_bytes) {
    *out = nullptr;
    *scratch_bytes = 0;
    *output_bytes = 0;
    if (!g || !valid_s(s, num_s)) return fail(wctx, SLG_ERR_INVALID_ARG, "bad graph or s-set");
    SLG_HIP(wctx, hipSetDevice(wctx->device));
    slg_plan *p = plan_new(wctx, g, s, num_s, st);
    if (!p) return fail(wctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->reserve = &reserve;
    slg_status rc = plan_build(p);
    *scratch_bytes = p->reserved;
    if (rc != SLG_OK) {
        plan_free(p);
        return rc;
    }
    slg_result *r = new (std::nothrow) slg_result();
    if (!r) {
        plan_free(p);
        return fail(wctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    r->st = st;
    r->k = num_s;
    r->m = g->inc.num_hyperedges;
    r->two_paths = p->two_paths;
    AllocList outs;
    for (int k = 0; k < num_s; ++k) {
        r->num_edges[k] = p->num_edges[k];
        outs.add(&r->row_ptr[k], r->m + 1);
        outs.add(&r->row[k], p->num_edges[k]);
        outs.add(&r->col[k], p->num_edges[k]);
        outs.add(&r->w[k], p->num_edges[k]);
    }
    auto drop = [&](slg_status code) {
        wctx->arena->put(r->owned, st);
        delete r;
        plan_free(p);  // also waits for the stream
        return code;
    };
    if (!reserve(outs.bytes)) return drop(fail(wctx, SLG_ERR_OUT_OF_MEMORY, "device-memory budget refused"));
    *output_bytes = outs.bytes;
    for (const auto &a : outs.items) {
        hipError_t e = wctx->arena->get(a.first, a.second, st);
        if (e != hipSuccess)
            return drop(fail(wctx, e == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE,
                             "output allocation: %s", hipGetErrorString(e)));
        r->owned.push_back(*a.first);
    }
    rc = slg_plan_emit(p, r->row_ptr, r->row, r->col, r->w, st);
    if (rc != SLG_OK) return drop(rc);
    plan_free(p);  // frees the scratch on `st` and waits for the stream: outputs are complete
    r->arena = wctx->arena;
    r->core = core;
    r->bytes = outs.bytes;
    *out = r;
    return SLG_OK;
}

}  // namespace slg

extern "C" {

slg_status slg_components(slg_context *ctx, slg_graph *g, int32_t s, const int32_t *row, const int32_t *col,
                          int64_t num_edges, int32_t *labels, int64_t *num_components, void *stream) {
    if (!ctx || !g || !labels || s < 1 || num_edges < 0 || (num_edges > 0 && (!row || !col)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad components arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t m = g->inc.num_hyperedges;
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int64_t *dev = nullptr;  // [0] roots, [1] error flags
    int32_t *parent = nullptr;
    SLG_HIP(ctx, sc.get(&dev, 2));
    SLG_HIP(ctx, sc.get(&parent, m));
    SLG_HIP(ctx, launch_fill_i64(dev, 2, 0, st));
    SLG_HIP(ctx, launch_cc_init(g->inc.he_ptr, m, s, parent, st));
    SLG_HIP(ctx, launch_cc_hook(row, col, num_edges, m, parent, reinterpret_cast<int *>(dev + 1), st));
    SLG_HIP(ctx, launch_cc_finish(m, parent, labels, reinterpret_cast<unsigned long long *>(dev), st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, dev, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    sc.release();
    const int64_t err = ctx->pinned[1];
    if (err & 4) return fail(ctx, SLG_ERR_INVALID_ARG, "an edge names a hyperedge id outside [0, m)");
    if (err & 2) return fail(ctx, SLG_ERR_INVALID_ARG, "an edge joins a hyperedge with fewer than s vertices");
    if (err & 1) return fail(ctx, SLG_ERR_DEVICE, "internal error: a union step did not settle");
    if (num_components) *num_components = ctx->pinned[0];
    return SLG_OK;
}

slg_status slg_components_noalloc(slg_context *ctx, slg_graph *g, int32_t s, const int32_t *row,
                                  const int32_t *col, int64_t num_edges, int32_t *labels, int64_t *num_components,
                                  void *stream) {
    if (!ctx || !g || !labels || s < 1 || num_edges < 0 || (num_edges > 0 && (!row || !col)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad components arguments");
    const int64_t m = g->inc.num_hyperedges;
    if (m > kNoAllocRows)
        return fail(ctx, SLG_ERR_INVALID_ARG,
                    "m = %lld exceeds the %lld hyperedges the fixed scratch holds (use slg_components)",
                    (long long)m, (long long)kNoAllocRows);
    if (!ctx->noalloc)
        return fail(ctx, SLG_ERR_DEVICE, "fixed scratch unavailable: %s", hipGetErrorString(ctx->noalloc_err));
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the same kernels as slg_components, on the device's fixed array: the
    // two counters are cleared here and every parent is written by cc_init
    int64_t *dev = static_cast<int64_t *>(ctx->noalloc);  // [0] roots, [1] error flags
    int32_t *parent = reinterpret_cast<int32_t *>(dev + 2);
    SLG_HIP(ctx, launch_fill_i64(dev, 2, 0, st));
    SLG_HIP(ctx, launch_cc_init(g->inc.he_ptr, m, s, parent, st));
    SLG_HIP(ctx, launch_cc_hook(row, col, num_edges, m, parent, reinterpret_cast<int *>(dev + 1), st));
    SLG_HIP(ctx, launch_cc_finish(m, parent, labels, reinterpret_cast<unsigned long long *>(dev), st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, dev, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    const int64_t err = ctx->pinned[1];
    if (err & 4) return fail(ctx, SLG_ERR_INVALID_ARG, "an edge names a hyperedge id outside [0, m)");
    if (err & 2) return fail(ctx, SLG_ERR_INVALID_ARG, "an edge joins a hyperedge with fewer than s vertices");
    if (err & 1) return fail(ctx, SLG_ERR_DEVICE, "internal error: a union step did not settle");
    if (num_components) *num_components = ctx->pinned[0];
    return SLG_OK;
}

slg_status slg_squeeze(slg_context *ctx, int64_t m, int32_t *row, int32_t *col, int64_t num_edges, int32_t remap,
                       int32_t *new_id, int64_t *num_kept, void *stream) {
    if (!ctx || !new_id || m < 0 || m >= (int64_t(1) << 31) || num_edges < 0 || (num_edges > 0 && (!row || !col)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad squeeze arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int32_t *flag = nullptr;
    int64_t *pre = nullptr, *part = nullptr, *err = nullptr;
    SLG_HIP(ctx, sc.get(&flag, m));
    SLG_HIP(ctx, sc.get(&pre, m + 1));
    SLG_HIP(ctx, sc.get(&part, scan_partials_size(m)));
    SLG_HIP(ctx, sc.get(&err, 1));
    SLG_HIP(ctx, launch_fill_i32(flag, m, 0, st));
    SLG_HIP(ctx, launch_fill_i64(err, 1, 0, st));
    SLG_HIP(ctx, launch_mark_ends(row, col, num_edges, m, flag, reinterpret_cast<int *>(err), st));
    SLG_HIP(ctx, launch_exclusive_scan_i32(flag, m, pre, part, st));
    SLG_HIP(ctx, launch_squeeze_ids(m, flag, pre, new_id, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned + 1, pre + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    if (ctx->pinned[0] & 4) {
        sc.release();
        return fail(ctx, SLG_ERR_INVALID_ARG, "an edge names a hyperedge id outside [0, m)");
    }
    if (remap) SLG_HIP(ctx, launch_remap_edges(row, col, num_edges, new_id, st));
    sc.release();
    if (num_kept) *num_kept = ctx->pinned[1];
    return SLG_OK;
}


slg_status slg_symmetrize(slg_context *ctx, int64_t m, const int64_t *row_ptr, const int32_t *row,
                          const int32_t *col, const int32_t *w, int64_t num_edges, int64_t *sym_ptr,
                          int32_t *sym_col, int32_t *sym_w, void *stream) {
    if (!ctx || m < 0 || m >= (int64_t(1) << 31) || num_edges < 0 || !row_ptr || !sym_ptr ||
        (num_edges > 0 && (!row || !col || !sym_col)) || (!w) != (!sym_w))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad symmetrize arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = num_edges;
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int64_t *err = nullptr, *lower_ptr = nullptr;
    const int32_t *sorted[3] = {};
    SLG_HIP(ctx, sc.get(&err, 1));
    SLG_HIP(ctx, sc.get(&lower_ptr, m + 1));
    SLG_HIP(ctx, launch_fill_i64(err, 1, 0, st));
    SLG_HIP(ctx, launch_check_upper(row_ptr, row, col, n, m, reinterpret_cast<int *>(err), st));
    // the upper triangle sorted by column (stable: rows stay ascending),
    // left in the sort's own buffers
    SLG_HIP(ctx, sort_pairs(sc, col, row, w, n, bits_for(m), nullptr, nullptr, nullptr, st, sorted));
    SLG_HIP(ctx, launch_symmetric(sorted[0], sorted[1], sorted[2], row_ptr, row, col, w, n, m, lower_ptr, sym_ptr,
                                  sym_col, sym_w, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    sc.release();
    if (ctx->pinned[0] & 1)
        return fail(ctx, SLG_ERR_INVALID_ARG, "input is not an upper triangle sorted by (row, col)");
    return SLG_OK;
}

slg_status slg_digest(slg_context *ctx, const int32_t *row, const int32_t *col, const int32_t *w,
                      int64_t num_edges, uint64_t *out, void *stream) {
    if (!ctx || !out || num_edges < 0 || (num_edges > 0 && (!row || !col || !w)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad digest arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int64_t *acc = nullptr;
    SLG_HIP(ctx, sc.get(&acc, 3));
    SLG_HIP(ctx, launch_fill_i64(acc, 3, 0, st));
    SLG_HIP(ctx, launch_digest(row, col, w, num_edges, reinterpret_cast<unsigned long long *>(acc), st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, acc, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    for (int t = 0; t < 3; ++t) out[t] = static_cast<uint64_t>(ctx->pinned[t]);
    return SLG_OK;
}

slg_status slg_relabel_order(slg_context *ctx, slg_graph *g, int32_t descending, int32_t *order, void *stream) {
    if (!ctx || !g || !order) return fail(ctx, SLG_ERR_INVALID_ARG, "bad relabel arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t m = g->inc.num_hyperedges, n = g->inc.num_vertices;
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int32_t *key = nullptr, *id = nullptr, *skey = nullptr;
    SLG_HIP(ctx, sc.get(&key, m));
    SLG_HIP(ctx, sc.get(&id, m));
    SLG_HIP(ctx, sc.get(&skey, m));
    SLG_HIP(ctx, launch_size_keys(g->inc.he_ptr, m, n, descending ? 1 : 0, key, id, st));
    // sizes lie in [0, n]: stable, so equal sizes keep their id order
    SLG_HIP(ctx, sort_pairs(sc, key, id, nullptr, m, bits_for(n + 1), skey, order, nullptr, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    return SLG_OK;
}

slg_status slg_toplexes(slg_context *ctx, slg_graph *g, const int32_t *row, const int32_t *col, const int32_t *w,
                        int64_t num_edges, int32_t *toplexes, int64_t *num_toplexes, void *stream) {
    if (!ctx || !g || !toplexes || num_edges < 0 || (num_edges > 0 && (!row || !col || !w)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad toplex arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t m = g->inc.num_hyperedges;
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int32_t *drop = nullptr, *keep = nullptr;
    int64_t *pre = nullptr, *part = nullptr, *err = nullptr;
    SLG_HIP(ctx, sc.get(&drop, m));
    SLG_HIP(ctx, sc.get(&keep, m));
    SLG_HIP(ctx, sc.get(&pre, m + 1));
    SLG_HIP(ctx, sc.get(&part, scan_partials_size(m)));
    SLG_HIP(ctx, sc.get(&err, 1));
    SLG_HIP(ctx, launch_fill_i64(err, 1, 0, st));
    SLG_HIP(ctx, launch_fill_i64(pre + m, 1, 0, st));  // m = 0: the count
    SLG_HIP(ctx, launch_toplex_flags(row, col, w, num_edges, g->inc.he_ptr, m, drop, keep,
                                     reinterpret_cast<int *>(err), st));
    SLG_HIP(ctx, launch_exclusive_scan_i32(keep, m, pre, part, st));
    SLG_HIP(ctx, launch_compact_ids(keep, pre, m, toplexes, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned + 1, pre + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    sc.release();
    if (ctx->pinned[0] & 1) return fail(ctx, SLG_ERR_INVALID_ARG, "an edge names an id outside [0, m) or a loop");
    if (ctx->pinned[0] & 2)
        return fail(ctx, SLG_ERR_INVALID_ARG, "an overlap exceeds a hyperedge size: not the edges of L_1");
    if (num_toplexes) *num_toplexes = ctx->pinned[1];
    return SLG_OK;
}

slg_status slg_select(slg_context *ctx, slg_graph *g, const int32_t *order, int64_t count, int64_t *he_ptr,
                      int32_t *he_idx, int64_t *v_ptr, int32_t *v_idx, int64_t *nnz, void *stream) {
    if (!ctx || !g || count < 0 || !he_ptr || !v_ptr || (count > 0 && !order) ||
        (g->inc.nnz > 0 && (!he_idx || !v_idx)))
        return fail(ctx, SLG_ERR_INVALID_ARG, "bad select arguments");
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const slg_incidence &inc = g->inc;
    const int64_t m = inc.num_hyperedges, n = inc.num_vertices;
    if (count > m) return fail(ctx, SLG_ERR_INVALID_ARG, "more hyperedges selected than the graph has");
    Scratch sc;
    sc.st = st;
    sc.arena = ctx->arena.get();
    int32_t *seen = nullptr, *row_of = nullptr, *skey = nullptr;
    int64_t *sizes = nullptr, *part = nullptr, *err = nullptr;
    SLG_HIP(ctx, sc.get(&seen, m));
    SLG_HIP(ctx, sc.get(&sizes, count));
    SLG_HIP(ctx, sc.get(&part, scan_partials_size(count)));
    SLG_HIP(ctx, sc.get(&err, 1));
    SLG_HIP(ctx, launch_fill_i64(err, 1, 0, st));
    SLG_HIP(ctx, launch_fill_i32(seen, m, 0, st));
    SLG_HIP(ctx, launch_fill_i64(he_ptr + count, 1, 0, st));  // count = 0: an empty graph
    SLG_HIP(ctx, launch_select_sizes(order, count, inc.he_ptr, m, seen, sizes, reinterpret_cast<int *>(err), st));
    SLG_HIP(ctx, launch_exclusive_scan_i64(sizes, count, he_ptr, part, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned, err, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipMemcpyAsync(ctx->pinned + 1, he_ptr + count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    const int64_t bad = ctx->pinned[0], nz = ctx->pinned[1];
    if (bad & 1) return fail(ctx, SLG_ERR_INVALID_ARG, "order names an id outside [0, m)");
    if (bad & 2) return fail(ctx, SLG_ERR_INVALID_ARG, "order names a hyperedge twice");
    if (nz > 0) {
        SLG_HIP(ctx, sc.get(&row_of, nz));
        SLG_HIP(ctx, sc.get(&skey, nz));
    }
    SLG_HIP(ctx, launch_select_rows(order, count, inc.he_ptr, inc.he_idx, m, he_ptr, he_idx, row_of, st));
    // vertex lists: the new incidences sorted by vertex, rows ascending
    SLG_HIP(ctx, sort_pairs(sc, he_idx, row_of, nullptr, nz, bits_for(n), skey, v_idx, nullptr, st));
    SLG_HIP(ctx, launch_key_bounds(skey, nz, n, v_ptr, st));
    SLG_HIP(ctx, hipStreamSynchronize(st));
    sc.release();
    if (nnz) *nnz = nz;
    return SLG_OK;
}

slg_status slg_result_info(const slg_result *r, int32_t k, int64_t *num_edges, int64_t *two_paths) {
    if (!r || k < 0 || k >= r->k) return SLG_ERR_INVALID_ARG;
    if (num_edges) *num_edges = r->num_edges[k];
    if (two_paths) *two_paths = r->two_paths;
    return SLG_OK;
}

slg_status slg_result_coo(const slg_result *r, int32_t k, const int32_t **i, const int32_t **j,
                          const int32_t **w) {
    if (!r || k < 0 || k >= r->k) return SLG_ERR_INVALID_ARG;
    if (i) *i = r->row[k];
    if (j) *j = r->col[k];
    if (w) *w = r->w[k];
    return SLG_OK;
}

slg_status slg_result_csr(const slg_result *r, int32_t k, const int64_t **row_ptr,
                          const int32_t **col, const int32_t **w) {
    if (!r || k < 0 || k >= r->k) return SLG_ERR_INVALID_ARG;
    if (row_ptr) *row_ptr = r->row_ptr[k];
    if (col) *col = r->col[k];
    if (w) *w = r->w[k];
    return SLG_OK;
}

slg_status slg_result_free(slg_result *r) {
    if (!r) return SLG_ERR_INVALID_ARG;
    if (r->core) {  // a served result: reusable after the work queued on the null stream
        r->arena->put(r->owned, nullptr);
        r->core->release(r->bytes, true);
        delete r;
        return SLG_OK;
    }
    if (r->arena) {
        r->arena->put(r->owned, r->st);
    } else {
        slg_context *ctx = r->ctx;
        for (void *ptr : r->owned) ctx->alloc.release(ctx->alloc.user, ptr, r->st);
    }
    delete r;
    return SLG_OK;
}

}  // extern "C"
