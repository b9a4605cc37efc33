// Host side of the C ABI declared in include/slg.h: contexts, graph
// registration and validation, the plan (prune -> work estimate -> count ->
// prefix sums), the emit pass and the one-shot result object.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "slg.h"
#include "slg_internal.h"

using namespace slg;

namespace {
enum Stage {
    kStPrune, kStRowPlan, kStPlanScans, kStSlots, kStBounds, kStCountLight, kStCountHeavy,
    kStCountHeavyWide, kStCountScans, kStEmitLight, kStEmitHeavy, kStEmitHeavyWide, kStRowPtr, kNumStages
};
const char *const kStageNames[kNumStages] = {
    "prune", "row_plan", "plan_scans", "slots", "bounds", "count_light", "count_heavy",
    "count_heavy_wide", "count_scans", "emit_light", "emit_heavy", "emit_heavy_wide", "row_ptr"};
struct PendingTime {
    int stage;
    hipEvent_t start, stop;
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
    uint64_t budget = 0;
    bool has_alloc = false;
    slg_allocator alloc{};
    std::string last_error;
    int64_t *pinned = nullptr;  // host staging for readbacks
};

struct slg_graph {
    slg_context *ctx = nullptr;
    slg_incidence inc{};
};

namespace {

constexpr int kPinnedSlots = 64;

// Layout of the plan's small device counter block (int64 entries).
constexpr int kCntClass = 0;                    // kNumLists: rows / slots per tier list
constexpr int kCntErr = kCntClass + kNumLists;  // malformed-input flag (low 32 bits)
constexpr int kCntFill = kCntErr + 1;           // kNumLists: append cursors of the tier lists
constexpr int kCntHeavyWork = kCntFill + kNumLists;  // 2-paths in heavy rows
constexpr int kCntTotal = kCntHeavyWork + 1;
static_assert(kCntTotal <= 32, "counter block");
// Host staging slots for readbacks.
constexpr int kHbSlots = kCntTotal;      // slot table size, then 2-paths, boundary entries
constexpr int kHbEdges = 40;             // SLG_MAX_S edge totals
constexpr int kHbHeavyEdges = kHbEdges + SLG_MAX_S;
static_assert(kHbSlots + 3 <= kHbEdges && kHbHeavyEdges + 1 < kPinnedSlots, "pinned staging layout");

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
    std::vector<void *> ptrs;
    hipError_t get(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 8;
        hipError_t e = hipMallocAsync(p, bytes, st);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    template <typename T>
    hipError_t get(T **p, size_t count) {
        return get(reinterpret_cast<void **>(p), count * sizeof(T));
    }
    void release() {
        for (void *p : ptrs) (void)hipFreeAsync(p, st);
        ptrs.clear();
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
        if (!ctx || !ctx->timing) return;
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

}  // namespace

struct slg_plan {
    slg_context *ctx = nullptr;
    slg_graph *g = nullptr;
    hipStream_t st = nullptr;
    EmitParams prm{};
    Pruned pr{};
    Scratch scratch;
    int64_t *slot_base = nullptr;  // [m+1]
    int64_t S = 0;                 // number of slots
    Slots slots{};
    int32_t *bounds = nullptr;
    int64_t *tickets = nullptr;    // work counters of the persistent heavy launches
    HeavyDesc *heavy[2] = {};      // heavy and heavy-wide slot descriptors
    int32_t *lists[kNumLists] = {};
    int64_t list_count[kNumLists] = {};
    int64_t *slot_cnt = nullptr;   // [K][S]
    int64_t *slot_off = nullptr;   // [K][S+1]
    int64_t two_paths = 0;
    int64_t heavy_two_paths = 0;
    int64_t heavy_edges = 0;
    int64_t nbounds = 0;
    int64_t num_edges[SLG_MAX_S] = {};
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
};

extern "C" {

const char *slg_version(void) { return "slg 0.1.0 (gfx950)"; }

slg_status slg_context_create(int device, uint64_t mem_budget_bytes, const slg_allocator *alloc,
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
    // keep freed scratch in the stream-ordered pool between calls
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    *out = ctx;
    return SLG_OK;
}

slg_status slg_context_destroy(slg_context *ctx) {
    if (!ctx) return SLG_ERR_INVALID_ARG;
    for (const PendingTime &pt : ctx->pending) {
        (void)hipEventSynchronize(pt.stop);
        ctx->event_pool.push_back(pt.start);
        ctx->event_pool.push_back(pt.stop);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
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
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (flags & SLG_VALIDATE) {
        Scratch sc;
        sc.st = st;
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
        if (code & 2) return fail(ctx, SLG_ERR_INVALID_GRAPH, "CSR pointer array malformed");
        if (code & 4) return fail(ctx, SLG_ERR_INVALID_GRAPH, "CSR row holds an out-of-range or repeated id");
        if (code & 8) return fail(ctx, SLG_ERR_INVALID_GRAPH, "vertex CSR is not the transpose");
    }
    slg_graph *g = new (std::nothrow) slg_graph();
    if (!g) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    g->ctx = ctx;
    g->inc = *inc;
    *out = g;
    return SLG_OK;
}

slg_status slg_graph_release(slg_graph *g) {
    if (!g) return SLG_ERR_INVALID_ARG;
    delete g;
    return SLG_OK;
}

slg_status slg_plan_create(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                           void *stream, slg_plan **out) {
    if (!ctx || !g || !out) return fail(ctx, SLG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (!valid_s(s, num_s))
        return fail(ctx, SLG_ERR_INVALID_ARG, "s must be strictly increasing, s[0] >= 1, 1 <= num_s <= %d",
                    SLG_MAX_S);
    SLG_HIP(ctx, hipSetDevice(ctx->device));
    slg_plan *p = new (std::nothrow) slg_plan();
    if (!p) return fail(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->ctx = ctx;
    p->g = g;
    p->st = static_cast<hipStream_t>(stream);
    p->scratch.st = p->st;
    p->prm.k = num_s;
    for (int t = 0; t < num_s; ++t) p->prm.s[t] = s[t];
    slg_status rc = SLG_OK;
    auto bail = [&](slg_status code) {
        p->scratch.release();
        (void)hipStreamSynchronize(p->st);
        delete p;
        return code;
    };
#define PLAN_HIP(call)                                                                             \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bail(fail(ctx, e_ == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE, \
                             "%s: %s", #call, hipGetErrorString(e_)));                              \
    } while (0)

    const slg_incidence &inc = g->inc;
    const int64_t m = inc.num_hyperedges, n = inc.num_vertices, nnz = inc.nnz;
    const int32_t s_min = s[0];
    hipStream_t st = p->st;
    Scratch &sc = p->scratch;

    // K1: vertex lists restricted to E_{s_min}
    Pruned &pr = p->pr;
    pr.m = m;
    pr.n = n;
    pr.nnz = nnz;
    pr.he_ptr = inc.he_ptr;
    pr.he_idx = inc.he_idx;
    if (s_min > 1 && nnz > 0) {
        uint8_t *flag;
        int64_t *pos, *part;
        int64_t *vs_ptr;
        int32_t *vs_idx;
        PLAN_HIP(sc.get(&flag, nnz));
        PLAN_HIP(sc.get(&pos, nnz + 1));
        PLAN_HIP(sc.get(&part, scan_partials_size(nnz)));
        PLAN_HIP(sc.get(&vs_ptr, n + 1));
        PLAN_HIP(sc.get(&vs_idx, nnz));
        StageTimer tm(ctx, kStPrune, st);
        PLAN_HIP(launch_keep_incidence(nnz, inc.v_idx, inc.he_ptr, m, s_min, flag, st));
        PLAN_HIP(launch_exclusive_scan_u8(flag, nnz, pos, part, st));
        PLAN_HIP(launch_compact_vertex_lists(n, nnz, inc.v_ptr, inc.v_idx, flag, pos, vs_ptr, vs_idx, st));
        pr.vs_ptr = vs_ptr;
        pr.vs_idx = vs_idx;
    } else {
        pr.vs_ptr = inc.v_ptr;
        pr.vs_idx = inc.v_idx;
    }

    // K2: tails, 2-path work and slot counts per row
    int32_t *tail_beg, *jmax, *nslots;
    int64_t *work, *work_pre, *counters, *part_m, *bsize, *bbase;
    uint8_t *rclass;
    PLAN_HIP(sc.get(&tail_beg, nnz));
    PLAN_HIP(sc.get(&work, m));
    PLAN_HIP(sc.get(&work_pre, m + 1));
    PLAN_HIP(sc.get(&jmax, m));
    PLAN_HIP(sc.get(&nslots, m));
    PLAN_HIP(sc.get(&rclass, m));
    PLAN_HIP(sc.get(&bsize, m));
    PLAN_HIP(sc.get(&bbase, m + 1));
    PLAN_HIP(sc.get(&counters, 32));
    PLAN_HIP(sc.get(&part_m, scan_partials_size(m)));
    PLAN_HIP(sc.get(&p->slot_base, m + 1));
    PLAN_HIP(launch_fill_i64(counters, 32, 0, st));
    pr.tail_beg = tail_beg;
    unsigned long long *class_count = reinterpret_cast<unsigned long long *>(counters + kCntClass);
    int *err = reinterpret_cast<int *>(counters + kCntErr);
    unsigned long long *list_fill = reinterpret_cast<unsigned long long *>(counters + kCntFill);
    {
        StageTimer tm(ctx, kStRowPlan, st);
        PLAN_HIP(launch_row_plan(pr, s_min, tail_beg, work, jmax, nslots, rclass, bsize, class_count, err,
                                 reinterpret_cast<unsigned long long *>(counters + kCntHeavyWork), st));
    }
    {
        StageTimer tm(ctx, kStPlanScans, st);
        PLAN_HIP(launch_exclusive_scan_i32(nslots, m, p->slot_base, part_m, st));
        PLAN_HIP(launch_exclusive_scan_i64(work, m, work_pre, part_m, st));
        PLAN_HIP(launch_exclusive_scan_i64(bsize, m, bbase, part_m, st));
    }
    int64_t *hb = ctx->pinned;
    PLAN_HIP(hipMemcpyAsync(hb, counters, kCntTotal * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PLAN_HIP(hipMemcpyAsync(hb + kHbSlots, p->slot_base + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PLAN_HIP(hipMemcpyAsync(hb + kHbSlots + 1, work_pre + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PLAN_HIP(hipMemcpyAsync(hb + kHbSlots + 2, bbase + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PLAN_HIP(hipStreamSynchronize(st));
    if (hb[kCntErr] & 0xffffffff)
        return bail(fail(ctx, SLG_ERR_INVALID_GRAPH,
                         "malformed incidence (bad pointer, id out of range, or vertex CSR not the transpose)"));
    for (int c = 0; c < kNumLists; ++c) p->list_count[c] = hb[kCntClass + c];
    p->S = hb[kHbSlots];
    if (p->S >= (int64_t(1) << 31)) return bail(fail(ctx, SLG_ERR_OVERFLOW, "more than 2^31 output slots"));
    p->two_paths = hb[kHbSlots + 1];
    const int64_t nbounds = hb[kHbSlots + 2];
    p->nbounds = nbounds;
    p->heavy_two_paths = hb[kCntHeavyWork];
    if (nbounds >= (int64_t(1) << 40))
        return bail(fail(ctx, SLG_ERR_OVERFLOW, "boundary table too large"));

    // slot table, tier lists and the heavy rows' boundary table
    int32_t *slot_row;
    PLAN_HIP(sc.get(&slot_row, p->S));
    PLAN_HIP(sc.get(&p->bounds, nbounds));
    PLAN_HIP(sc.get(&p->tickets, 5));
    // lists start zeroed: an entry the fill kernels refuse to write (list
    // overflow, flagged in err) names slot 0 / an empty descriptor
    for (int c = 0; c < kLightClasses; ++c) {
        PLAN_HIP(sc.get(&p->lists[c], p->list_count[c]));
        PLAN_HIP(launch_fill_i32(p->lists[c], p->list_count[c], 0, st));
    }
    for (int h = 0; h < 2; ++h) {
        PLAN_HIP(sc.get(&p->heavy[h], p->list_count[kLightClasses + h]));
        PLAN_HIP(launch_fill_i64(reinterpret_cast<int64_t *>(p->heavy[h]),
                                 p->list_count[kLightClasses + h] * (int64_t)(sizeof(HeavyDesc) / 8), 0, st));
    }
    static_assert(sizeof(HeavyDesc) % 8 == 0, "HeavyDesc is filled as int64 words");
    int64_t *hat;  // first descriptor of each heavy row in its list
    PLAN_HIP(sc.get(&hat, m));
    {
        StageTimer tm(ctx, kStSlots, st);
        PLAN_HIP(launch_fill_slots(m, inc.he_ptr, p->slot_base, nslots, jmax, rclass, bbase, hat, slot_row,
                                   p->lists, p->heavy, p->list_count, list_fill, err, st));
    }
    {
        StageTimer tm(ctx, kStBounds, st);
        for (int h = 0; h < 2; ++h)
            PLAN_HIP(launch_bounds(pr, p->heavy[h], p->list_count[kLightClasses + h], p->bounds, st));
    }
    p->slots.count = p->S;
    p->slots.row = slot_row;

    // K3-K5 counting pass: per slot, per threshold, the number of edges
    const int K = num_s;
    PLAN_HIP(sc.get(&p->slot_cnt, (size_t)K * p->S));
    PLAN_HIP(sc.get(&p->slot_off, (size_t)K * (p->S + 1)));
    int64_t *part_s;
    PLAN_HIP(sc.get(&part_s, scan_partials_size(p->S)));
    {
        StageTimer tm(ctx, kStCountLight, st);
        for (int c = 0; c < kLightClasses; ++c)
            PLAN_HIP(launch_light(c, false, p->lists[c], p->list_count[c], p->slots, pr, p->prm, p->slot_cnt,
                                  nullptr, st));
    }
    PLAN_HIP(launch_fill_i64(p->tickets, 4, 0, st));
    for (int wide = 0; wide < 2; ++wide) {
        if (p->list_count[kLightClasses + wide] <= 0) continue;
        StageTimer tm(ctx, wide ? kStCountHeavyWide : kStCountHeavy, st);
        PLAN_HIP(launch_heavy(false, wide, p->heavy[wide], p->list_count[kLightClasses + wide], p->S,
                              p->bounds, pr, p->prm, p->slot_cnt, nullptr, p->tickets + wide,
                              ctx->heavy_resident, st));
    }
    {
        StageTimer tm(ctx, kStCountScans, st);
        for (int k = 0; k < K; ++k) {
            PLAN_HIP(launch_exclusive_scan_i64(p->slot_cnt + (size_t)k * p->S, p->S,
                                               p->slot_off + (size_t)k * (p->S + 1), part_s, st));
            PLAN_HIP(hipMemcpyAsync(hb + kHbEdges + k, p->slot_off + (size_t)k * (p->S + 1) + p->S,
                                    sizeof(int64_t), hipMemcpyDeviceToHost, st));
        }
    }
    PLAN_HIP(launch_fill_i64(p->tickets + 4, 1, 0, st));
    for (int h = 0; h < 2; ++h)
        PLAN_HIP(launch_heavy_edges(p->heavy[h], p->list_count[kLightClasses + h], p->slot_cnt, p->S, K,
                                    p->tickets + 4, st));
    PLAN_HIP(hipMemcpyAsync(hb + kHbHeavyEdges, p->tickets + 4, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PLAN_HIP(hipMemcpyAsync(hb + kHbHeavyEdges + 1, counters + kCntErr, sizeof(int64_t), hipMemcpyDeviceToHost,
                            st));
    PLAN_HIP(hipStreamSynchronize(st));
    if (hb[kHbHeavyEdges + 1] & 0xffffffff)
        return bail(fail(ctx, SLG_ERR_DEVICE, "internal error: a tier list overflowed its planned size"));
    for (int k = 0; k < K; ++k) p->num_edges[k] = hb[kHbEdges + k];
    p->heavy_edges = hb[kHbHeavyEdges];
#undef PLAN_HIP
    (void)rc;
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
slg_status emit_range(slg_plan *p, int64_t r0, int64_t r1, int64_t s0, int64_t s1, const int64_t *base,
                      int64_t *const *row_ptr, int32_t *const *row, int32_t *const *col, int32_t *const *w,
                      hipStream_t st) {
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
        for (int c = 0; c < kLightClasses; ++c)
            SLG_HIP(ctx, launch_light(c, true, p->lists[c], p->list_count[c], p->slots, p->pr, prm, nullptr,
                                      p->slot_off, st));
    }
    SLG_HIP(ctx, launch_fill_i64(p->tickets + 2, 2, 0, st));
    for (int wide = 0; wide < 2; ++wide) {
        if (p->list_count[kLightClasses + wide] <= 0) continue;
        StageTimer tm(ctx, wide ? kStEmitHeavyWide : kStEmitHeavy, st);
        SLG_HIP(ctx, launch_heavy(true, wide, p->heavy[wide], p->list_count[kLightClasses + wide], p->S,
                                  p->bounds, p->pr, prm, nullptr, p->slot_off, p->tickets + 2 + wide,
                                  ctx->heavy_resident, st));
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

slg_status slg_line_graph_stream(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                                 int64_t chunk_bytes, slg_chunk_fn fn, void *user, void *stream) {
    if (!ctx || !g || !fn || chunk_bytes <= 0) return fail(ctx, SLG_ERR_INVALID_ARG, "bad stream arguments");
    slg_plan *p = nullptr;
    slg_status rc = slg_plan_create(ctx, g, s, num_s, stream, &p);
    if (rc != SLG_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int K = num_s;
    const int64_t m = p->pr.m;
    std::vector<void *> bufs;
    auto cleanup = [&](slg_status code) {
        (void)hipStreamSynchronize(st);
        for (void *b : bufs) (void)hipFreeAsync(b, st);
        slg_plan_destroy(p);
        (void)hipStreamSynchronize(st);
        return code;
    };
#define STREAM_HIP(call)                                                                            \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return cleanup(fail(ctx, e_ == hipErrorOutOfMemory ? SLG_ERR_OUT_OF_MEMORY : SLG_ERR_DEVICE, \
                                "%s: %s", #call, hipGetErrorString(e_)));                           \
    } while (0)
    // output bytes before every row; chunks are greedy row ranges
    int64_t *dbytes;
    STREAM_HIP(hipMallocAsync(reinterpret_cast<void **>(&dbytes), (m + 1) * sizeof(int64_t), st));
    bufs.push_back(dbytes);
    STREAM_HIP(launch_row_bytes(m, p->slot_base, p->slot_off, p->S, K, dbytes, st));
    std::vector<int64_t> rbytes(m + 1);
    STREAM_HIP(hipMemcpyAsync(rbytes.data(), dbytes, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    STREAM_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> cuts{0};
    while (cuts.back() < m) {
        const int64_t r0 = cuts.back();
        const int64_t limit = rbytes[r0] + chunk_bytes - 8 * K;  // room for the closing row_ptr entry
        int64_t r1 = (int64_t)(std::upper_bound(rbytes.begin() + r0 + 1, rbytes.end(), limit) - rbytes.begin()) - 1;
        if (r1 <= r0) {
            return cleanup(fail(ctx, SLG_ERR_OUT_OF_MEMORY,
                                "row %lld alone needs %lld bytes, more than chunk_bytes", (long long)r0,
                                (long long)(rbytes[r0 + 1] - rbytes[r0] + 8 * K)));
        }
        cuts.push_back(r1);
    }
    // slot offsets of every threshold at every cut
    const int64_t nc = (int64_t)cuts.size();
    int64_t *dcuts, *doffs;
    STREAM_HIP(hipMallocAsync(reinterpret_cast<void **>(&dcuts), nc * sizeof(int64_t), st));
    bufs.push_back(dcuts);
    STREAM_HIP(hipMallocAsync(reinterpret_cast<void **>(&doffs), nc * K * sizeof(int64_t), st));
    bufs.push_back(doffs);
    STREAM_HIP(hipMemcpyAsync(dcuts, cuts.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice, st));
    STREAM_HIP(launch_gather_offsets(dcuts, nc, p->slot_base, p->slot_off, p->S, K, doffs, st));
    std::vector<int64_t> offs(nc * K), sb(nc);
    STREAM_HIP(hipMemcpyAsync(offs.data(), doffs, nc * K * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    for (int64_t c = 0; c < nc; ++c)  // first slot of every cut row
        STREAM_HIP(hipMemcpyAsync(&sb[c], p->slot_base + cuts[c], sizeof(int64_t), hipMemcpyDeviceToHost, st));
    STREAM_HIP(hipStreamSynchronize(st));
    // chunk buffers sized for the largest chunk of every threshold
    int64_t max_rows = 0, max_e[SLG_MAX_S] = {};
    for (int64_t c = 0; c + 1 < nc; ++c) {
        max_rows = std::max(max_rows, cuts[c + 1] - cuts[c]);
        for (int k = 0; k < K; ++k) max_e[k] = std::max(max_e[k], offs[(c + 1) * K + k] - offs[c * K + k]);
    }
    int64_t *rp[SLG_MAX_S];
    int32_t *ri[SLG_MAX_S], *rj[SLG_MAX_S], *rw[SLG_MAX_S];
    for (int k = 0; k < K; ++k) {
        STREAM_HIP(hipMallocAsync(reinterpret_cast<void **>(&rp[k]), (max_rows + 1) * sizeof(int64_t), st));
        bufs.push_back(rp[k]);
        void *q[3];
        for (int t = 0; t < 3; ++t) {
            STREAM_HIP(hipMallocAsync(&q[t], std::max<int64_t>(max_e[k], 1) * sizeof(int32_t), st));
            bufs.push_back(q[t]);
        }
        ri[k] = static_cast<int32_t *>(q[0]);
        rj[k] = static_cast<int32_t *>(q[1]);
        rw[k] = static_cast<int32_t *>(q[2]);
    }
    for (int64_t c = 0; c + 1 < nc; ++c) {
        const int64_t r0 = cuts[c], r1 = cuts[c + 1];
        rc = emit_range(p, r0, r1, sb[c], sb[c + 1], &offs[c * K], rp, ri, rj, rw, st);
        if (rc != SLG_OK) return cleanup(rc);
        STREAM_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < K; ++k) {
            const int64_t e0 = offs[c * K + k], ne = offs[(c + 1) * K + k] - e0;
            if (fn(user, k, s[k], r0, r1, e0, ne, rp[k], ri[k], rj[k], rw[k], stream) != 0)
                return cleanup(fail(ctx, SLG_ERR_CANCELLED, "chunk callback stopped the stream at row %lld",
                                    (long long)r0));
        }
    }
#undef STREAM_HIP
    return cleanup(SLG_OK);
}

slg_status slg_plan_stats(const slg_plan *p, int64_t *out, int32_t cap, int32_t *count) {
    if (!p || (!out && cap > 0) || cap < 0) return SLG_ERR_INVALID_ARG;
    int64_t vals[13];
    vals[0] = p->S;
    for (int c = 0; c < kLightClasses; ++c) vals[1 + c] = p->list_count[c];
    vals[7] = p->list_count[kLightClasses];
    vals[8] = p->list_count[kLightClasses + 1];
    vals[9] = p->two_paths;
    vals[10] = p->heavy_two_paths;
    vals[11] = p->nbounds;
    vals[12] = p->heavy_edges;
    static_assert(kLightClasses == 6, "plan stats layout");
    int32_t n = cap < 13 ? cap : 13;
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
    return SLG_OK;
}

slg_status slg_plan_destroy(slg_plan *p) {
    if (!p) return SLG_ERR_INVALID_ARG;
    p->scratch.release();
    delete p;
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
    r->k = num_s;
    r->m = g->inc.num_hyperedges;
    r->two_paths = p->two_paths;
    auto get = [&](void **ptr, size_t bytes) -> bool {
        if (bytes == 0) bytes = 8;
        if (ctx->has_alloc) {
            *ptr = ctx->alloc.alloc(ctx->alloc.user, bytes, stream);
        } else if (hipMallocAsync(ptr, bytes, r->st) != hipSuccess) {
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
    slg_context *ctx = r->ctx;
    for (void *ptr : r->owned) {
        if (ctx && ctx->has_alloc)
            ctx->alloc.release(ctx->alloc.user, ptr, r->st);
        else
            (void)hipFreeAsync(ptr, r->st);
    }
    delete r;
    return SLG_OK;
}

}  // extern "C"
