// gfx950 kernels for s-line graph construction.
//
// The path (Section III-B/C, Algorithms 2 and 3):
//   K1  prune: drop hyperedges with |e| < s_min from every vertex list
//       (degree-based pruning on both sides of a pair; a pair that meets
//       the threshold has both sizes >= s, so no edge is lost).
//   K2  plan: per kept hyperedge e_i and member v, the tail of v's list after
//       i (the partners e_j, j > i, reached through v: the upper triangle),
//       the 2-path work w_i = sum of tail lengths, and a slot table that
//       splits heavy rows by hyperedge-id range and by work.
//   K3  count overlaps |e_i n e_j| by walking every 2-path (e_i, v, e_j):
//         tiny rows (w_i <= 8): one lane sorts its partners in registers;
//         light rows (w_i <= 2048): one wavefront gathers the 2-path
//           partners into LDS, sorts them in registers (bitonic) and
//           run-length counts them;
//         heavy slots: one workgroup marks partners in an LDS bitmap over
//           the slot's id range, ranks them by prefix popcount, and counts
//           each repeated partner in an LDS counter indexed by its rank;
//           heavy vertex tails are cut into equal pieces across the
//           wavefronts.
//       The counting pass tallies every threshold's survivors (output
//       sizes) and, when memory allows, keeps each row's or slot's
//       (partner, overlap) pairs for the emit pass (the count stores).
//   K4/5 threshold-and-emit for every s_k of the ensemble from the same
//       counts (the stored overlap is the largest s for which the pair
//       survives), compacted with wavefront ballots + prefix sums. The rank
//       order is the hyperedge-id order, so rows come out sorted.
//   K6  assembly: prefix sums of per-slot counts give each slot's output
//       offset and the CSR row pointers.
// Every step is exact integer work; no floating point is involved.
#include <limits.h>

#include <type_traits>

#include "slg_internal.h"

namespace slg {
namespace {

// ---------------------------------------------------------------------------
// wavefront / workgroup primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Pointers that reach a kernel through LDS or a struct in memory lose their
// address space; naming it keeps their accesses global_* (flat accesses also
// count against the LDS wait counter, so every LDS wait would wait for them).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Wavefront-uniform values moved to scalar registers.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long uniform(long long x) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x & 0xFFFFFFFFll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T *uniform(T *p) {
    return reinterpret_cast<T *>(uniform((long long)reinterpret_cast<uintptr_t>(p)));
}

__device__ __forceinline__ int bits_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// LDS writes of this wavefront become visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan over a workgroup of NT threads; `wsum` holds NT/64 entries.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *wsum, T &total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    T incl = wave_incl_scan(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T t = wsum[w];
        pre += (w < wave) ? t : T(0);
        tot += t;
    }
    total = tot;
    __syncthreads();
    return pre + incl - x;
}

// As block_excl_scan, without the trailing barrier: the caller guarantees
// a workgroup barrier before `wsum` is written again.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan_open(T x, T *wsum, T &total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    T incl = wave_incl_scan(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T t = wsum[w];
        pre += (w < wave) ? t : T(0);
        tot += t;
    }
    total = tot;
    return pre + incl - x;
}

// Copy the by-value parameter block into LDS, one dword per thread (the
// caller follows with a workgroup barrier).
__device__ __forceinline__ void stage_params(EmitParams *dst, const EmitParams &src) {
    constexpr int kWords = (int)(sizeof(EmitParams) / 4);
    static_assert(sizeof(EmitParams) % 4 == 0, "EmitParams is dword-sized");
    const int32_t *from = reinterpret_cast<const int32_t *>(&src);
    int32_t *to = reinterpret_cast<int32_t *>(dst);
    for (int x = threadIdx.x; x < kWords; x += blockDim.x) to[x] = from[x];
}

// First position in a[lo, hi) holding a value >= key (a sorted ascending).
__device__ __forceinline__ int lower_bound_i32(const int32_t *__restrict__ a, int lo, int hi,
                                               int key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan (int64 output, out[n] = total)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const T *__restrict__ in,
                                                                   int64_t n,
                                                                   int64_t *__restrict__ partials) {
    __shared__ int64_t ws[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int t = threadIdx.x; t < kScanTile; t += kScanThreads) {
        int64_t idx = base + t;
        if (idx < n) s += (int64_t)in[idx];
    }
    s = wave_sum(s);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t += ws[w];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void scan_top_kernel(int64_t *__restrict__ partials, int64_t nb) {
    __shared__ int64_t ws[16];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t idx = base + threadIdx.x;
        int64_t x = idx < nb ? partials[idx] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan<1024>(x, ws, tot);
        if (idx < nb) partials[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) partials[nb] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const T *__restrict__ in, int64_t n,
                                                                 const int64_t *__restrict__ partials,
                                                                 int64_t *__restrict__ out) {
    __shared__ int64_t ws[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        int64_t idx = base + r;
        v[r] = idx < n ? (int64_t)in[idx] : 0;
        local += v[r];
    }
    int64_t tot;
    int64_t run = partials[blockIdx.x] + block_excl_scan<kScanThreads>(local, ws, tot);
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        int64_t idx = base + r;
        if (idx < n) out[idx] = run;
        run += v[r];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = partials[gridDim.x];
}

__global__ void fill_i64_kernel(int64_t *__restrict__ p, int64_t n, int64_t value) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) p[idx] = value;
}

__global__ void fill_i32_kernel(int32_t *__restrict__ p, int64_t n, int32_t value) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) p[idx] = value;
}

template <typename T>
hipError_t exclusive_scan(const T *in, int64_t n, int64_t *out, int64_t *partials, hipStream_t st) {
    if (n <= 0) return launch_fill_i64(out, 1, 0, st);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    scan_reduce_kernel<T><<<dim3((unsigned)nb), dim3(kScanThreads), 0, st>>>(in, n, partials);
    scan_top_kernel<<<1, 1024, 0, st>>>(partials, nb);
    scan_down_kernel<T><<<dim3((unsigned)nb), dim3(kScanThreads), 0, st>>>(in, n, partials, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K1: prune hyperedges smaller than s_min out of the vertex lists
// ---------------------------------------------------------------------------
__global__ void keep_incidence_kernel(int64_t nnz, const int32_t *__restrict__ v_idx,
                                      const int64_t *__restrict__ he_ptr, int64_t m, int32_t s_min,
                                      const int32_t *__restrict__ row_s, uint8_t *__restrict__ flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    int32_t e = v_idx[p];
    uint8_t keep = 0;
    if (e >= 0 && e < m) keep = (he_ptr[e + 1] - he_ptr[e]) >= (row_s ? row_s[e] : s_min);
    flag[p] = keep;
}

__global__ void compact_idx_kernel(int64_t nnz, const int32_t *__restrict__ v_idx,
                                   const uint8_t *__restrict__ flag, const int64_t *__restrict__ pos,
                                   int32_t *__restrict__ vs_idx) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz && flag[p]) vs_idx[pos[p]] = v_idx[p];
}

__global__ void compact_ptr_kernel(int64_t n, int64_t nnz, const int64_t *__restrict__ v_ptr,
                                   const int64_t *__restrict__ pos, int64_t *__restrict__ vs_ptr) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    int64_t q = v_ptr[v];
    q = q < 0 ? 0 : (q > nnz ? nnz : q);
    vs_ptr[v] = pos[q];
}

// E_s positions of the kept rows (the dense tier's counter index): the rank
// of every kept row among the kept rows, its inverse, and the pruned vertex
// lists rewritten in ranks. Ranks keep the id order, so a list stays sorted
// and its tails are at the same positions.
__global__ void row_keep_kernel(int64_t m, const int64_t *__restrict__ he_ptr, int32_t s_min,
                                const int32_t *__restrict__ row_s, uint8_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t size = he_ptr[i + 1] - he_ptr[i];
    flag[i] = size > 0 && size >= (row_s ? row_s[i] : s_min);
}

__global__ void cid_kernel(int64_t m, const uint8_t *__restrict__ flag, const int64_t *__restrict__ pre,
                           int32_t *__restrict__ cid, int32_t *__restrict__ cid_row) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const bool kept = flag[i] != 0;
    cid[i] = kept ? (int32_t)pre[i] : -1;
    if (kept) cid_row[pre[i]] = (int32_t)i;
}

// An id outside [0, m) (a malformed vertex CSR, which the row plan flags)
// gets -1, which no window holds. vs_win keeps the low kDenseBits bits of
// each rank: windows are aligned, so that is the rank's place in its window.
__global__ void vs_cid_kernel(int64_t n, int64_t m, int64_t cap, const int64_t *__restrict__ vs_ptr,
                              const int32_t *__restrict__ vs_idx, const int32_t *__restrict__ cid,
                              int32_t *__restrict__ vs_cid, uint16_t *__restrict__ vs_win) {
    int64_t total = vs_ptr[n];
    if (total > cap) total = cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += stride) {
        const int32_t r = vs_idx[p];
        const int32_t c = (r >= 0 && r < m) ? cid[r] : -1;
        vs_cid[p] = c;
        vs_win[p] = (uint16_t)(c & (kDenseWindow - 1));
    }
}

// ---------------------------------------------------------------------------
// K2: per-row plan (one wavefront per hyperedge, grid-stride)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int light_class(int64_t w) {
    if (w <= kTinyMax) return 0;
    int c = 1;
    while (c < kLightClasses - 1 && w > (int64_t(64) << (c - 1))) ++c;
    return c;
}

// Per-row work estimate (Section III-E's cost: the 2-paths of row i) and
// tier. Rows of at most kSmallRow members are walked by one lane each, rows
// of at most kWaveRow by the wavefront of their row group; larger rows are
// cut into pieces of kPlanPiece members, one wavefront per piece, so that a
// run of large rows (an input sorted by size) spreads over the whole grid. For every incidence (i, v) of a kept row: tail_beg = first
// position after i in v's (pruned) list; w_i = sum of the tails; jm =
// largest partner id.
constexpr int kSmallRow = 16;
constexpr int kWaveRow = 64;
constexpr int kPlanPiece = 256;

struct RowPlanOut {
    int32_t *tail_beg;
    int64_t *work;
    int32_t *jmax;
    int32_t *nslots;
    uint8_t *rclass;
    int64_t *bsize;
    int32_t dense_ratio;  // the dense tier's rule (0: off)
    int32_t dense_min;
    unsigned long long *dense_work;
};

// One member of row i: its tail in v's list; returns false when the
// incidence is malformed.
__device__ __forceinline__ bool plan_member(const Pruned &g, int64_t i, int64_t p, int32_t *tail_beg, int64_t &w,
                                            int &jm) {
    const int v = g.he_idx[p];
    if (v < 0 || v >= g.n) {
        tail_beg[p] = 0;
        return false;
    }
    const int64_t lo = g.vs_ptr[v], hi = g.vs_ptr[v + 1];
    if (lo < 0 || hi < lo || hi > g.nnz) {
        tail_beg[p] = 0;
        return false;
    }
    const int a = lower_bound_i32(g.vs_idx, (int)lo, (int)hi, (int)i);
    const bool found = a < hi && g.vs_idx[a] == (int)i;  // the vertex CSR must be the transpose
    const int beg = found ? a + 1 : a;
    tail_beg[p] = beg;
    w += hi - beg;
    if (beg < hi) jm = max(jm, g.vs_idx[hi - 1]);
    return found;
}

// Tier, slot count and boundary-table size of row i from its totals. A
// heavy row goes to the dense tier when its candidate partners (the kept
// rows in (i, jm]) number at least dense_min and it has at least
// dense_ratio 2-paths per eight candidates: its slots are then the aligned
// kDenseWindow windows of E_s positions that (i, jm] touches.
__device__ __forceinline__ void plan_finish(const Pruned &g, int64_t i, int64_t p0, int64_t p1, int64_t w, int jm,
                                            bool bad, int32_t light_max, int64_t slot_work, const RowPlanOut &o,
                                            unsigned long long *ccount, unsigned long long *hwork, int *err) {
    int cls = kNone;
    int64_t ns = 0;
    if (bad) {
        atomicOr(err, 1);
    } else if (w > 0) {
        int64_t ci = -1, cj = -1;
        if (w > light_max && o.dense_ratio > 0 && g.cid && p1 - p0 < kWideMembers && jm > i && jm < g.m) {
            ci = g.cid[i];
            cj = g.cid[jm];
        }
        const int64_t crange = cj - ci;  // kept rows in (i, jm]
        if (w <= light_max) {
            cls = kLight0 + light_class(w);
            ns = 1;
        } else if (ci >= 0 && cj > ci && crange >= o.dense_min && 8 * w >= (int64_t)o.dense_ratio * crange) {
            cls = kDense;
            ns = (cj >> kDenseBits) - ((ci + 1) >> kDenseBits) + 1;
        } else {
            cls = (p1 - p0 >= kWideMembers) ? kHeavyWide : kHeavy;
            const int64_t range = (int64_t)jm - i;  // partners lie in [i+1, jm]
            const int64_t by_range = (range + kRangeBits - 1) / kRangeBits;
            const int64_t by_work = (w + slot_work - 1) / slot_work;
            ns = by_range > by_work ? by_range : by_work;
            if (ns > range) ns = range;
        }
    }
    o.work[i] = w;
    o.jmax[i] = jm;
    o.nslots[i] = (int32_t)ns;
    o.rclass[i] = (uint8_t)cls;
    o.bsize[i] = cls >= kHeavy ? (ns + 1) * (p1 - p0) : 0;
    if (cls != kNone) atomicAdd(&ccount[cls - 1], (unsigned long long)ns);
    if (cls == kHeavy || cls == kHeavyWide) atomicAdd(hwork, (unsigned long long)w);
    if (cls == kDense) atomicAdd(o.dense_work, (unsigned long long)w);
}

// Small and middle rows, and the piece list of the large ones: a large row
// appends ceil(size / kPlanPiece) entries (row | piece << 32), one row's
// pieces side by side.
__global__ __launch_bounds__(256) void row_plan_kernel(Pruned g, int32_t s_min, int32_t light_max,
                                                       int64_t slot_work, int64_t row_lo, int64_t row_hi,
                                                       RowPlanOut o,
                                                       unsigned long long *__restrict__ class_count,
                                                       int *__restrict__ err,
                                                       unsigned long long *__restrict__ heavy_work,
                                                       int64_t *__restrict__ pieces, int64_t pieces_cap,
                                                       unsigned long long *__restrict__ num_pieces) {
    __shared__ unsigned long long ccount[kNumLists];
    __shared__ unsigned long long hwork;
    if (threadIdx.x < kNumLists) ccount[threadIdx.x] = 0;
    if (threadIdx.x == 0) hwork = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64 * 64; i0 < g.m; i0 += nwaves * 64) {
        const int64_t i = i0 + lane;
        unsigned long long np = 0;  // pieces of a large row
        bool mid = false;           // a middle row, walked by the wavefront below
        if (i < g.m) {
            const int64_t p0 = g.he_ptr[i], p1 = g.he_ptr[i + 1];
            if (p0 < 0 || p1 > g.nnz || p1 < p0) {  // malformed pointers
                plan_finish(g, i, p0, p1, 0, -1, true, light_max, slot_work, o, ccount, &hwork, err);
            } else {
                const int64_t size = p1 - p0;
                // rows outside [row_lo, row_hi) are planned as pruned ones
                const bool kept = size > 0 && size >= (g.row_s ? g.row_s[i] : s_min) && i >= row_lo && i < row_hi;
                if (kept && size > kWaveRow) {
                    np = (unsigned long long)((size + kPlanPiece - 1) / kPlanPiece);
                } else if (kept && size > kSmallRow) {
                    mid = true;
                } else {  // a small (or pruned) row, walked by its own lane
                    int64_t w = 0;
                    int jm = -1;
                    bool rbad = false;
                    if (kept)
                        for (int64_t p = p0; p < p1; ++p) rbad |= !plan_member(g, i, p, o.tail_beg, w, jm);
                    plan_finish(g, i, p0, p1, w, jm, rbad, light_max, slot_work, o, ccount, &hwork, err);
                }
            }
        }
        // the middle rows of this group, one after another by the whole
        // wavefront (one member per lane)
        unsigned long long todo = __ballot(mid);
        while (todo) {
            const int l = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int64_t r = i0 + l;
            const int64_t q0 = g.he_ptr[r], q1 = g.he_ptr[r + 1];
            int64_t w = 0;
            int jm = -1;
            int rbad = 0;
            if (q0 + lane < q1) rbad = !plan_member(g, r, q0 + lane, o.tail_beg, w, jm);
            w = wave_sum(w);
            jm = wave_max(jm);
            rbad = wave_max(rbad);
            if (lane == 0) plan_finish(g, r, q0, q1, w, jm, rbad != 0, light_max, slot_work, o, ccount, &hwork, err);
        }
        // one reservation per wavefront for the pieces of its large rows
        const unsigned long long incl = wave_incl_scan(np);
        const unsigned long long total = __shfl(incl, 63);
        if (total) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(num_pieces, total);
            base = __shfl(base, 0) + incl - np;
            // within the capacity unless the row pointers overlap (malformed)
            for (unsigned long long k = 0; k < np; ++k) {
                if (base + k < (unsigned long long)pieces_cap)
                    pieces[base + k] = (int64_t)((unsigned long long)i | (k << 32));
                else
                    atomicOr(err, 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumLists && ccount[threadIdx.x])
        atomicAdd(&class_count[threadIdx.x], ccount[threadIdx.x]);
    if (threadIdx.x == 0 && hwork) atomicAdd(heavy_work, hwork);
}

// One wavefront per piece of a large row: the piece's tails and its largest
// partner id, into the piece's own partial slots.
__global__ __launch_bounds__(256) void row_piece_kernel(Pruned g, int32_t *__restrict__ tail_beg,
                                                        const int64_t *__restrict__ pieces, int64_t pieces_cap,
                                                        const unsigned long long *__restrict__ num_pieces,
                                                        int64_t *__restrict__ piece_w,
                                                        int32_t *__restrict__ piece_jm, int *__restrict__ err) {
    const int lane = lane_id();
    const int64_t count = min((int64_t)*num_pieces, pieces_cap);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; t < count; t += nwaves) {
        const unsigned long long e = (unsigned long long)pieces[t];
        const int64_t r = (int64_t)(e & 0xFFFFFFFFull), k = (int64_t)(e >> 32);
        const int64_t q0 = g.he_ptr[r], q1 = g.he_ptr[r + 1];
        const int64_t a = q0 + k * kPlanPiece, b = min(q1, a + kPlanPiece);
        int64_t w = 0;
        int jm = -1, rbad = 0;
        for (int64_t p = a + lane; p < b; p += 64) rbad |= !plan_member(g, r, p, tail_beg, w, jm);
        w = wave_sum(w);
        jm = wave_max(jm);
        rbad = wave_max(rbad);
        if (lane == 0) {
            piece_w[t] = w;
            piece_jm[t] = jm;
            if (rbad) atomicOr(err, 1);
        }
    }
}

// One lane per row's first piece: the row's totals from its pieces, then the
// tier decision.
__global__ __launch_bounds__(256) void row_piece_finish_kernel(Pruned g, int32_t light_max, int64_t slot_work,
                                                               RowPlanOut o,
                                                               unsigned long long *__restrict__ class_count,
                                                               int *__restrict__ err,
                                                               unsigned long long *__restrict__ heavy_work,
                                                               const int64_t *__restrict__ pieces,
                                                               int64_t pieces_cap,
                                                               const unsigned long long *__restrict__ num_pieces,
                                                               const int64_t *__restrict__ piece_w,
                                                               const int32_t *__restrict__ piece_jm) {
    __shared__ unsigned long long ccount[kNumLists];
    __shared__ unsigned long long hwork;
    if (threadIdx.x < kNumLists) ccount[threadIdx.x] = 0;
    if (threadIdx.x == 0) hwork = 0;
    __syncthreads();
    const int64_t count = min((int64_t)*num_pieces, pieces_cap);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long e = (unsigned long long)pieces[t];
        if (e >> 32) continue;  // not the row's first piece
        const int64_t r = (int64_t)(e & 0xFFFFFFFFull);
        const int64_t q0 = g.he_ptr[r], q1 = g.he_ptr[r + 1];
        const int64_t np = min((q1 - q0 + kPlanPiece - 1) / kPlanPiece, count - t);
        int64_t w = 0;
        int jm = -1;
        for (int64_t k = 0; k < np; ++k) {
            w += piece_w[t + k];
            jm = max(jm, piece_jm[t + k]);
        }
        // a malformed member has already set err
        plan_finish(g, r, q0, q1, w, jm, false, light_max, slot_work, o, ccount, &hwork, err);
    }
    __syncthreads();
    if (threadIdx.x < kNumLists && ccount[threadIdx.x])
        atomicAdd(&class_count[threadIdx.x], ccount[threadIdx.x]);
    if (threadIdx.x == 0 && hwork) atomicAdd(heavy_work, hwork);
}

// A row block: rows outside [r0, r1) get no slots, no class and no boundary
// entries (from the rows phase's values of every row), and the block's
// list sizes and heavy / dense 2-paths are summed as the row plan sums them.
__global__ __launch_bounds__(256) void block_mask_kernel(int64_t m, int64_t r0, int64_t r1,
                                                         const int32_t *__restrict__ nslots_all,
                                                         const uint8_t *__restrict__ rclass_all,
                                                         const int64_t *__restrict__ bsize_all,
                                                         const int64_t *__restrict__ work,
                                                         int32_t *__restrict__ nslots, uint8_t *__restrict__ rclass,
                                                         int64_t *__restrict__ bsize,
                                                         unsigned long long *__restrict__ class_count,
                                                         unsigned long long *__restrict__ heavy_work,
                                                         unsigned long long *__restrict__ dense_work) {
    __shared__ unsigned long long cc[kNumLists];
    __shared__ unsigned long long hw, dw;
    if (threadIdx.x < kNumLists) cc[threadIdx.x] = 0;
    if (threadIdx.x == 0) hw = dw = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const bool in = i >= r0 && i < r1;
        const int c = in ? rclass_all[i] : kNone;
        const int ns = in ? nslots_all[i] : 0;
        nslots[i] = ns;
        rclass[i] = (uint8_t)c;
        bsize[i] = in ? bsize_all[i] : 0;
        if (c != kNone) atomicAdd(&cc[c - 1], (unsigned long long)ns);
        if (c == kHeavy || c == kHeavyWide) atomicAdd(&hw, (unsigned long long)work[i]);
        if (c == kDense) atomicAdd(&dw, (unsigned long long)work[i]);
    }
    __syncthreads();
    if (threadIdx.x < kNumLists && cc[threadIdx.x]) atomicAdd(&class_count[threadIdx.x], cc[threadIdx.x]);
    if (threadIdx.x == 0 && hw) atomicAdd(heavy_work, hw);
    if (threadIdx.x == 0 && dw) atomicAdd(dense_work, dw);
}

// Tier lists filled by fill_slots_kernel.
struct LightLists {
    int32_t *l[kLightClasses];
    int64_t cap[kNumLists];  // capacity of every tier list (light, heavy, heavy-wide)
    int *err;                // set when an append would overflow a list
};

// Writes every light row's slot and appends it to its tier list, and
// reserves each heavy row's slot descriptors in the heavy lists. Rows are
// appended in blocks: a workgroup takes 256 * kFillRows rows, counts them per
// list with wavefront sums into LDS,
// reserves each list's share with one global atomic, then places its rows
// through LDS cursors (global atomics on the few list counters would
// serialise).
constexpr int kFillRows = 4;

__global__ __launch_bounds__(256) void fill_slots_kernel(
    int64_t m, const int64_t *__restrict__ he_ptr, const int64_t *__restrict__ slot_base,
    const int32_t *__restrict__ nslots, const int32_t *__restrict__ jmax,
    const uint8_t *__restrict__ rclass, const int64_t *__restrict__ bbase,
    int32_t *__restrict__ slot_row, LightLists ll, int64_t *__restrict__ hat,
    unsigned long long *__restrict__ list_fill) {
    __shared__ unsigned long long cursor[kNumLists];
    const int tid = threadIdx.x, lane = lane_id();
    const int64_t i0 = (int64_t)blockIdx.x * (256 * kFillRows);
    int cls[kFillRows], ns[kFillRows];
    int64_t base[kFillRows];
#pragma unroll
    for (int r = 0; r < kFillRows; ++r) {
        const int64_t i = i0 + r * 256 + tid;
        cls[r] = kNone;
        ns[r] = 0;
        base[r] = 0;
        if (i < m) {
            cls[r] = rclass[i];
            ns[r] = nslots[i];
            base[r] = slot_base[i];
        }
    }
    if (tid < kNumLists) cursor[tid] = 0;
    __syncthreads();
    // entries per light list: one per row (heavy descriptors are placed by
    // heavy_desc_kernel, in slot order)
    for (int c = kLight0; c < kLight0 + kLightClasses; ++c) {
        int mine = 0;
#pragma unroll
        for (int r = 0; r < kFillRows; ++r)
            if (cls[r] == c) mine += 1;
        const int tot = wave_sum(mine);
        if (lane == 0 && tot) atomicAdd(&cursor[c - 1], (unsigned long long)tot);
    }
    __syncthreads();
    if (tid < kNumLists && cursor[tid]) cursor[tid] = atomicAdd(&list_fill[tid], cursor[tid]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kFillRows; ++r) {
        const int64_t i = i0 + r * 256 + tid;
        for (int c = kLight0; c < kLight0 + kLightClasses; ++c) {
            const int w = (cls[r] == c) ? 1 : 0;
            const int incl = wave_incl_scan(w);
            const int tot = __shfl(incl, 63);
            if (!tot) continue;
            unsigned long long at = 0;
            if (lane == 63) at = atomicAdd(&cursor[c - 1], (unsigned long long)tot);
            at = __shfl(at, 63);
            if (!w) continue;
            const unsigned long long pos = at + incl - w;
            if (pos < (unsigned long long)ll.cap[c - 1]) {
                ll.l[c - 1][pos] = (int32_t)base[r];
                slot_row[base[r]] = (int32_t)i;
            } else {
                atomicOr(ll.err, 16);
            }
        }
    }
}

// One wavefront per heavy row, one lane per slot: the slot descriptors.
// Heavy slots per row, by class: the prefix sums place every heavy row's
// descriptors in row order, so each heavy list is in slot order.
__global__ void heavy_counts_kernel(int64_t m, const uint8_t *__restrict__ rclass, const int32_t *__restrict__ nslots,
                                    int32_t *__restrict__ cnt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = rclass[i];
        cnt[i] = c == kHeavy ? nslots[i] : 0;
        cnt[m + i] = c == kHeavyWide ? nslots[i] : 0;
        cnt[2 * m + i] = c == kDense ? nslots[i] : 0;
    }
}

// For every c, the position of the first slot >= slots[c] in a heavy list
// ordered by slot (one thread per c).
__global__ void list_cuts_kernel(const HeavyDesc *__restrict__ desc, int64_t count,
                                 const int64_t *__restrict__ slots, int64_t n, int64_t *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t key = slots[c];
    int64_t lo = 0, hi = count;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)desc[mid].slot < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    out[c] = lo;
}

// First and one-past-last positions of the slots in [s0, s1) in a heavy
// list ordered by slot.
__global__ void heavy_range_kernel(const HeavyDesc *__restrict__ desc, int64_t count, int64_t s0, int64_t s1,
                                   int64_t *__restrict__ out) {
    if (threadIdx.x >= 2) return;
    const int64_t key = threadIdx.x == 0 ? s0 : s1;
    int64_t lo = 0, hi = count;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)desc[mid].slot < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    out[threadIdx.x] = lo;
}

struct HeavyLists {
    HeavyDesc *l[kNumHeavyLists];  // heavy, heavy-wide, dense
    int64_t cap[kNumHeavyLists];
};

__global__ __launch_bounds__(256) void heavy_desc_kernel(
    int64_t m, const int64_t *__restrict__ he_ptr, const int64_t *__restrict__ slot_base,
    const int32_t *__restrict__ nslots, const int32_t *__restrict__ jmax,
    const uint8_t *__restrict__ rclass, const int64_t *__restrict__ bbase,
    const int64_t *__restrict__ hat, int32_t *__restrict__ slot_row, HeavyLists hl,
    const int32_t *__restrict__ cid, int *__restrict__ err) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; i < m; i += nwaves) {
        const int cls = rclass[i];
        if (cls < kHeavy) continue;
        const int h = cls - kHeavy;  // list: heavy, heavy-wide, dense
        const int ns = nslots[i];
        const int64_t at = hat[h * (m + 1) + i];  // prefix of the class's slots
        if (at < 0 || at + ns > hl.cap[h]) {
            if (lane == 0) atomicOr(err, 16);
            continue;
        }
        HeavyDesc *lst = hl.l[h] + at;
        const int64_t base = slot_base[i];
        const int64_t range = (int64_t)jmax[i] - i;
        const int k = (int)(he_ptr[i + 1] - he_ptr[i]);
        const int64_t bb = bbase[i];
        // dense slots: aligned windows of E_s positions from the window of
        // the row's first candidate (its own position + 1)
        const int64_t w0 = cls == kDense ? ((int64_t)cid[i] + 1) >> kDenseBits : 0;
        for (int t = lane; t < ns; t += 64) {
            HeavyDesc d;
            d.row = (int32_t)i;
            if (cls == kDense) {
                d.ja = (int32_t)((w0 + t) << kDenseBits);
                d.jb = (int32_t)((w0 + t + 1) << kDenseBits);
            } else {
                d.ja = (int32_t)(i + 1 + range * t / ns);
                d.jb = (int32_t)(i + 1 + range * (t + 1) / ns);
            }
            d.k = k;
            d.slot = (int32_t)(base + t);
            d.last = t == ns - 1;
            d.bptr = bb + (int64_t)t * k;
            slot_row[base + t] = (int32_t)i;
            lst[t] = d;
        }
    }
}

// ---------------------------------------------------------------------------
// K3-K5 light tier: one wavefront per row, sort-and-count in registers
// ---------------------------------------------------------------------------
// Bitonic sort of 64*KPL keys; element e = lane*KPL + r lives in key[r].
template <int KPL>
__device__ __forceinline__ void wave_bitonic(int (&key)[KPL], int lane) {
    constexpr int P = 64 * KPL;
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < KPL) {
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    const int pr = r ^ j;
                    if (pr > r) {
                        const bool asc = ((lane * KPL + r) & k) == 0;
                        const int a = key[r], b = key[pr];
                        const bool sw = asc ? (a > b) : (a < b);
                        key[r] = sw ? b : a;
                        key[pr] = sw ? a : b;
                    }
                }
            } else {
                const int lx = j / KPL;
                const bool lower = (lane & lx) == 0;
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    const int other = __shfl_xor(key[r], lx);
                    const bool asc = ((lane * KPL + r) & k) == 0;
                    key[r] = (lower == asc) ? min(key[r], other) : max(key[r], other);
                }
            }
        }
    }
}

// Rows with at most kTinyMax 2-paths: one lane per row. The lane collects
// its row's partners (the tails of its members' vertex lists), sorts them
// with a fixed 8-key network in registers, and writes the runs that reach
// each threshold to its own slot's place in the output.
template <bool EMIT>
__global__ __launch_bounds__(256) void tiny_kernel(const int32_t *__restrict__ list, int64_t count, Slots sl,
                                                   Pruned g, EmitParams prm, int64_t *__restrict__ slot_cnt,
                                                   const int64_t *__restrict__ slot_off) {
    static_assert(kTinyMax == 8, "8-key sorting network");
    __shared__ int32_t keys[kTinyMax][256];  // column per thread: conflict-free
    __shared__ EmitParams sp;
    stage_params(&sp, prm);
    __syncthreads();
    const EmitParams *ep = &sp;
    const int tid = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * 256 + tid;
    if (t >= count) return;
    const int slot = list[t];
    if (EMIT && (slot < ep->slot_lo || slot >= ep->slot_hi)) return;  // outside the emitted chunk
    const int i = sl.row[slot];
    const int64_t p0 = g.he_ptr[i], p1 = g.he_ptr[i + 1];
    int n = 0;
    for (int64_t p = p0; p < p1 && n < kTinyMax; ++p) {
        const int v = g.he_idx[p];
        const int64_t end = g.vs_ptr[v + 1];
        for (int64_t q = g.tail_beg[p]; q < end && n < kTinyMax; ++q) keys[n++][tid] = g.vs_idx[q];
    }
    int k[kTinyMax];
#pragma unroll
    for (int r = 0; r < kTinyMax; ++r) k[r] = r < n ? keys[r][tid] : INT_MAX;
    // Batcher's odd-even merge sort network for 8 keys (19 compare-exchanges)
    auto cx = [&](int a, int b) {
        const int lo = min(k[a], k[b]), hi = max(k[a], k[b]);
        k[a] = lo;
        k[b] = hi;
    };
    cx(0, 1); cx(2, 3); cx(4, 5); cx(6, 7);
    cx(0, 2); cx(1, 3); cx(4, 6); cx(5, 7);
    cx(1, 2); cx(5, 6);
    cx(0, 4); cx(1, 5); cx(2, 6); cx(3, 7);
    cx(2, 4); cx(3, 5);
    cx(1, 2); cx(3, 4); cx(5, 6);
    // the head of each run of equal partners holds the overlap
    int c[kTinyMax];
#pragma unroll
    for (int r = 0; r < kTinyMax; ++r) {
        int run = 0;
        if (r < n && (r == 0 || k[r] != k[r - 1])) {
#pragma unroll
            for (int q = r; q < kTinyMax; ++q) run += (q < n && k[q] == k[r]) ? 1 : 0;
        }
        c[r] = run;  // 0 for non-heads
    }
    const int K = ep->k;
    const int64_t S = sl.count;
    const int id0 = ep->row_base ? as_global(ep->row_base)[i] : 0;  // caller's id of row i is i - id0
    const int srow = ep->row_s ? as_global(ep->row_s)[i] : 0;
    for (int kk = 0; kk < K; ++kk) {
        const int sk = ep->row_s ? srow : ep->s[kk];
        int64_t pos = EMIT ? slot_off[(int64_t)kk * (S + 1) + slot] - ep->out_base[kk] : 0;
        const int64_t start = pos;
        const auto col = as_global(EMIT ? ep->col[kk] : nullptr);
        const auto wo = as_global(EMIT ? ep->w[kk] : nullptr);
        const auto ro = as_global(EMIT ? ep->row[kk] : nullptr);
#pragma unroll
        for (int r = 0; r < kTinyMax; ++r) {
            if (c[r] >= sk) {  // sk >= 1, so only run heads
                if (EMIT) {
                    col[pos] = k[r] - id0;
                    wo[pos] = c[r];
                    if (ro) ro[pos] = i - id0;
                }
                ++pos;
            }
        }
        if (!EMIT) slot_cnt[(int64_t)kk * S + slot] = pos - start;
    }
}

// STORE (counting pass): the row's partners and overlaps are also written
// to the light store, in partner order.
template <int KPL, bool EMIT, bool STORE>
__global__ __launch_bounds__(256) void light_kernel(const int32_t *__restrict__ list, int64_t count,
                                                    Slots sl, Pruned g, EmitParams prm,
                                                    int64_t *__restrict__ slot_cnt,
                                                    const int64_t *__restrict__ slot_off, LightStore ls) {
    static_assert(!(STORE && EMIT), "the store is written by the counting pass");
    constexpr int P = 64 * KPL;
    __shared__ int32_t buf[4][P];
    __shared__ int32_t seg_a[4][64];
    __shared__ int32_t seg_p[4][65];
    __shared__ EmitParams sp;  // thresholds and outputs, indexed by a uniform k
    stage_params(&sp, prm);
    __syncthreads();
    const EmitParams *ep = &sp;
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * 4 + wv;
    if (wid >= count) return;
    int32_t *kb = buf[wv];
    const int slot = list[wid];
    if (EMIT && (slot < ep->slot_lo || slot >= ep->slot_hi)) return;  // outside the emitted chunk
    const int i = sl.row[slot];
    const int64_t p0 = g.he_ptr[i], p1 = g.he_ptr[i + 1];

    // gather the partners e_j of every 2-path (e_i, v, e_j), j > i: members
    // are taken 64 at a time; their tails are flattened and every lane finds
    // the tail of each of its positions by binary search, so all loads of a
    // batch are independent and coalesced within a tail
    int32_t *sa = seg_a[wv];
    int32_t *sp0 = seg_p[wv];
    int w = 0;
    for (int64_t q = p0; q < p1; q += 64) {
        const int64_t p = q + lane;
        int beg = 0, len = 0;
        if (p < p1) {
            const int v = g.he_idx[p];
            beg = g.tail_beg[p];
            len = (int)(g.vs_ptr[v + 1] - beg);
        }
        const int incl = wave_incl_scan(len);
        const int tot = __shfl(incl, 63);
        sa[lane] = beg;
        sp0[lane] = incl - len;
        if (lane == 0) sp0[64] = tot;
        wave_lds_sync();
        for (int fb = 0; fb < tot; fb += 256) {
            int jr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = min(fb + lane + 64 * r, tot - 1);
                int lo = 0, hi = 63;  // largest u with sp0[u] <= f
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sp0[mid] <= f)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                jr[r] = g.vs_idx[sa[lo] + (f - sp0[lo])];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = fb + lane + 64 * r;
                const int e = w + f;
                if (f < tot && e < P) kb[e] = jr[r];
            }
        }
        w += tot;
        wave_lds_sync();
    }
    if (w > P) w = P;  // the planner's class bound makes this unreachable
    wave_lds_sync();

    int key[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int e = lane * KPL + r;
        key[r] = e < w ? kb[e] : INT_MAX;
    }
    wave_bitonic<KPL>(key, lane);
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < KPL; ++r) kb[lane * KPL + r] = key[r];
    wave_lds_sync();

    // run-length count: the head of each run of equal j holds the overlap
    int x[KPL], c[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int e = r * 64 + lane;
        x[r] = e < w ? kb[e] : INT_MAX;
        const bool head = e < w && (e == 0 || kb[e - 1] != x[r]);
        int n = 0;
        if (head) {
            n = 1;
            while (e + n < w && kb[e + n] == x[r]) ++n;
        }
        c[r] = n;  // 0 for non-heads
    }

    if (STORE) {  // every run head, in partner order
        const int64_t base = as_global(ls.off)[i];
        int tot = 0;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const bool head = c[r] > 0;
            const unsigned long long mask = __ballot(head);
            if (head) {
                const int64_t pos = base + tot + bits_below(mask);
                as_global(ls.key)[pos] = x[r];
                as_global(ls.cnt)[pos] = (uint16_t)c[r];
            }
            tot += __popcll(mask);
        }
        if (lane == 0) as_global(ls.n)[i] = tot;
    }

    const int K = ep->k;
    const int64_t S = sl.count;
    const int id0 = ep->row_base ? as_global(ep->row_base)[i] : 0;  // caller's id of row i is i - id0
    const int srow = ep->row_s ? as_global(ep->row_s)[i] : 0;
    for (int k = 0; k < K; ++k) {
        const int sk = ep->row_s ? srow : ep->s[k];
        int64_t base = EMIT ? slot_off[(int64_t)k * (S + 1) + slot] - ep->out_base[k] : 0;
        auto col = as_global(EMIT ? ep->col[k] : nullptr);
        auto wo = as_global(EMIT ? ep->w[k] : nullptr);
        auto ro = as_global(EMIT ? ep->row[k] : nullptr);
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const bool surv = c[r] >= sk;  // sk >= 1, so only run heads
            const unsigned long long mask = __ballot(surv);
            if (EMIT && surv) {
                const int64_t pos = base + bits_below(mask);
                col[pos] = x[r] - id0;
                wo[pos] = c[r];
                if (ro) ro[pos] = i - id0;
            }
            base += __popcll(mask);
        }
        if (!EMIT && lane == 0) slot_cnt[(int64_t)k * S + slot] = base;
    }
}

// ---------------------------------------------------------------------------
// K3-K5 heavy tier: one workgroup per slot, LDS bitmap + rank counters
// ---------------------------------------------------------------------------
constexpr int kHW = kHeavyThreads / 64;              // wavefronts per heavy workgroup
constexpr int kSuperWords = 1024;                    // words per rank superblock (32768 bits)
constexpr int kSupers = kRangeWords / kSuperWords;

// Emit pass of a wavefront-sort class from the light store: one wavefront
// per row reads its (partner, overlap) pairs in partner order and compacts
// every threshold's survivors with ballots.
__global__ __launch_bounds__(256) void light_store_emit_kernel(const int32_t *__restrict__ list, int64_t count,
                                                               Slots sl, LightStore ls, EmitParams prm,
                                                               const int64_t *__restrict__ slot_off) {
    __shared__ EmitParams sp;
    stage_params(&sp, prm);
    __syncthreads();
    const int lane = lane_id();
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= count) return;
    const int slot = list[wid];
    if (slot < prm.slot_lo || slot >= prm.slot_hi) return;  // outside the emitted chunk
    const int i = sl.row[slot];
    const int n = as_global(ls.n)[i];
    const int64_t off = as_global(ls.off)[i];
    const int K = prm.k;
    const int64_t S = sl.count;
    const int id0 = prm.row_base ? as_global(prm.row_base)[i] : 0;
    const int srow = prm.row_s ? as_global(prm.row_s)[i] : 0;
    long long b[SLG_MAX_S];
    int sk[SLG_MAX_S];
#pragma unroll
    for (int kk = 0; kk < SLG_MAX_S; ++kk) {
        b[kk] = kk < K ? slot_off[(int64_t)kk * (S + 1) + slot] - sp.out_base[kk] : 0;
        sk[kk] = kk < K ? (prm.row_s ? srow : sp.s[kk]) : INT_MAX;
    }
    for (int r0 = 0; r0 < n; r0 += 64) {
        const int r = r0 + lane;
        const bool in = r < n;
        const int key = in ? as_global(ls.key)[off + r] - id0 : 0;
        const int c = in ? (int)as_global(ls.cnt)[off + r] : 0;
#pragma unroll
        for (int kk = 0; kk < SLG_MAX_S; ++kk) {
            if (kk >= K) break;
            const bool surv = c >= sk[kk];
            const unsigned long long mask = __ballot(surv);
            if (mask == 0ull) break;
            if (surv) {
                const int64_t pos = b[kk] + bits_below(mask);
                as_global(sp.col[kk])[pos] = key;
                as_global(sp.w[kk])[pos] = c;
                if (sp.row[kk]) as_global(sp.row[kk])[pos] = i - id0;
            }
            b[kk] += __popcll(mask);
        }
    }
}

__global__ void light_work_kernel(int64_t m, const uint8_t *__restrict__ rclass, const int64_t *__restrict__ work,
                                  int32_t *__restrict__ lw) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = rclass[i];
        lw[i] = (c > kLight0 && c < kLight0 + kLightClasses) ? (int32_t)work[i] : 0;
    }
}

template <bool WIDE>
struct CounterCap {  // u16 counters packed in pairs, or u32 counters
    static constexpr int ranks = WIDE ? kRankCap / 2 : kRankCap;
};

constexpr int kThrTable = 128;  // overlaps below this find their threshold by table

struct HeavySmem {
    uint32_t bitmap[kRangeWords];        // partner j of the slot range present
    uint16_t wpre[kRangeWords];          // low 16 bits of the word's exclusive popcount prefix
    uint32_t sup[kSupers + 1];           // full prefix at each superblock start; sup[kSupers] = total
    uint32_t cnt[kRankCap / 2];          // overlap counters of the current rank window
    int32_t buf[kRankCap];               // pass-1 partners, then partner id per rank (emit)
    int32_t seg_a[kHeavyThreads];        // segment start per member of the batch
    int32_t seg_pre[kHeavyThreads + 1];  // flattened start per member of the batch
    int32_t wsum[kHW];
    int32_t nrep;                        // pass-1 repeats (partners already marked)
    int32_t wtot[SLG_MAX_S][kHW];
    unsigned long long acc[SLG_MAX_S];
    long long obase[SLG_MAX_S];
    long long wbase[SLG_MAX_S][kHW];     // output position of each wavefront's first survivor
    uint8_t thr_of[kThrTable];           // threshold index of an overlap value (0xFF: none)
};

// Rank of the first bit of word x (x < number of words in use).
__device__ __forceinline__ uint32_t word_rank(const HeavySmem &sm, int x) {
    const uint32_t base = sm.sup[x / kSuperWords];
    if ((x % kSuperWords) == 0) return base;
    return base + ((uint32_t)(sm.wpre[x] - (uint16_t)base) & 0xFFFFu);
}

// Lay out segments [a, a+len) of one batch of members for the balanced
// walk; returns the batch's 2-path count. Ends with a workgroup barrier.
__device__ __forceinline__ int layout_segments(int a, int len, HeavySmem &sm) {
    const int tid = threadIdx.x;
    int total;
    const int excl = block_excl_scan_open<kHeavyThreads>(len, sm.wsum, total);
    sm.seg_a[tid] = a;
    sm.seg_pre[tid] = excl;
    if (tid == 0) sm.seg_pre[kHeavyThreads] = total;
    __syncthreads();
    return total;
}

// Segment of member q = qb + tid from the boundary table, optionally clipped
// to [ka, kb) by binary search.
template <bool CLIP>
__device__ __forceinline__ void member_segment(const int32_t *__restrict__ vs_idx,
                                               const int32_t *__restrict__ bounds, int64_t bptr,
                                               int k, int qb, int ka, int kb, int &a, int &len) {
    const int q = qb + threadIdx.x;
    a = 0;
    len = 0;
    if (q < k) {
        a = bounds[bptr + q];
        int b = bounds[bptr + k + q];
        if (CLIP && a < b) {
            if (vs_idx[a] < ka) a = lower_bound_i32(vs_idx, a, b, ka);
            if (a < b && vs_idx[b - 1] >= kb) b = lower_bound_i32(vs_idx, a, b, kb);
        }
        len = b > a ? b - a : 0;
    }
}

// Largest u in [lo, hi] with seg_pre[u] <= f (seg_pre is non-decreasing).
__device__ __forceinline__ int segment_of(const int32_t *seg_pre, int lo, int hi, int f) {
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_pre[mid] <= f)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Calls f(f_idx, j, valid) with every lane of the wavefront for every piece
// of the laid-out segments (valid marks the lanes that hold a partner j,
// f_idx being its position in the batch's flattened 2-path list). Each wavefront takes
// an equal share of the list (so a heavy vertex's tail is shared by all
// wavefronts) and walks it in pieces of 64*kWalkUnroll positions: every
// lane finds the segment of each of its positions by binary search between
// the piece's first and last segment, then issues all its loads together,
// so a piece costs one round trip however many tails it touches.
constexpr int kWalkUnroll = 8;

template <typename F>
__device__ __forceinline__ void walk_segments(const int32_t *__restrict__ vs_idx, int total, int nseg,
                                              const HeavySmem &sm, F &&f) {
    if (total <= 0) return;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int per = (total + kHW - 1) / kHW;
    const int c0 = wave * per;
    const int c1 = min(total, c0 + per);
    if (c0 >= c1) return;
    const int useg = min(nseg, kHeavyThreads) - 1;  // last segment of the batch
    int ufirst = segment_of(sm.seg_pre, 0, useg, c0);
    for (int pb = c0; pb < c1; pb += 64 * kWalkUnroll) {
        const int plast = min(c1, pb + 64 * kWalkUnroll) - 1;
        const int ulast = segment_of(sm.seg_pre, ufirst, useg, plast);
        // the lane's positions search [ufirst, ulast] in lockstep, with a
        // fixed step count, so that their LDS reads overlap
        int fq[kWalkUnroll], u[kWalkUnroll];
#pragma unroll
        for (int r = 0; r < kWalkUnroll; ++r) {
            fq[r] = min(pb + lane + 64 * r, plast);
            u[r] = ufirst;
        }
        for (int len = ulast - ufirst + 1; len > 1;) {
            const int half = len >> 1;
#pragma unroll
            for (int r = 0; r < kWalkUnroll; ++r)
                u[r] = sm.seg_pre[u[r] + half] <= fq[r] ? u[r] + half : u[r];
            len -= half;
        }
        int jr[kWalkUnroll];
#pragma unroll
        for (int r = 0; r < kWalkUnroll; ++r) jr[r] = vs_idx[sm.seg_a[u[r]] + (fq[r] - sm.seg_pre[u[r]])];
#pragma unroll
        for (int r = 0; r < kWalkUnroll; ++r) {
            const int fr = pb + lane + 64 * r;
            f(fr, jr[r], fr <= plast);
        }
        ufirst = ulast;
    }
}

// Largest u in [lo, hi] with seg_pre[u] <= f, for wave-uniform lo, hi and f
// (seg_pre[lo] <= f): every lane tests one of 64 evenly spaced candidates,
// so 512 segments take two LDS round trips.
__device__ __forceinline__ int wave_segment_of(const int32_t *seg_pre, int lo, int hi, int f) {
    const int lane = lane_id();
    while (hi > lo) {
        const int step = (hi - lo + 64) / 64;
        const int cand = lo + lane * step;
        const bool ok = cand <= hi && seg_pre[cand] <= f;
        lo += (__popcll(__ballot(ok)) - 1) * step;  // the candidates that pass form a prefix
        hi = min(hi, lo + step - 1);
    }
    return lo;
}

// Pass 1 of a heavy slot: marks partner j of every laid-out 2-path in the
// bitmap over [ja, ja + span). With RECORD, a 2-path whose partner was
// already marked (a repeat) is appended to buf (up to cap entries; nrep
// counts them all). The walk is that of walk_segments, with each piece's
// atomics issued together and one list reservation per piece.
// Pass 1 takes pieces of 4 positions per lane: a slot holds about 2,600
// 2-paths on the power-law workload, so larger pieces leave wavefronts idle
// at the slot's end (8 positions measured 4 % slower, 16 positions 18 %).
constexpr int kMarkUnroll = 4;

template <bool RECORD>
__device__ __forceinline__ void walk_mark(const int32_t *__restrict__ vs_idx, int total, int nseg, HeavySmem &sm,
                                          int ja, unsigned span, int cap) {
    if (total <= 0) return;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int per = (total + kHW - 1) / kHW;
    const int c0 = wave * per;
    const int c1 = min(total, c0 + per);
    if (c0 >= c1) return;
    const int useg = min(nseg, kHeavyThreads) - 1;
    int ufirst = wave_segment_of(sm.seg_pre, 0, useg, c0);
    for (int pb = c0; pb < c1; pb += 64 * kMarkUnroll) {
        const int plast = min(c1, pb + 64 * kMarkUnroll) - 1;
        const int ulast = wave_segment_of(sm.seg_pre, ufirst, useg, plast);
        int fq[kMarkUnroll], u[kMarkUnroll];
#pragma unroll
        for (int r = 0; r < kMarkUnroll; ++r) {
            fq[r] = min(pb + lane + 64 * r, plast);
            u[r] = ufirst;
        }
        for (int len = ulast - ufirst + 1; len > 1;) {
            const int half = len >> 1;
#pragma unroll
            for (int r = 0; r < kMarkUnroll; ++r)
                u[r] = sm.seg_pre[u[r] + half] <= fq[r] ? u[r] + half : u[r];
            len -= half;
        }
        int jr[kMarkUnroll];
#pragma unroll
        for (int r = 0; r < kMarkUnroll; ++r) jr[r] = vs_idx[sm.seg_a[u[r]] + (fq[r] - sm.seg_pre[u[r]])];
        // rows of the piece past its end are skipped; lanes past it OR
        // nothing into a word of their own bank
        unsigned bit[kMarkUnroll], old[kMarkUnroll];
#pragma unroll
        for (int r = 0; r < kMarkUnroll; ++r) {
            bit[r] = 0u;
            old[r] = 0u;
            if (pb + 64 * r <= plast) {  // wave-uniform
                const unsigned off = (unsigned)(jr[r] - ja);
                const bool ok = pb + lane + 64 * r <= plast && off < span;
                bit[r] = ok ? 1u << (off & 31) : 0u;
                const unsigned word = ok ? off >> 5 : (unsigned)(lane & 31);
                if (RECORD)
                    old[r] = atomicOr(&sm.bitmap[word], bit[r]);
                else
                    atomicOr(&sm.bitmap[word], bit[r]);
            }
        }
        if (RECORD) {
            unsigned long long m[kMarkUnroll];
            int tot = 0;
#pragma unroll
            for (int r = 0; r < kMarkUnroll; ++r) {
                m[r] = __ballot((old[r] & bit[r]) != 0u);
                tot += __popcll(m[r]);
            }
            if (tot) {  // wave-uniform
                int at = 0;
                if (lane == 0) at = atomicAdd(&sm.nrep, tot);
                at = __builtin_amdgcn_readfirstlane(at);
#pragma unroll
                for (int r = 0; r < kMarkUnroll; ++r) {
                    if ((old[r] & bit[r]) != 0u) {
                        const int pos = at + bits_below(m[r]);
                        if (pos < cap) sm.buf[pos] = jr[r];
                    }
                    at += __popcll(m[r]);
                }
            }
        }
        ufirst = ulast;
    }
}

// Adds one to rank r's counter and returns the count it held before.
template <bool WIDE>
__device__ __forceinline__ int count_add_rtn(uint32_t *cnt, uint32_t r) {
    if (WIDE) return (int)atomicAdd(&cnt[r], 1u);
    const unsigned sh = (r & 1u) << 4;
    return (int)((atomicAdd(&cnt[r >> 1], 1u << sh) >> sh) & 0xFFFFu);
}

template <bool WIDE>
__device__ __forceinline__ int count_get(const uint32_t *cnt, int r) {
    if (WIDE) return (int)cnt[r];
    return (int)((cnt[r >> 1] >> ((r & 1) << 4)) & 0xFFFFu);
}

// Four 256-thread workgroups per CU (4 waves per SIMD) is what the LDS
// footprint allows; the register budget is held to match (<= 128 VGPRs).
// Four slots in flight per CU hide the latency of each slot's phases.
// STORE (counting pass of non-wide slots): the pass also writes every
// slot's partners and overlaps in rank order, so that the emit pass reads
// them instead of walking the 2-paths again.
template <bool EMIT, bool WIDE, bool STORE>
__global__ __launch_bounds__(kHeavyThreads) __attribute__((amdgpu_waves_per_eu(4))) void heavy_kernel(const HeavyDesc *__restrict__ desc,
                                                              int64_t count, int64_t S,
                                                              const int32_t *__restrict__ bounds,
                                                              const int32_t *__restrict__ vs_idx,
                                                              EmitParams prm,
                                                              int64_t *__restrict__ slot_cnt,
                                                              const int64_t *__restrict__ slot_off,
                                                              unsigned long long *__restrict__ ticket,
                                                              CountStore cs) {
    static_assert(!STORE || (!EMIT && !WIDE), "the store is written by the non-wide counting pass");
    constexpr int kCap = CounterCap<WIDE>::ranks;
    __shared__ HeavySmem sm;
    __shared__ EmitParams sp;  // thresholds and outputs, indexed by a uniform k
    __shared__ int64_t next_pair;  // first slot of the pair claimed to follow the current one
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    stage_params(&sp, prm);
    if (tid == 0) next_pair = (int64_t)atomicAdd(ticket, 2ull);
    for (int x = tid; x < kRangeWords; x += kHeavyThreads) sm.bitmap[x] = 0u;
    for (int x = tid; x < kRankCap / 2; x += kHeavyThreads) sm.cnt[x] = 0u;
    if (tid < SLG_MAX_S * kHW) sm.wtot[tid / kHW][tid % kHW] = 0;
    if (tid < kThrTable) sm.thr_of[tid] = 0xFF;
    __syncthreads();
    if (tid < prm.k && prm.s[tid] < kThrTable) sm.thr_of[prm.s[tid]] = (uint8_t)tid;
    __syncthreads();
    const EmitParams *ep = &sp;
    const int K = prm.k;
    const bool row_thr = prm.row_s != nullptr;  // batched form: one threshold per row
    int64_t pair = next_pair;  // first slot of the current pair
    int64_t it = pair;         // the current slot
    if (it >= count) return;

    // Persistent workgroups claim slots two at a time from a ticket counter.
    // Software pipeline: the claim of the next pair is made during the
    // first slot of the current pair and read one slot later; the next
    // slot's descriptor, output bases, per-row values and this thread's
    // member segment are loaded while the current slot is processed.
    HeavyDesc nd = desc[it];
    int na = 0, nb = 0, nsrow = 0, nid0 = 0;
    int64_t nob = 0;
    auto prefetch = [&](const HeavyDesc &n) {
        if (tid < n.k) {
            na = bounds[n.bptr + tid];
            nb = bounds[n.bptr + n.k + tid];
        }
        if (EMIT && tid < K) nob = slot_off[(int64_t)tid * (S + 1) + n.slot] - ep->out_base[tid];
        if (ep->row_s) nsrow = as_global(ep->row_s)[n.row];  // per-row threshold (batched form)
        if (ep->row_base) nid0 = as_global(ep->row_base)[n.row];
    };
    prefetch(nd);
    unsigned long long claim = 0;  // tid 0's claim of the next pair
    while (true) {
        const HeavyDesc d = nd;
        const int ra = na, rb = nb, srow = nsrow, id0 = nid0;
        const bool first = it == pair;
        if (first && tid == 0) claim = atomicAdd(ticket, 2ull);  // read at the end of this slot

        const int i = d.row, ja = d.ja, jb = d.jb, k = d.k, slot = d.slot;
        const int s_bottom = row_thr ? srow : ep->s[0];   // smallest and largest threshold
        const int s_top = row_thr ? srow : ep->s[K - 1];
        const bool only_presence = !EMIT && !STORE && K == 1 && s_bottom <= 1;
        const int nw = (jb - ja + 31) >> 5;
        const unsigned span = (unsigned)(jb - ja);
        // bitmap and counters are all-zero here: cleared before the first
        // slot and at the end of every slot
        if (tid < SLG_MAX_S) {
            sm.acc[tid] = 0;
            sm.obase[tid] = (EMIT && tid < K) ? nob : 0;
        }
        if (tid == 0) sm.nrep = 0;
        __syncthreads();
        // the pair's second slot, else the first of the claimed pair (published
        // at the end of the current pair's first slot)
        const int64_t it_next = first ? (it + 1 < count ? it + 1 : count) : next_pair;
        const bool have_next = it_next < count;
        if (have_next) nd = desc[it_next];
        bool acc_out = !EMIT;  // slot_cnt takes the per-threshold tallies
        do {
        if (EMIT && (slot < ep->slot_lo || slot >= ep->slot_hi)) {  // outside the emitted chunk
            if (have_next) prefetch(nd);
            break;
        }

        // pass 1: mark every partner j of the slot's range. A 2-path whose
        // partner was already marked is a repeat; repeats are listed in LDS
        // (while they fit), so that pass 2 only has to count them: a
        // partner's overlap is 1 + its number of repeats.
        const bool one_batch = k <= kHeavyThreads;
        int total1 = 0;
        if (one_batch) {
            const int len = (tid < k && rb > ra) ? rb - ra : 0;
            total1 = layout_segments(ra, len, sm);
            walk_mark<true>(vs_idx, total1, k, sm, ja, span, kRankCap);
            __syncthreads();
        } else {
            for (int qb = 0; qb < k; qb += kHeavyThreads) {
                int a, len;
                member_segment<false>(vs_idx, bounds, d.bptr, k, qb, 0, 0, a, len);
                walk_mark<true>(vs_idx, layout_segments(a, len, sm), k - qb, sm, ja, span, kRankCap);
                __syncthreads();
            }
        }
        if (have_next) prefetch(nd);

        // rank of a partner = number of marked partners below it. Each thread
        // owns 8 consecutive bitmap words, read and written 16 bytes at a time
        // (words past the slot's range are zero).
        static_assert(kRangeWords == 8 * kHeavyThreads, "8 bitmap words per thread");
        const uint4 q0 = reinterpret_cast<const uint4 *>(sm.bitmap)[2 * tid];
        const uint4 q1 = reinterpret_cast<const uint4 *>(sm.bitmap)[2 * tid + 1];
        const int loc[8] = {(int)__popc(q0.x), (int)__popc(q0.y), (int)__popc(q0.z), (int)__popc(q0.w),
                            (int)__popc(q1.x), (int)__popc(q1.y), (int)__popc(q1.z), (int)__popc(q1.w)};
        int mine = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) mine += loc[r];
        int distinct;
        int run = block_excl_scan_open<kHeavyThreads>(mine, sm.wsum, distinct);
        if ((tid * 8) % kSuperWords == 0) sm.sup[tid * 8 / kSuperWords] = (uint32_t)run;
        uint32_t pk[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t lo = (uint32_t)run & 0xFFFFu;
            run += loc[2 * r];
            pk[r] = lo | (((uint32_t)run & 0xFFFFu) << 16);
            run += loc[2 * r + 1];
        }
        reinterpret_cast<uint4 *>(sm.wpre)[tid] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
        if (tid == 0) sm.sup[kSupers] = (uint32_t)distinct;
        if (STORE && tid == 0) as_global(cs.n)[it] = distinct;
        __syncthreads();

        if (only_presence) {  // L_1 alone: every marked partner is an edge
            if (tid == 0) slot_cnt[slot] = distinct;
            acc_out = false;
            break;
        }

        // windows of at most kCap ranks, cut at word boundaries
        int w0 = 0;
        while (w0 < nw) {
            const uint32_t r0 = word_rank(sm, w0);
            int wl = w0 + 1, wh = nw;
            if ((uint32_t)distinct - r0 <= (uint32_t)kCap) wl = wh = nw;  // one window holds the rest
            while (wl < wh) {
                const int mid = (wl + wh + 1) >> 1;
                if ((mid == nw ? (uint32_t)distinct : word_rank(sm, mid)) - r0 <= (uint32_t)kCap)
                    wl = mid;
                else
                    wh = mid - 1;
            }
            const int w1 = wl;
            const int nr = (int)((w1 == nw ? (uint32_t)distinct : word_rank(sm, w1)) - r0);
            if (nr > 0) {
                const int nwords = WIDE ? nr : (nr + 1) >> 1;
                // every wavefront owns a contiguous range of ranks
                const int per = (((nr + kHW - 1) / kHW) + 63) & ~63;
                const int rlo = wave * per;
                const int rhi = min(nr, rlo + per);
                const bool whole = w0 == 0 && w1 == nw;
                // the repeat list serves every window of the counting pass, and
                // the single window of the emit pass (whose rank-to-partner map
                // reuses the list's storage afterwards)
                const int nrep = sm.nrep;
                const bool by_repeats = nrep <= kRankCap && (whole || !(EMIT || STORE));
                const int c_add = by_repeats ? 1 : 0;  // partners start at overlap 1
                // pass 2: count 2-paths into their partner's rank. The overlap of
                // a partner passes every value up to its final one exactly once,
                // so the 2-path that takes it to s_k makes it a survivor of
                // threshold k: one tally for the wavefront that owns its rank.
                auto add = [&](int, int j, bool valid) {
                    const unsigned off = (unsigned)(j - ja);
                    if (!valid || off >= span) return;
                    const int x = (int)(off >> 5);
                    const uint32_t r = word_rank(sm, x) + __popc(sm.bitmap[x] & ((1u << (off & 31)) - 1u)) - r0;
                    if (r >= (uint32_t)nr) return;
                    const int reached = count_add_rtn<WIDE>(sm.cnt, r) + 1 + c_add;
                    if (reached > s_top) return;
                    int hit = -1;
                    if (row_thr) {
                        hit = reached == srow ? 0 : -1;
                    } else if (reached < kThrTable) {
                        const int t = sm.thr_of[reached];
                        hit = t == 0xFF ? -1 : t;
                    } else {
                        for (int kk = 0; kk < K; ++kk) {
                            const int s = ep->s[kk];
                            if (s >= reached) {
                                hit = s == reached ? kk : -1;
                                break;
                            }
                        }
                    }
                    if (hit >= 0) atomicAdd(&sm.wtot[hit][r / per], 1);
                };
                if (by_repeats) {
                    int f = tid;
                    for (; f + 3 * kHeavyThreads < nrep; f += 4 * kHeavyThreads) {
                        const int j0 = sm.buf[f], j1 = sm.buf[f + kHeavyThreads];
                        const int j2 = sm.buf[f + 2 * kHeavyThreads], j3 = sm.buf[f + 3 * kHeavyThreads];
                        add(f, j0, true);
                        add(f, j1, true);
                        add(f, j2, true);
                        add(f, j3, true);
                    }
                    for (; f < nrep; f += kHeavyThreads) add(f, sm.buf[f], true);
                    __syncthreads();
                } else if (one_batch && whole) {
                    walk_segments(vs_idx, total1, k, sm, add);  // segments of pass 1 still laid out
                    __syncthreads();
                } else {
                    const int ka = ja + 32 * w0;
                    const int kb = min(jb, ja + 32 * w1);
                    for (int qb = 0; qb < k; qb += kHeavyThreads) {
                        int a, len;
                        member_segment<true>(vs_idx, bounds, d.bptr, k, qb, ka, kb, a, len);
                        walk_segments(vs_idx, layout_segments(a, len, sm), k - qb, sm, add);
                        __syncthreads();
                    }
                }
                // threshold 1 over the repeat list: every rank survives
                if (c_add && lane == 0 && s_bottom == 1) sm.wtot[0][wave] = rhi > rlo ? rhi - rlo : 0;
                if (EMIT || STORE) {
                    // partner of every rank of the window: neighbouring threads
                    // take neighbouring words, so a dense stretch of partners is
                    // shared out (4 % faster than each thread's own 8 words)
                    for (int x = w0 + tid; x < w1; x += kHeavyThreads) {
                        unsigned bits = sm.bitmap[x];
                        if (!bits) continue;
                        int rr = (int)(word_rank(sm, x) - r0);
                        const int jbase = ja + 32 * x;
                        do {
                            sm.buf[rr++] = jbase + __ffs(bits) - 1;
                            bits &= bits - 1u;
                        } while (bits);
                    }
                }
                __syncthreads();
                if (STORE) {  // the window's partners and overlaps, coalesced
                    static_assert(kRangeBits <= (1 << 16) && kWideMembers <= (1 << 16), "16-bit store fields");
                    const int64_t base = as_global(cs.off)[it] + r0;
                    for (int r = tid; r < nr; r += kHeavyThreads)  // whole lines, read much later
                        __builtin_nontemporal_store(
                            (uint32_t)(sm.buf[r] - ja) | ((uint32_t)(count_get<WIDE>(sm.cnt, r) + c_add) << 16),
                            &as_global(cs.ent)[base + r]);
                }
                if (tid < K) {  // each threshold's wavefront offsets and total, by one thread
                    long long b = EMIT ? sm.obase[tid] : 0;
#pragma unroll
                    for (int w = 0; w < kHW; ++w) {
                        if (EMIT) sm.wbase[tid][w] = b;
                        b += sm.wtot[tid][w];
                    }
                    if (EMIT)
                        sm.obase[tid] = b;
                    else
                        sm.acc[tid] += (unsigned long long)b;
                }
                if (EMIT && K <= 4) {
                    __syncthreads();
                    // up to four thresholds in one sweep over this wavefront's
                    // ranks: each count and partner is read once, thresholds
                    // and output positions stay in scalar registers
                    int sk4[4], left[4];
                    long long b4[4];
                    int32_t *col4[4], *w4[4], *row4[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        sk4[kk] = uniform(kk < K ? (row_thr ? srow : ep->s[kk]) : INT_MAX);
                        left[kk] = uniform(kk < K ? sm.wtot[kk][wave] : 0);
                        b4[kk] = uniform(kk < K ? sm.wbase[kk][wave] : 0ll);
                        col4[kk] = uniform(kk < K ? ep->col[kk] : nullptr);
                        w4[kk] = uniform(kk < K ? ep->w[kk] : nullptr);
                        row4[kk] = uniform(kk < K ? ep->row[kk] : nullptr);
                    }
                    for (int rbase = rlo; rbase < rhi && left[0] + left[1] + left[2] + left[3] > 0; rbase += 64) {
                        const int r = rbase + lane;
                        const int c = r < rhi ? count_get<WIDE>(sm.cnt, r) + c_add : 0;
                        const bool any = c >= sk4[0];  // thresholds increase
                        const int key = any ? sm.buf[r] - id0 : 0;
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            if (left[kk] == 0) continue;  // wave-uniform
                            const bool surv = c >= sk4[kk];
                            const unsigned long long mask = __ballot(surv);
                            if (surv) {
                                const int64_t pos = b4[kk] + bits_below(mask);
                                as_global(col4[kk])[pos] = key;
                                as_global(w4[kk])[pos] = c;
                                if (row4[kk]) as_global(row4[kk])[pos] = i - id0;
                            }
                            b4[kk] += __popcll(mask);
                            left[kk] -= __popcll(mask);
                        }
                    }
                } else if (EMIT) {
                    __syncthreads();
                    // per threshold, this wavefront's survivors in rank order,
                    // compacted with ballots into consecutive positions
                    for (int kk = 0; kk < K; ++kk) {
                        int left = sm.wtot[kk][wave];
                        if (left == 0) continue;
                        const int sk = row_thr ? srow : ep->s[kk];
                        int64_t base = sm.wbase[kk][wave];
                        const auto colp = as_global(ep->col[kk]);
                        const auto wp = as_global(ep->w[kk]);
                        const auto rowp = as_global(ep->row[kk]);
                        // two groups of 64 ranks per step: their LDS reads overlap
                        for (int rbase = rlo; rbase < rhi && left > 0; rbase += 128) {
                            const int ra_ = rbase + lane, rb_ = rbase + 64 + lane;
                            const int ca = ra_ < rhi ? count_get<WIDE>(sm.cnt, ra_) + c_add : 0;
                            const int cb = rb_ < rhi ? count_get<WIDE>(sm.cnt, rb_) + c_add : 0;
                            const bool sa = ca >= sk, sb = cb >= sk;
                            const int ka_ = sa ? sm.buf[ra_] : 0;
                            const int kb_ = sb ? sm.buf[rb_] : 0;
                            const unsigned long long ma = __ballot(sa), mb = __ballot(sb);
                            const int na_ = __popcll(ma);
                            if (sa) {
                                const int64_t pos = base + bits_below(ma);
                                colp[pos] = ka_ - id0;
                                wp[pos] = ca;
                                if (rowp) rowp[pos] = i - id0;
                            }
                            if (sb) {
                                const int64_t pos = base + na_ + bits_below(mb);
                                colp[pos] = kb_ - id0;
                                wp[pos] = cb;
                                if (rowp) rowp[pos] = i - id0;
                            }
                            base += na_ + __popcll(mb);
                            left -= na_ + __popcll(mb);
                        }
                    }
                }
                __syncthreads();
                for (int x = tid; x < nwords; x += kHeavyThreads) sm.cnt[x] = 0u;
                if (tid < SLG_MAX_S * kHW) sm.wtot[tid / kHW][tid % kHW] = 0;
                if (w1 < nw) __syncthreads();  // the next window counts into cleared counters
            }
            w0 = w1;
        }
        } while (false);
        for (int x = tid; x < nw; x += kHeavyThreads) sm.bitmap[x] = 0u;
        if (first && tid == 0) next_pair = (int64_t)claim;
        __syncthreads();
        if (acc_out && tid < K) slot_cnt[(int64_t)tid * S + slot] = (int64_t)sm.acc[tid];
        if (!have_next) break;
        if (!first) pair = it_next;
        it = it_next;
    }
}

// 2-paths of every heavy slot: the lengths of its members' segments in the
// boundary table, one wavefront per slot.
__global__ __launch_bounds__(256) void slot_work_kernel(const HeavyDesc *__restrict__ desc, int64_t count,
                                                        const int32_t *__restrict__ bounds,
                                                        int64_t *__restrict__ work) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; t < count; t += nwaves) {
        const HeavyDesc d = desc[t];
        int64_t w = 0;
        for (int q = lane; q < d.k; q += 64) w += bounds[d.bptr + d.k + q] - bounds[d.bptr + q];
        w = wave_sum(w);
        if (lane == 0) work[t] = w;
    }
}

// Emit pass of the heavy slots from the counting pass's store: one
// wavefront per slot reads its entries in rank (partner id) order, eight
// groups of 64 ranks per step (all loads issued before any is used). Each
// threshold's survivors are compacted with ballots into a small LDS queue
// of the wavefront and written out 64 at a time, so that every global store
// is a full, coalesced 256-byte row even for sparse thresholds; what is
// left is written at the end of the slot. Thresholds increase, so a group
// with no survivor of s_k has none of the larger ones either. MAXK: 4 for
// ensembles of up to four thresholds, else SLG_MAX_S (no queues).
constexpr int kStoreGroups = 8;
constexpr int kQueue = 128;  // entries per threshold queue: < 64 kept + <= 64 appended

// Entries are (partner - ja) | overlap << 16. DENSE: ja is a window of E_s
// positions and the partner's id is cid_row[ja + low half], looked up for a
// whole group of entries at once (the lookups overlap) before they are
// queued as id << 16 | overlap. Slots are taken in list (row) order, so the
// outputs are written in order; taking them window by window kept cid_row
// in L2 but scattered the writes, and measured a third slower.
template <int MAXK, bool DENSE>
__global__ __launch_bounds__(256) void heavy_store_emit_kernel(const HeavyDesc *__restrict__ desc, int64_t count,
                                                               int64_t S, CountStore cs, EmitParams prm,
                                                               const int64_t *__restrict__ slot_off,
                                                               const int32_t *__restrict__ cid_row) {
    using E = uint32_t;                                        // stored entry
    using Q = typename std::conditional<DENSE, unsigned long long, uint32_t>::type;  // queued entry
    constexpr bool kQueued = MAXK <= 4;
    __shared__ EmitParams sp;
    __shared__ Q queue[kQueued ? 4 : 1][kQueued ? MAXK : 1][kQueued ? kQueue : 1];
    stage_params(&sp, prm);
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int K = prm.k;
    const bool row_thr = prm.row_s != nullptr;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    // one slot: its stored entries to the outputs of every threshold
    auto emit_slot = [&](int64_t t) {
        const HeavyDesc d = desc[t];
        if (d.slot < prm.slot_lo || d.slot >= prm.slot_hi) return;  // outside the emitted chunk
        const int n = as_global(cs.n)[t];
        if (n < 0) return;  // the store was full: the slot's emit walks its 2-paths again
        const int64_t off = as_global(cs.off)[t];
        const int i = d.row;
        const int id0 = prm.row_base ? as_global(prm.row_base)[i] : 0;
        const int srow = row_thr ? as_global(prm.row_s)[i] : 0;
        const int jbase = d.ja - id0;
        const int32_t *crow = DENSE ? cid_row + d.ja : nullptr;
        long long b[MAXK];
        int sk[MAXK], fill[MAXK];
#pragma unroll
        for (int kk = 0; kk < MAXK; ++kk) {
            b[kk] = kk < K ? slot_off[(int64_t)kk * (S + 1) + d.slot] - sp.out_base[kk] : 0;
            sk[kk] = kk < K ? (row_thr ? srow : sp.s[kk]) : INT_MAX;
            fill[kk] = 0;
        }
        // queued entry: DENSE, the partner's id << 16 | overlap; else the stored entry
        auto partner = [&](Q e) -> int {
            return DENSE ? (int)(e >> 16) - id0 : jbase + (int)(e & 0xFFFFu);
        };
        auto overlap = [&](Q e) -> int { return DENSE ? (int)(e & 0xFFFFu) : (int)(e >> 16); };
        // writes `m` queued entries of threshold kk (lanes below m) at b[kk]
        auto flush = [&](int kk, int m) {
            if (lane < m) {
                const Q e = queue[wave][kk][lane];
                const int64_t pos = b[kk] + lane;
                as_global(sp.col[kk])[pos] = partner(e);
                as_global(sp.w[kk])[pos] = overlap(e);
                if (sp.row[kk]) as_global(sp.row[kk])[pos] = i - id0;
            }
            b[kk] += m;
        };
        for (int r0 = 0; r0 < n; r0 += 64 * kStoreGroups) {
            E e[kStoreGroups];
#pragma unroll
            for (int q = 0; q < kStoreGroups; ++q) {
                const int r = r0 + 64 * q + lane;
                e[q] = r < n ? as_global(cs.ent)[off + r] : E(0);
            }
            Q v[kStoreGroups];
#pragma unroll
            for (int q = 0; q < kStoreGroups; ++q) {
                if (DENSE)
                    v[q] = r0 + 64 * q + lane < n
                               ? ((Q)(uint32_t)as_global(crow)[e[q] & 0xFFFFu] << 16) | (Q)(e[q] >> 16)
                               : Q(0);
                else
                    v[q] = (Q)e[q];
            }
#pragma unroll
            for (int q = 0; q < kStoreGroups; ++q) {
                if (r0 + 64 * q >= n) break;  // wave-uniform
                const int c = overlap(v[q]);
#pragma unroll
                for (int kk = 0; kk < MAXK; ++kk) {
                    if (kk >= K) break;
                    const bool surv = c >= sk[kk];
                    const unsigned long long mask = __ballot(surv);
                    if (mask == 0ull) break;
                    if (kQueued) {
                        if (surv) queue[wave][kk][fill[kk] + bits_below(mask)] = v[q];
                        fill[kk] += __popcll(mask);
                        if (fill[kk] >= 64) {  // a full row out, the rest moves down
                            wave_lds_sync();
                            flush(kk, 64);
                            const Q rest = lane < fill[kk] - 64 ? queue[wave][kk][64 + lane] : Q(0);
                            wave_lds_sync();
                            if (lane < fill[kk] - 64) queue[wave][kk][lane] = rest;
                            fill[kk] -= 64;
                        }
                    } else if (surv) {
                        const int64_t pos = b[kk] + bits_below(mask);
                        as_global(sp.col[kk])[pos] = partner(v[q]);
                        as_global(sp.w[kk])[pos] = c;
                        if (sp.row[kk]) as_global(sp.row[kk])[pos] = i - id0;
                    }
                    if (!kQueued) b[kk] += __popcll(mask);
                }
            }
        }
        if (kQueued) {
            wave_lds_sync();
#pragma unroll
            for (int kk = 0; kk < MAXK; ++kk)
                if (kk < K && fill[kk] > 0) flush(kk, fill[kk]);
            wave_lds_sync();  // the queues are reused by the next slot
        }
    };
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; t < count; t += nwaves) emit_slot(t);
}

__global__ void sum_i32_kernel(const int32_t *__restrict__ n, int64_t count, unsigned long long *__restrict__ out) {
    unsigned long long acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        acc += (unsigned long long)n[t];
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(out, acc);
}

// Edges of every threshold emitted by heavy slots (for measurement).
__global__ __launch_bounds__(256) void heavy_edges_kernel(const HeavyDesc *__restrict__ desc,
                                                          int64_t count, const int64_t *__restrict__ slot_cnt,
                                                          int64_t S, int32_t K,
                                                          unsigned long long *__restrict__ out) {
    __shared__ unsigned long long ws[4];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long sum = 0;
    if (t < count) {
        const int slot = desc[t].slot;
        for (int k = 0; k < K; ++k) sum += (unsigned long long)slot_cnt[(int64_t)k * S + slot];
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long b = ws[0] + ws[1] + ws[2] + ws[3];
        if (b) atomicAdd(out, b);
    }
}

// One wavefront per heavy slot: the segment start of every member of the
// row at the slot's first partner id (and, on the row's last slot, the
// tail end). Partners of member q form a sorted tail, so the start is a
// lower bound; quick tests skip the search when the tail misses the slot.
__global__ __launch_bounds__(256) void bounds_kernel(
    const HeavyDesc *__restrict__ desc, int64_t count, const int64_t *__restrict__ he_ptr,
    const int32_t *__restrict__ he_idx, const int64_t *__restrict__ vs_ptr,
    const int32_t *__restrict__ vs_idx, const int32_t *__restrict__ tail_beg,
    int32_t *__restrict__ bounds) {
    // workgroups are dealt to the 8 XCDs in turn; each XCD takes runs of 16
    // consecutive blocks (64 slots) instead, so that a row's slots (which
    // search the same vertex lists) mostly share one L2, while the runs
    // still rotate over the XCDs (rows of very different cost, e.g. sorted
    // by size, stay spread). The tail past whole rounds keeps its place.
    constexpr uint32_t kRun = 16;
    const uint32_t nb = gridDim.x, b = blockIdx.x, q = b / 8u;
    const uint32_t blk = b >= nb / (8u * kRun) * (8u * kRun) ? b : q / kRun * (8u * kRun) + b % 8u * kRun + q % kRun;
    const int lane = lane_id();
    const int64_t w = ((int64_t)blk * blockDim.x + threadIdx.x) / 64;
    if (w >= count) return;
    const HeavyDesc d = desc[w];
    const int64_t p0 = he_ptr[d.row];
    for (int q = lane; q < d.k; q += 64) {
        const int64_t p = p0 + q;
        const int v = he_idx[p];
        const int beg = tail_beg[p];
        const int end = (int)vs_ptr[v + 1];
        int val = beg;
        if (beg < end && vs_idx[beg] < d.ja)
            val = vs_idx[end - 1] < d.ja ? end : lower_bound_i32(vs_idx, beg, end, d.ja);
        bounds[d.bptr + q] = val;
        if (d.last) bounds[d.bptr + d.k + q] = end;
    }
}

// ---------------------------------------------------------------------------
// K3-K5 dense tier: one workgroup per slot, direct LDS counters
// ---------------------------------------------------------------------------
// A dense slot is a row i and an aligned window [ja, ja + kDenseWindow) of
// E_s positions; its 2-paths are the parts of its members' tails that fall
// in the window (vertex lists in E_s positions, so the counter of partner c
// is c - ja with no search). One u32 counter per position. The walk reads
// the lists as 16-bit places in the window (c - ja = c mod kDenseWindow,
// since windows are aligned): 2 bytes per 2-path instead of 4 (6.5 % off
// the counting pass), and the counter's byte address is one shift, so a
// 2-path costs one load, one shift and one LDS add. A row of fewer than
// 2^16 members cannot reach 2^16 in a counter (the store keeps 16 bits).
constexpr int kDW = kDenseThreads / 64;                       // wavefronts per dense workgroup
constexpr int kDenseWordsPer = kDenseWindow / kDenseThreads;  // counters per thread (32)
constexpr int kDenseUnroll = 16;                              // loads in flight per lane
constexpr int kDensePiece = 64 * kDenseUnroll;                // 2-paths per wavefront step
// vs_win is allocated kDensePad entries longer: a step inside one tail
// loads whole rows past the tail's end (those values are not counted)
static_assert(kDensePad >= kDensePiece, "padding of the E_s-position lists");
static_assert(kDenseWordsPer % 4 == 0, "16-byte LDS accesses");
static_assert(kWideMembers < (1 << 16), "16-bit overlaps in the dense store");

struct DenseSmem {
    uint32_t cnt[kDenseWindow + 4];      // counters (and 4 spare words)
    int32_t seg_a[kDenseThreads];        // segment start per member of the batch
    int32_t seg_pre[kDenseThreads + 1];  // flattened start per member of the batch
    int32_t wsum[2][kDW];                // wavefront totals of a scan (two, used in turn)
    unsigned long long tally[SLG_MAX_S];
    long long base;                      // store room of the slot (or -1)
    long long chunk_at, chunk_end;       // the workgroup's store room not yet handed out
    int64_t next[2];                     // tickets claimed ahead, by slot parity
    int32_t tn;                          // the following slot's position in the descriptor list
};

// Exclusive scan over the dense workgroup. wsum is read after the scan's
// barrier: the next scan takes the other buffer, so that no second barrier
// is needed.
__device__ __forceinline__ int dense_scan(int x, int32_t *wsum, int &total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int incl = wave_incl_scan(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kDW; ++w) {
        const int t = wsum[w];
        pre += (w < wave) ? t : 0;
        tot += t;
    }
    total = tot;
    return pre + incl - x;
}

// Adds one to the counter at byte offset a of the counters.
__device__ __forceinline__ void dense_add(DenseSmem &sm, uint32_t a) {
    atomicAdd(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(sm.cnt) + a), 1u);
}

// Walks the laid-out segments (2-path f of the batch is member u's tail
// position seg_a[u] + f - seg_pre[u], whose place in the window is
// vs_win[that position]) and adds one to the counter of each
// partner. Each wavefront takes an equal share of the flattened list, in
// steps of kDensePiece positions whose loads are all issued first. The
// wavefront keeps its current tail (start and end) in scalar registers: a
// step inside it (the common case: the 2-paths of a dense slot come mostly
// from long tails) takes one address and the loads' immediate offsets, with
// no LDS lookup; a step across tails finds each position's tail by binary
// search. (Keeping the next step's loads in flight while adding the
// current one's measured the same: the walk is not bound by load latency.)
__device__ __forceinline__ void dense_walk(const uint16_t *__restrict__ vs_win, int total, int nseg,
                                           DenseSmem &sm) {
    if (total <= 0) return;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int per = (total + kDW - 1) / kDW;
    const int c0 = wave * per;
    const int c1 = min(total, c0 + per);
    if (c0 >= c1) return;
    const int useg = min(nseg, kDenseThreads) - 1;
    // tail u covers flattened positions [seg_pre[u], uend); position f of it
    // is vs_win[ubase + f]
    int u = wave_segment_of(sm.seg_pre, 0, useg, c0);
    int uend = uniform(sm.seg_pre[u + 1]);
    int ubase = uniform(sm.seg_a[u] - sm.seg_pre[u]);
    // adds the step at b (its positions up to c1 - 1) from values c
    auto add_step = [&](const int (&c)[kDenseUnroll], int b) {
        const int last = min(c1, b + kDensePiece) - 1;
        if (last == b + kDensePiece - 1) {  // wave-uniform: every position of the step counts
#pragma unroll
            for (int r = 0; r < kDenseUnroll; ++r) dense_add(sm, (uint32_t)c[r] * 4u);
        } else {
#pragma unroll
            for (int r = 0; r < kDenseUnroll; ++r)
                if (b + lane + 64 * r <= last) dense_add(sm, (uint32_t)c[r] * 4u);
        }
    };
    int pb = c0;
    while (pb < c1) {
        if (pb >= uend) {
            u = wave_segment_of(sm.seg_pre, u, useg, pb);
            uend = uniform(sm.seg_pre[u + 1]);
            ubase = uniform(sm.seg_a[u] - sm.seg_pre[u]);
        }
        const int plast = min(c1, pb + kDensePiece) - 1;
        if (plast < uend) {
            // a step inside tail u
            const uint16_t *src = vs_win + ((int64_t)ubase + lane);
            int ca[kDenseUnroll];
#pragma unroll
            for (int r = 0; r < kDenseUnroll; ++r) ca[r] = src[pb + 64 * r];
            add_step(ca, pb);
            pb += kDensePiece;
        } else {
            const int ulast = wave_segment_of(sm.seg_pre, u, useg, plast);
            constexpr int kHalf = kDenseUnroll / 2;
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {
                const int hb = pb + 64 * kHalf * h;
                if (hb > plast) break;  // wave-uniform
                int fq[kHalf], uq[kHalf], c[kHalf];
#pragma unroll
                for (int r = 0; r < kHalf; ++r) {
                    fq[r] = min(hb + lane + 64 * r, plast);
                    uq[r] = u;
                }
                for (int len = ulast - u + 1; len > 1;) {
                    const int half = len >> 1;
#pragma unroll
                    for (int r = 0; r < kHalf; ++r)
                        uq[r] = sm.seg_pre[uq[r] + half] <= fq[r] ? uq[r] + half : uq[r];
                    len -= half;
                }
#pragma unroll
                for (int r = 0; r < kHalf; ++r) c[r] = vs_win[sm.seg_a[uq[r]] + (fq[r] - sm.seg_pre[uq[r]])];
#pragma unroll
                for (int r = 0; r < kHalf; ++r)
                    if (hb + lane + 64 * r <= plast) dense_add(sm, (uint32_t)c[r] * 4u);
            }
            u = ulast;
            uend = uniform(sm.seg_pre[u + 1]);
            ubase = uniform(sm.seg_a[u] - sm.seg_pre[u]);
            pb += kDensePiece;
        }
    }
}

// EMIT = false: the counting pass. Every threshold's survivors are tallied
// into slot_cnt; with a store, the survivors of the smallest threshold are
// kept, in partner order, for the emit pass. EMIT = true: the emit pass of
// the slots without stored survivors (every slot when there is no store),
// writing each threshold's edges in partner order at the slot's offsets.
// Persistent workgroups take slots from a ticket counter; two fit per CU
// (LDS), which takes at most 128 VGPRs (4 waves per SIMD). The next slot's
// ticket, position, descriptor and first member segments are loaded while
// the current slot is counted, so that a slot starts with no global round
// trip. Store room is taken kDenseChunk entries at a time per workgroup
// (one global atomic per chunk rather than per slot); cursor[0] is the room
// taken, cursor[1] and cursor[2] sum the survivors asked for and kept.
template <bool EMIT>
__global__ __launch_bounds__(kDenseThreads) __attribute__((amdgpu_waves_per_eu(4))) void dense_kernel(const HeavyDesc *__restrict__ desc, int64_t count,
                                                              const int32_t *__restrict__ order,
                                                              int64_t S, const int32_t *__restrict__ bounds,
                                                              const uint16_t *__restrict__ vs_win,
                                                              const int32_t *__restrict__ cid_row, EmitParams prm,
                                                              int64_t *__restrict__ slot_cnt,
                                                              const int64_t *__restrict__ slot_off,
                                                              unsigned long long *__restrict__ ticket,
                                                              CountStore cs, unsigned long long *__restrict__ cursor,
                                                              int64_t cap) {
    __shared__ DenseSmem sm;
    __shared__ EmitParams sp;
    const int tid = threadIdx.x, lane = lane_id();
    stage_params(&sp, prm);
    for (int x = tid; x < kDenseWindow + 4; x += kDenseThreads) sm.cnt[x] = 0u;
    if (tid == 0) {
        sm.next[0] = (int64_t)atomicAdd(ticket, 1ull);
        sm.chunk_at = 0;
        sm.chunk_end = 0;
    }
    __syncthreads();
    const int K = sp.k;
    const bool store = cs.ent != nullptr;
    // the slot of ticket tk: its position in desc (window-major order) and
    // descriptor; this thread's member segment of its first batch
    auto slot_of = [&](int64_t tk) -> int64_t { return order ? (int64_t)order[tk] : tk; };
    auto first_segment = [&](const HeavyDesc &d, int &a, int &len) {
        a = 0;
        len = 0;
        if (tid < d.k) {
            a = bounds[d.bptr + tid];
            const int b = bounds[d.bptr + d.k + tid];
            len = b > a ? b - a : 0;
        }
    };
    // zero, in a form the compiler treats as varying by lane: a load indexed
    // with it is a vector load (waited for with the vector loads, not with
    // every LDS access as a scalar load would be)
    const int64_t lane_zero = (int64_t)lane * (count >> 62);
    int64_t tk = uniform((long long)sm.next[0]);
    if (tid == 0) sm.next[1] = (int64_t)atomicAdd(ticket, 1ull);  // the following slot
    int par = 1;  // next[par] holds the following slot's ticket
    int64_t t = 0;
    HeavyDesc d{};
    int a0 = 0, len0 = 0;
    if (tk < count) {
        t = uniform((long long)slot_of(tk));
        d = desc[t];
        first_segment(d, a0, len0);
    }
    while (tk < count) {
        // the following slot's ticket is in next[par]; the previous slot's
        // counters are cleared and its reads of the shared arrays are done
        __syncthreads();
        const int64_t tkn = uniform((long long)sm.next[par]);
        // the following slot's position, loaded by one lane now and shared
        // through LDS after the walk (a scalar load would be waited for at
        // the walk's first LDS access)
        int tn_v = 0;
        if (tid == 0 && tkn < count) tn_v = order ? order[tkn + lane_zero] : (int)tkn;
        const int ja = uniform(d.ja), k = uniform(d.k);
        bool skip = false;
        if (EMIT) skip = d.slot < sp.slot_lo || d.slot >= sp.slot_hi || (store && as_global(cs.n)[t] >= 0);
        if (tid < SLG_MAX_S) sm.tally[tid] = 0ull;
        if (!skip && k > 0) {  // workgroup-uniform
            // count: every member's part of its tail inside the window
            for (int qb = 0; qb < k; qb += kDenseThreads) {
                int a = a0, len = len0;
                if (qb > 0) {
                    const int q = qb + tid;
                    a = 0;
                    len = 0;
                    if (q < k) {
                        a = bounds[d.bptr + q];
                        const int b = bounds[d.bptr + k + q];
                        len = b > a ? b - a : 0;
                    }
                }
                int total;
                const int excl = dense_scan(len, sm.wsum[0], total);
                sm.seg_a[tid] = a;
                sm.seg_pre[tid] = excl;
                if (tid == 0) sm.seg_pre[kDenseThreads] = total;
                __syncthreads();
                dense_walk(vs_win, total, k - qb, sm);
                if (tid == 0) sm.tn = tn_v;
                __syncthreads();
            }
        } else {
            if (tid == 0) sm.tn = tn_v;
            __syncthreads();
        }
        // the slot after the following one (next[par ^ 1] was read before this slot's first barrier)
        if (tid == 0) sm.next[par ^ 1] = (int64_t)atomicAdd(ticket, 1ull);
        par ^= 1;
        const int64_t tn = tkn < count ? (int64_t)sm.tn : 0;
        HeavyDesc dn{};
        if (tkn < count) dn = desc[tn + lane_zero];  // vector loads: waited for at the next slot's start
        int an = 0, lenn = 0;
        // this thread's counters: positions [tid * 32, tid * 32 + 32), read
        // 16 bytes at a time; `f(position, count)` sees each in order, and
        // with `clear` they are zeroed for the next slot. A compiler barrier
        // keeps every pass a fresh read.
        auto for_words = [&](bool clear, auto &&f) {
            __asm__ volatile("" ::: "memory");
            uint4 *q = reinterpret_cast<uint4 *>(sm.cnt) + tid * (kDenseWordsPer / 4);
#pragma unroll 2
            for (int r = 0; r < kDenseWordsPer / 4; ++r) {
                const uint4 v = q[r];
                const int x = tid * kDenseWordsPer + 4 * r;
                f(x, v.x);
                f(x + 1, v.y);
                f(x + 2, v.z);
                f(x + 3, v.w);
                if (clear) q[r] = make_uint4(0u, 0u, 0u, 0u);
            }
        };
        const unsigned s0 = (unsigned)sp.s[0];
        const auto crow = as_global(cid_row) + ja;
        if (skip) {
            if (tkn < count) first_segment(dn, an, lenn);
        } else if (!EMIT) {
            // every threshold's survivors (one pass for up to two
            // thresholds), then the survivors of the smallest kept in the store
            int n0 = 0;
            if (K <= 2) {
                const unsigned s1 = K > 1 ? (unsigned)sp.s[1] : ~0u;
                int n1 = 0;
                for_words(!store, [&](int, unsigned v) {
                    n0 += v >= s0;
                    n1 += v >= s1;
                });
                n1 = wave_sum(n1);
                if (K > 1 && lane == 0 && n1) atomicAdd(&sm.tally[1], (unsigned long long)n1);
            } else {
                for (int kk = 1; kk < K; ++kk) {
                    const unsigned sk = (unsigned)sp.s[kk];
                    int c = 0;
                    for_words(false, [&](int, unsigned v) { c += v >= sk; });
                    c = wave_sum(c);
                    if (lane == 0 && c) atomicAdd(&sm.tally[kk], (unsigned long long)c);
                }
                for_words(!store, [&](int, unsigned v) { n0 += v >= s0; });
            }
            int n;
            const int pos0 = dense_scan(n0, sm.wsum[1], n);
            if (tkn < count) first_segment(dn, an, lenn);  // the descriptor has arrived by now
            if (tid == 0) sm.tally[0] = (unsigned long long)n;
            if (store && tid == 0) {  // room for the slot's survivors, from the workgroup's chunk
                long long b = -1;
                if (n > 0) {
                    if ((long long)n > sm.chunk_end - sm.chunk_at) {
                        // a chunk, or less in a small store (a quarter of it over the workgroups)
                        long long want = cap / (4ll * (long long)gridDim.x);
                        want = want < kDenseChunk ? want : kDenseChunk;
                        want = (long long)n > want ? (long long)n : want;
                        const long long at = (long long)atomicAdd(cursor, (unsigned long long)want);
                        sm.chunk_at = at;
                        sm.chunk_end = at + want <= cap ? at + want : (at + n <= cap ? at + n : at);
                    }
                    if ((long long)n <= sm.chunk_end - sm.chunk_at) {
                        b = sm.chunk_at;
                        sm.chunk_at += n;
                        atomicAdd(cursor + 2, (unsigned long long)n);
                    }
                    atomicAdd(cursor + 1, (unsigned long long)n);
                }
                sm.base = b;
                as_global(cs.off)[t] = b < 0 ? 0 : b;
                as_global(cs.n)[t] = (n > 0 && b < 0) ? -1 : n;
            }
            __syncthreads();
            if (store) {  // window position | overlap << 16
                const long long base = sm.base;
                const auto ent = as_global(cs.ent);
                long long q0 = base + pos0;
                for_words(true, [&](int x, unsigned v) {
                    if (base >= 0 && v >= s0) ent[q0++] = (uint32_t)x | (v << 16);
                });
            }
            if (tid < K) slot_cnt[(int64_t)tid * S + d.slot] = (int64_t)sm.tally[tid];
        } else {
            // per threshold, this slot's survivors in partner order
            if (tkn < count) first_segment(dn, an, lenn);
            const int i = d.row;
            for (int kk = 0; kk < K; ++kk) {
                const unsigned sk = (unsigned)sp.s[kk];
                int n0 = 0;
                for_words(false, [&](int, unsigned v) { n0 += v >= sk; });
                int tot;
                const int pos0 = dense_scan(n0, sm.wsum[(kk + 1) & 1], tot);
                if (tot == 0) break;  // workgroup-uniform: larger thresholds have none either
                const int64_t b = slot_off[(int64_t)kk * (S + 1) + d.slot] - sp.out_base[kk];
                const auto colp = as_global(sp.col[kk]);
                const auto wp = as_global(sp.w[kk]);
                const auto rowp = as_global(sp.row[kk]);
                int64_t q0 = b + pos0;
                for_words(false, [&](int x, unsigned v) {
                    if (v >= sk) {
                        colp[q0] = crow[x];
                        wp[q0] = (int)v;
                        if (rowp) rowp[q0] = i;
                        ++q0;
                    }
                });
            }
            for_words(true, [](int, unsigned) {});  // cleared for the next slot
        }
        tk = tkn;
        t = tn;
        d = dn;
        a0 = an;
        len0 = lenn;
    }
}

__global__ void dense_keys_kernel(const HeavyDesc *__restrict__ desc, int64_t count, int32_t *__restrict__ key,
                                  int32_t *__restrict__ id) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    key[t] = desc[t].ja >> kDenseBits;
    id[t] = (int32_t)t;
}

// ---------------------------------------------------------------------------
// K6: CSR row pointers from slot offsets
// ---------------------------------------------------------------------------
__global__ void row_ptr_kernel(int64_t row_lo, int64_t row_hi, const int64_t *__restrict__ slot_base,
                               const int64_t *__restrict__ slot_off, int64_t S, EmitParams prm) {
    __shared__ EmitParams sp;
    stage_params(&sp, prm);
    __syncthreads();
    const int64_t i = row_lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > row_hi) return;
    const int64_t sb = slot_base[i];
    for (int k = 0; k < sp.k; ++k)
        as_global(sp.row_ptr[k])[i - row_lo] = slot_off[(int64_t)k * (S + 1) + sb] - sp.out_base[k];
}

// Output bytes of rows [0, i) over all thresholds, i in [0, m].
__global__ void row_bytes_kernel(int64_t m, const int64_t *__restrict__ slot_base,
                                 const int64_t *__restrict__ slot_off, int64_t S, int32_t K,
                                 int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > m) return;
    const int64_t sb = slot_base[i];
    int64_t b = 0;
    for (int k = 0; k < K; ++k) b += 12 * slot_off[(int64_t)k * (S + 1) + sb] + 8 * i;
    out[i] = b;
}

// out[c * K + k] = slot_off[k][slot_base[rows[c]]].
__global__ void gather_offsets_kernel(const int64_t *__restrict__ rows, int64_t count,
                                      const int64_t *__restrict__ slot_base,
                                      const int64_t *__restrict__ slot_off, int64_t S, int32_t K,
                                      int64_t *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    const int64_t sb = slot_base[rows[c]];
    for (int k = 0; k < K; ++k) out[c * K + k] = slot_off[(int64_t)k * (S + 1) + sb];
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
__global__ void validate_ptr_kernel(const int64_t *__restrict__ ptr, int64_t rows, int64_t nnz,
                                    int *__restrict__ err) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > rows) return;
    const int64_t x = ptr[r];
    bool bad = x < 0 || x > nnz;
    if (r == 0) bad |= x != 0;
    if (r == rows) bad |= x != nnz;
    if (r < rows) bad |= ptr[r + 1] < x;
    if (bad) atomicOr(err, 2);
}

// One wavefront per row: ids in range and strictly increasing.
__global__ __launch_bounds__(256) void validate_rows_kernel(const int64_t *__restrict__ ptr,
                                                            const int32_t *__restrict__ idx,
                                                            int64_t rows, int64_t limit,
                                                            int *__restrict__ err) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; r < rows; r += nwaves) {
        const int64_t a = ptr[r], b = ptr[r + 1];
        int bad = 0;
        for (int64_t p = a + lane; p < b; p += 64) {
            const int32_t x = idx[p];
            bad |= (x < 0 || x >= limit);
            if (p > a) bad |= idx[p - 1] >= x;
        }
        if (wave_max(bad) && lane == 0) atomicOr(err, 4);
    }
}

// Every incidence (i, v) of the hyperedge CSR appears in v's list. With equal
// nnz and set-valued rows on both sides, this makes the lists transposes.
__global__ __launch_bounds__(256) void validate_transpose_kernel(
    const int64_t *__restrict__ he_ptr, const int32_t *__restrict__ he_idx, int64_t m,
    const int64_t *__restrict__ v_ptr, const int32_t *__restrict__ v_idx, int64_t n,
    int *__restrict__ err) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; i < m; i += nwaves) {
        int bad = 0;
        for (int64_t p = he_ptr[i] + lane; p < he_ptr[i + 1]; p += 64) {
            const int v = he_idx[p];
            if (v < 0 || v >= n) {
                bad = 1;
                continue;
            }
            const int lo = (int)v_ptr[v], hi = (int)v_ptr[v + 1];
            const int a = lower_bound_i32(v_idx, lo, hi, (int)i);
            bad |= !(a < hi && v_idx[a] == (int)i);
        }
        if (wave_max(bad) && lane == 0) atomicOr(err, 8);
    }
}

// Disjoint union of a batch of hypergraphs: graph g's hyperedges and
// vertices get ids offset by the sizes of the graphs before it.
__global__ __launch_bounds__(256) void union_kernel(const UnionPart *__restrict__ parts,
                                                    int64_t *__restrict__ he_ptr, int32_t *__restrict__ he_idx,
                                                    int64_t *__restrict__ v_ptr, int32_t *__restrict__ v_idx,
                                                    int32_t *__restrict__ row_s, int32_t *__restrict__ row_base) {
    const UnionPart u = parts[blockIdx.y];
    const int64_t lim = max(max(u.m + 1, u.n + 1), u.nnz);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < lim; t += (int64_t)gridDim.x * blockDim.x) {
        if (t <= u.m) he_ptr[u.m_off + t] = as_global(u.he_ptr)[t] + u.nnz_off;  // the shared end entry agrees
        if (t < u.m) {
            row_s[u.m_off + t] = u.s;
            row_base[u.m_off + t] = (int32_t)u.m_off;
        }
        if (t <= u.n) v_ptr[u.n_off + t] = as_global(u.v_ptr)[t] + u.nnz_off;
        if (t < u.nnz) {
            he_idx[u.nnz_off + t] = as_global(u.he_idx)[t] + (int32_t)u.n_off;
            v_idx[u.nnz_off + t] = as_global(u.v_idx)[t] + (int32_t)u.m_off;
        }
    }
}

__global__ void gather_i64_kernel(const int64_t *__restrict__ src, const int64_t *__restrict__ idx,
                                  int64_t count, int64_t *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < count) out[c] = src[idx[c]];
}

// ---------------------------------------------------------------------------
// s-connected components (Section II-B: maximal sets of E_s joined by
// s-walks) and ID squeezing, on the emitted edge list
// ---------------------------------------------------------------------------
// label[] doubles as the union-find parent array: label[x] <= x for kept x,
// and a root is its own label. Loads and stores go to the device-coherent
// level so that concurrent hooks see each other; values only decrease, so a
// stale read still names an ancestor.
__device__ __forceinline__ int cc_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cc_store(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x's tree, halving the path on the way (each step strictly
// decreases, so the walk ends within x steps).
__device__ __forceinline__ int cc_root(int32_t *label, int x) {
    int cur = cc_load(&label[x]);
    if (cur == x) return x;
    int prev = x;
    while (true) {
        const int next = cc_load(&label[cur]);
        if (next >= cur) return cur;  // a root (next == cur)
        cc_store(&label[prev], next);
        prev = cur;
        cur = next;
    }
}

__global__ void cc_init_kernel(const int64_t *__restrict__ he_ptr, int64_t m, int32_t s, int32_t *__restrict__ label) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) label[i] = (he_ptr[i + 1] - he_ptr[i] >= s) ? (int32_t)i : -1;
}

constexpr int kHookTries = 1 << 20;  // far above any real retry count

__global__ void cc_hook_kernel(const int32_t *__restrict__ row, const int32_t *__restrict__ col, int64_t num_edges,
                               int64_t m, int32_t *label, int *err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < num_edges; e += stride) {
        const int u = row[e], v = col[e];
        if (u < 0 || u >= m || v < 0 || v >= m) {  // not a hyperedge id
            atomicOr(err, 4);
            continue;
        }
        if (cc_load(&label[u]) < 0 || cc_load(&label[v]) < 0) {  // an end outside E_s: not an edge of L_s
            atomicOr(err, 2);
            continue;
        }
        int ru = cc_root(label, u), rv = cc_root(label, v);
        int tries = 0;
        while (ru != rv) {
            const int lo = min(ru, rv), hi = max(ru, rv);
            const int old = atomicCAS(&label[hi], hi, lo);  // hang the larger root under the smaller
            if (old == hi) break;
            // hi stopped being a root meanwhile: start again from the current roots
            ru = cc_root(label, lo);
            rv = cc_root(label, old);
            if (++tries >= kHookTries) {
                atomicOr(err, 1);
                break;
            }
        }
    }
}

// Roots into a separate array: the trees are read, never written, here (a
// path-halving walk racing with the final stores could leave a label at an
// ancestor that is not the root).
__global__ __launch_bounds__(256) void cc_finish_kernel(int64_t m, const int32_t *__restrict__ label,
                                                        int32_t *__restrict__ out, unsigned long long *count) {
    __shared__ unsigned long long blk;
    if (threadIdx.x == 0) blk = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int root = 0;
    if (i < m) {
        int cur = label[i];
        if (cur >= 0) {
            int next;
            while ((next = label[cur]) < cur) cur = next;
            root = cur == (int)i;
        }
        out[i] = cur;
    }
    const unsigned long long b = __ballot(root);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&blk, (unsigned long long)__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0 && blk) atomicAdd(count, blk);
}

__global__ void mark_ends_kernel(const int32_t *__restrict__ row, const int32_t *__restrict__ col, int64_t num_edges,
                                 int64_t m, int32_t *__restrict__ flag, int *err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < num_edges; e += stride) {
        const int u = row[e], v = col[e];
        if (u < 0 || u >= m || v < 0 || v >= m) {
            atomicOr(err, 4);
            continue;
        }
        flag[u] = 1;
        flag[v] = 1;
    }
}

__global__ void squeeze_ids_kernel(int64_t m, const int32_t *__restrict__ flag, const int64_t *__restrict__ pre,
                                   int32_t *__restrict__ new_id) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) new_id[i] = flag[i] ? (int32_t)pre[i] : -1;
}

__global__ void remap_edges_kernel(int32_t *__restrict__ row, int32_t *__restrict__ col, int64_t num_edges,
                                   const int32_t *__restrict__ new_id) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < num_edges; e += stride) {
        row[e] = new_id[row[e]];
        col[e] = new_id[col[e]];
    }
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : b);
}

inline unsigned stride_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

inline unsigned wave_grid(int64_t rows, int waves_per_block, int64_t cap) {
    int64_t b = (rows + waves_per_block - 1) / waves_per_block;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int64_t scan_partials_size(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// A large row of S > kWaveRow >= kSmallRow members has ceil(S / 256) <=
// (S + 255) / 256 <= S / 16 pieces (S >= 17): at most nnz / 16 in all when
// the rows do not overlap. The piece list holds, per piece, its entry, its 2-paths (int64)
// and its largest partner (int32): 3 * cap int64 in all.
static_assert(kPlanPiece == 256 && kWaveRow >= kSmallRow && kSmallRow >= 16 && kWaveRow <= 64, "piece bound");
int64_t plan_pieces_cap(int64_t nnz) { return nnz / 16 + 1; }

int heavy_resident(int device) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 0;
    // the grid is shared by every variant: take the least resident one
    const void *variants[5] = {reinterpret_cast<const void *>(heavy_kernel<false, false, false>),
                               reinterpret_cast<const void *>(heavy_kernel<false, true, false>),
                               reinterpret_cast<const void *>(heavy_kernel<true, false, false>),
                               reinterpret_cast<const void *>(heavy_kernel<true, true, false>),
                               reinterpret_cast<const void *>(heavy_kernel<false, false, true>)};
    for (const void *f : variants) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, f, kHeavyThreads, 0) != hipSuccess) v = 0;
        per = (per == 0 || (v > 0 && v < per)) ? v : per;
    }
    if (cus <= 0) cus = 256;
    if (per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t value, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    fill_i64_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, n, value);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    fill_i32_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, n, value);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *partials,
                                     hipStream_t st) {
    return exclusive_scan(in, n, out, partials, st);
}
hipError_t launch_exclusive_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *partials,
                                     hipStream_t st) {
    return exclusive_scan(in, n, out, partials, st);
}
hipError_t launch_exclusive_scan_u8(const uint8_t *in, int64_t n, int64_t *out, int64_t *partials,
                                    hipStream_t st) {
    return exclusive_scan(in, n, out, partials, st);
}

hipError_t launch_keep_incidence(int64_t nnz, const int32_t *v_idx, const int64_t *he_ptr, int64_t m,
                                 int32_t s_min, const int32_t *row_s, uint8_t *flag, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    keep_incidence_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(nnz, v_idx, he_ptr, m, s_min, row_s, flag);
    return hipGetLastError();
}

hipError_t launch_compact_vertex_lists(int64_t n, int64_t nnz, const int64_t *v_ptr,
                                       const int32_t *v_idx, const uint8_t *flag,
                                       const int64_t *pos, int64_t *vs_ptr, int32_t *vs_idx,
                                       hipStream_t st) {
    if (nnz > 0) compact_idx_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(nnz, v_idx, flag, pos, vs_idx);
    compact_ptr_kernel<<<grid_for(n + 1, 256), 256, 0, st>>>(n, nnz, v_ptr, pos, vs_ptr);
    return hipGetLastError();
}

hipError_t launch_row_keep(int64_t m, const int64_t *he_ptr, int32_t s_min, const int32_t *row_s, uint8_t *flag,
                           hipStream_t st) {
    if (m <= 0) return hipSuccess;
    row_keep_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, he_ptr, s_min, row_s, flag);
    return hipGetLastError();
}

hipError_t launch_cid(int64_t m, const uint8_t *flag, const int64_t *pre, int32_t *cid, int32_t *cid_row,
                      hipStream_t st) {
    if (m <= 0) return hipSuccess;
    cid_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, flag, pre, cid, cid_row);
    return hipGetLastError();
}

hipError_t launch_vs_cid(int64_t n, int64_t m, int64_t nnz, const int64_t *vs_ptr, const int32_t *vs_idx,
                         const int32_t *cid, int32_t *vs_cid, uint16_t *vs_win, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    vs_cid_kernel<<<stride_grid(nnz), 256, 0, st>>>(n, m, nnz, vs_ptr, vs_idx, cid, vs_cid, vs_win);
    return hipGetLastError();
}

hipError_t launch_row_plan(const Pruned &g, int32_t s_min, int32_t light_max, int64_t slot_work, int64_t row_lo,
                           int64_t row_hi, int32_t dense_ratio, int32_t dense_min, int32_t *tail_beg, int64_t *work,
                           int32_t *jmax, int32_t *nslots, uint8_t *rclass, int64_t *bsize,
                           unsigned long long *class_count, int *err, unsigned long long *heavy_work,
                           unsigned long long *dense_work, int64_t *pieces, unsigned long long *num_pieces,
                           hipStream_t st) {
    if (g.m <= 0) return hipSuccess;
    if (light_max <= 0 || light_max > kLightMax) light_max = kLightMax;
    if (slot_work <= 0) slot_work = kSlotWork;
    if (!g.cid) dense_ratio = 0;
    const RowPlanOut o{tail_beg, work, jmax, nslots, rclass, bsize, dense_ratio, dense_min, dense_work};
    row_plan_kernel<<<wave_grid((g.m + 63) / 64, 4, 8192), 256, 0, st>>>(g, s_min, light_max, slot_work, row_lo,
                                                                          row_hi, o,
                                                                          class_count, err, heavy_work, pieces,
                                                                          plan_pieces_cap(g.nnz), num_pieces);
    // the piece count is known on the device only: grids for the bound
    const int64_t cap = plan_pieces_cap(g.nnz);
    int64_t *piece_w = pieces + cap;
    int32_t *piece_jm = reinterpret_cast<int32_t *>(pieces + 2 * cap);
    row_piece_kernel<<<wave_grid(cap, 4, 4096), 256, 0, st>>>(g, tail_beg, pieces, cap, num_pieces, piece_w,
                                                              piece_jm, err);
    row_piece_finish_kernel<<<grid_for(cap, 256), 256, 0, st>>>(g, light_max, slot_work, o, class_count, err,
                                                                heavy_work, pieces, cap, num_pieces, piece_w,
                                                                piece_jm);
    return hipGetLastError();
}

hipError_t launch_fill_slots(int64_t m, const int64_t *he_ptr, const int64_t *slot_base,
                             const int32_t *nslots, const int32_t *jmax, const uint8_t *rclass,
                             const int64_t *bbase, const int32_t *cid, int64_t *hat, int32_t *hcnt,
                             int64_t *partials, int32_t *slot_row, int32_t *const *lists, HeavyDesc *const *heavy,
                             const int64_t *caps, unsigned long long *list_fill, int *err, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    LightLists ll;
    for (int c = 0; c < kLightClasses; ++c) ll.l[c] = lists[c];
    for (int c = 0; c < kNumLists; ++c) ll.cap[c] = caps[c];
    ll.err = err;
    fill_slots_kernel<<<grid_for(m, 256 * kFillRows), 256, 0, st>>>(m, he_ptr, slot_base, nslots, jmax, rclass,
                                                                     bbase, slot_row, ll, hat, list_fill);
    heavy_counts_kernel<<<grid_for(m, 256) < 8192 ? grid_for(m, 256) : 8192, 256, 0, st>>>(m, rclass, nslots, hcnt);
    hipError_t e;
    for (int h = 0; h < kNumHeavyLists; ++h)
        if ((e = exclusive_scan(hcnt + (int64_t)h * m, m, hat + (int64_t)h * (m + 1), partials, st)) != hipSuccess)
            return e;
    HeavyLists hl;
    for (int h = 0; h < kNumHeavyLists; ++h) {
        hl.l[h] = heavy[h];
        hl.cap[h] = caps[kLightClasses + h];
    }
    heavy_desc_kernel<<<wave_grid(m, 4, 8192), 256, 0, st>>>(m, he_ptr, slot_base, nslots, jmax, rclass,
                                                              bbase, hat, slot_row, hl, cid, err);
    return hipGetLastError();
}

hipError_t launch_block_mask(int64_t m, int64_t r0, int64_t r1, const int32_t *nslots_all, const uint8_t *rclass_all,
                             const int64_t *bsize_all, const int64_t *work, int32_t *nslots, uint8_t *rclass,
                             int64_t *bsize, unsigned long long *class_count, unsigned long long *heavy_work,
                             unsigned long long *dense_work, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const unsigned grid = grid_for(m, 256) < 4096 ? grid_for(m, 256) : 4096;
    block_mask_kernel<<<grid, 256, 0, st>>>(m, r0, r1, nslots_all, rclass_all, bsize_all, work, nslots, rclass, bsize,
                                            class_count, heavy_work, dense_work);
    return hipGetLastError();
}

hipError_t launch_list_cuts(const HeavyDesc *desc, int64_t count, const int64_t *slots, int64_t n, int64_t *out,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    list_cuts_kernel<<<grid_for(n, 256), 256, 0, st>>>(desc, count, slots, n, out);
    return hipGetLastError();
}

hipError_t launch_heavy_range(const HeavyDesc *desc, int64_t count, int64_t s0, int64_t s1, int64_t *out,
                              hipStream_t st) {
    heavy_range_kernel<<<1, 64, 0, st>>>(desc, count, s0, s1, out);
    return hipGetLastError();
}

hipError_t launch_light(int cls, bool emit, const int32_t *list, int64_t count, const Slots &sl,
                        const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, const LightStore *store, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (store && emit) return hipErrorInvalidValue;
    if (cls == 0) {  // one lane per row
        if (emit)
            tiny_kernel<true><<<grid_for(count, 256), 256, 0, st>>>(list, count, sl, g, ep, slot_cnt, slot_off);
        else
            tiny_kernel<false><<<grid_for(count, 256), 256, 0, st>>>(list, count, sl, g, ep, slot_cnt, slot_off);
        return hipGetLastError();
    }
    const unsigned grid = grid_for(count, 4);
    const LightStore ls = store ? *store : LightStore{};
#define SLG_LIGHT(KPL)                                                                              \
    do {                                                                                           \
        if (emit)                                                                                  \
            light_kernel<KPL, true, false><<<grid, 256, 0, st>>>(list, count, sl, g, ep, slot_cnt,  \
                                                                 slot_off, ls);                    \
        else if (store)                                                                            \
            light_kernel<KPL, false, true><<<grid, 256, 0, st>>>(list, count, sl, g, ep, slot_cnt,  \
                                                                 slot_off, ls);                    \
        else                                                                                       \
            light_kernel<KPL, false, false><<<grid, 256, 0, st>>>(list, count, sl, g, ep, slot_cnt, \
                                                                  slot_off, ls);                   \
    } while (0)
    switch (cls) {
        case 1: SLG_LIGHT(1); break;
        case 2: SLG_LIGHT(2); break;
        case 3: SLG_LIGHT(4); break;
        case 4: SLG_LIGHT(8); break;
        case 5: SLG_LIGHT(16); break;
        case 6: SLG_LIGHT(32); break;
        default: return hipErrorInvalidValue;
    }
#undef SLG_LIGHT
    return hipGetLastError();
}

hipError_t launch_light_store_emit(const int32_t *list, int64_t count, const Slots &sl, const LightStore &store,
                                   const EmitParams &ep, const int64_t *slot_off, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    light_store_emit_kernel<<<grid_for(count, 4), 256, 0, st>>>(list, count, sl, store, ep, slot_off);
    return hipGetLastError();
}

hipError_t launch_light_work(int64_t m, const uint8_t *rclass, const int64_t *work, int32_t *lw, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    light_work_kernel<<<grid_for(m, 256) < 8192 ? grid_for(m, 256) : 8192, 256, 0, st>>>(m, rclass, work, lw);
    return hipGetLastError();
}

hipError_t launch_heavy(bool emit, bool wide, const HeavyDesc *desc, int64_t count, int64_t slots,
                        const int32_t *bounds, const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, int64_t *ticket, int resident, const CountStore *store,
                        hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (store && (emit || wide)) return hipErrorInvalidValue;
    const int64_t want = resident > 0 ? resident : 512;
    const unsigned grid = (unsigned)(count < want ? count : want);
    unsigned long long *tk = reinterpret_cast<unsigned long long *>(ticket);
    const CountStore cs = store ? *store : CountStore{};
#define SLG_HEAVY(E, W, ST)                                                                          \
    heavy_kernel<E, W, ST><<<grid, kHeavyThreads, 0, st>>>(desc, count, slots, bounds, g.vs_idx, ep, slot_cnt, \
                                                           slot_off, tk, cs)
    if (emit && wide) SLG_HEAVY(true, true, false);
    else if (emit) SLG_HEAVY(true, false, false);
    else if (wide) SLG_HEAVY(false, true, false);
    else if (store) SLG_HEAVY(false, false, true);
    else SLG_HEAVY(false, false, false);
#undef SLG_HEAVY
    return hipGetLastError();
}

hipError_t launch_slot_work(const HeavyDesc *desc, int64_t count, const int32_t *bounds, int64_t *work,
                            hipStream_t st) {
    if (count <= 0) return hipSuccess;
    slot_work_kernel<<<wave_grid(count, 4, 8192), 256, 0, st>>>(desc, count, bounds, work);
    return hipGetLastError();
}

hipError_t launch_heavy_store_emit(const HeavyDesc *desc, int64_t count, int64_t slots, const CountStore &store,
                                   const EmitParams &ep, const int64_t *slot_off, const int32_t *cid_row,
                                   hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned grid = wave_grid(count, 4, 16384);
    if (cid_row) {
        if (ep.k <= 4)
            heavy_store_emit_kernel<4, true><<<grid, 256, 0, st>>>(desc, count, slots, store, ep, slot_off, cid_row);
        else
            heavy_store_emit_kernel<SLG_MAX_S, true><<<grid, 256, 0, st>>>(desc, count, slots, store, ep, slot_off,
                                                                           cid_row);
    } else if (ep.k <= 4) {
        heavy_store_emit_kernel<4, false><<<grid, 256, 0, st>>>(desc, count, slots, store, ep, slot_off, nullptr);
    } else {
        heavy_store_emit_kernel<SLG_MAX_S, false><<<grid, 256, 0, st>>>(desc, count, slots, store, ep, slot_off,
                                                                        nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_dense_keys(const HeavyDesc *desc, int64_t count, int32_t *key, int32_t *id, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    dense_keys_kernel<<<grid_for(count, 256), 256, 0, st>>>(desc, count, key, id);
    return hipGetLastError();
}

hipError_t launch_dense(bool emit, const HeavyDesc *desc, int64_t count, const int32_t *order, int64_t slots,
                        const int32_t *bounds, const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, int64_t *ticket, int resident, const CountStore *store,
                        int64_t *store_cursor, int64_t store_cap, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (!g.vs_win || !g.cid_row || (store && !emit && !store_cursor)) return hipErrorInvalidValue;
    const int64_t want = resident > 0 ? resident : 512;
    const unsigned grid = (unsigned)(count < want ? count : want);
    unsigned long long *tk = reinterpret_cast<unsigned long long *>(ticket);
    unsigned long long *cur = reinterpret_cast<unsigned long long *>(store_cursor);
    const CountStore cs = store ? *store : CountStore{};
    if (emit)
        dense_kernel<true><<<grid, kDenseThreads, 0, st>>>(desc, count, order, slots, bounds, g.vs_win, g.cid_row, ep,
                                                            slot_cnt, slot_off, tk, cs, cur, store_cap);
    else
        dense_kernel<false><<<grid, kDenseThreads, 0, st>>>(desc, count, order, slots, bounds, g.vs_win, g.cid_row, ep,
                                                             slot_cnt, slot_off, tk, cs, cur, store_cap);
    return hipGetLastError();
}

int dense_resident(int device) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 0;
    const void *variants[2] = {reinterpret_cast<const void *>(dense_kernel<false>),
                               reinterpret_cast<const void *>(dense_kernel<true>)};
    for (const void *f : variants) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, f, kDenseThreads, 0) != hipSuccess) v = 0;
        per = (per == 0 || (v > 0 && v < per)) ? v : per;
    }
    if (cus <= 0) cus = 256;
    if (per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_sum_i32(const int32_t *n, int64_t count, int64_t *out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    sum_i32_kernel<<<grid_for(count, 256) < 4096 ? grid_for(count, 256) : 4096, 256, 0, st>>>(
        n, count, reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t launch_heavy_edges(const HeavyDesc *desc, int64_t count, const int64_t *slot_cnt, int64_t S,
                              int32_t K, int64_t *out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    heavy_edges_kernel<<<grid_for(count, 256), 256, 0, st>>>(desc, count, slot_cnt, S, K,
                                                              reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t launch_bounds(const Pruned &g, const HeavyDesc *desc, int64_t count, int32_t *bounds,
                         hipStream_t st) {
    if (count <= 0) return hipSuccess;
    bounds_kernel<<<grid_for(count, 4), 256, 0, st>>>(desc, count, g.he_ptr, g.he_idx, g.vs_ptr, g.vs_idx,
                                                       g.tail_beg, bounds);
    return hipGetLastError();
}

hipError_t launch_row_ptr(int64_t row_lo, int64_t row_hi, const int64_t *slot_base,
                          const int64_t *slot_off, int64_t slots, const EmitParams &ep, hipStream_t st) {
    const int64_t n = row_hi - row_lo + 1;
    if (n <= 0) return hipSuccess;
    row_ptr_kernel<<<grid_for(n, 256), 256, 0, st>>>(row_lo, row_hi, slot_base, slot_off, slots, ep);
    return hipGetLastError();
}

hipError_t launch_row_bytes(int64_t m, const int64_t *slot_base, const int64_t *slot_off, int64_t slots,
                            int32_t K, int64_t *out, hipStream_t st) {
    row_bytes_kernel<<<grid_for(m + 1, 256), 256, 0, st>>>(m, slot_base, slot_off, slots, K, out);
    return hipGetLastError();
}

hipError_t launch_gather_offsets(const int64_t *rows, int64_t count, const int64_t *slot_base,
                                 const int64_t *slot_off, int64_t slots, int32_t K, int64_t *out,
                                 hipStream_t st) {
    if (count <= 0) return hipSuccess;
    gather_offsets_kernel<<<grid_for(count, 256), 256, 0, st>>>(rows, count, slot_base, slot_off, slots, K,
                                                                 out);
    return hipGetLastError();
}

hipError_t launch_union(const UnionPart *parts, int32_t count, int64_t max_elems, int64_t *he_ptr,
                        int32_t *he_idx, int64_t *v_ptr, int32_t *v_idx, int32_t *row_s, int32_t *row_base,
                        hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t bx = (max_elems + 255) / 256;
    if (bx > 256) bx = 256;
    if (bx < 1) bx = 1;
    union_kernel<<<dim3((unsigned)bx, (unsigned)count), 256, 0, st>>>(parts, he_ptr, he_idx, v_ptr, v_idx, row_s,
                                                                       row_base);
    return hipGetLastError();
}


hipError_t launch_cc_init(const int64_t *he_ptr, int64_t m, int32_t s, int32_t *label, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    cc_init_kernel<<<grid_for(m, 256), 256, 0, st>>>(he_ptr, m, s, label);
    return hipGetLastError();
}

hipError_t launch_cc_hook(const int32_t *row, const int32_t *col, int64_t num_edges, int64_t m, int32_t *label,
                          int *err, hipStream_t st) {
    if (num_edges <= 0) return hipSuccess;
    cc_hook_kernel<<<stride_grid(num_edges), 256, 0, st>>>(row, col, num_edges, m, label, err);
    return hipGetLastError();
}

hipError_t launch_cc_finish(int64_t m, const int32_t *label, int32_t *out, unsigned long long *count,
                            hipStream_t st) {
    if (m <= 0) return hipSuccess;
    cc_finish_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, label, out, count);
    return hipGetLastError();
}

hipError_t launch_mark_ends(const int32_t *row, const int32_t *col, int64_t num_edges, int64_t m, int32_t *flag,
                            int *err, hipStream_t st) {
    if (num_edges <= 0) return hipSuccess;
    mark_ends_kernel<<<stride_grid(num_edges), 256, 0, st>>>(row, col, num_edges, m, flag, err);
    return hipGetLastError();
}

hipError_t launch_squeeze_ids(int64_t m, const int32_t *flag, const int64_t *pre, int32_t *new_id, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    squeeze_ids_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, flag, pre, new_id);
    return hipGetLastError();
}

hipError_t launch_remap_edges(int32_t *row, int32_t *col, int64_t num_edges, const int32_t *new_id,
                              hipStream_t st) {
    if (num_edges <= 0) return hipSuccess;
    remap_edges_kernel<<<stride_grid(num_edges), 256, 0, st>>>(row, col, num_edges, new_id);
    return hipGetLastError();
}

hipError_t launch_gather_i64(const int64_t *src, const int64_t *idx, int64_t count, int64_t *out,
                             hipStream_t st) {
    if (count <= 0) return hipSuccess;
    gather_i64_kernel<<<grid_for(count, 256), 256, 0, st>>>(src, idx, count, out);
    return hipGetLastError();
}

hipError_t launch_validate_ptr(const int64_t *ptr, int64_t rows, int64_t nnz, int *err,
                               hipStream_t st) {
    validate_ptr_kernel<<<grid_for(rows + 1, 256), 256, 0, st>>>(ptr, rows, nnz, err);
    return hipGetLastError();
}

hipError_t launch_validate_rows(const int64_t *ptr, const int32_t *idx, int64_t rows,
                                int64_t limit, int *err, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    validate_rows_kernel<<<wave_grid(rows, 4, 8192), 256, 0, st>>>(ptr, idx, rows, limit, err);
    return hipGetLastError();
}

hipError_t launch_validate_transpose(const int64_t *he_ptr, const int32_t *he_idx, int64_t m,
                                     const int64_t *v_ptr, const int32_t *v_idx, int64_t n, int *err,
                                     hipStream_t st) {
    if (m <= 0) return hipSuccess;
    validate_transpose_kernel<<<wave_grid(m, 4, 8192), 256, 0, st>>>(he_ptr, he_idx, m, v_ptr, v_idx,
                                                                      n, err);
    return hipGetLastError();
}

}  // namespace slg
