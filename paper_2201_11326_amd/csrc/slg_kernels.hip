// gfx950 kernels for s-line graph construction.
//
// The path (Section III-B/C, Algorithms 2 and 3):
//   K1  prune: drop hyperedges with |e| < s_min from every vertex list
//       (degree-based pruning on both sides of a pair; a pair that meets
//       the threshold has both sizes >= s, so no edge is lost).
//   K2  plan: per kept hyperedge e_i and member v, the tail of v's list after
//       i (the partners e_j, j > i, reached through v: the upper triangle),
//       the 2-path work w_i = sum of tail lengths, and a slot table that
//       splits heavy rows by hyperedge-id range.
//   K3  count overlaps |e_i n e_j| by walking every 2-path (e_i, v, e_j):
//         light rows (w_i <= 512): one wavefront gathers the 2-path
//           partners into LDS, sorts them in registers (bitonic) and
//           run-length counts them;
//         heavy slots: one workgroup marks partners in an LDS bitmap over
//           the slot's id range, ranks them by prefix popcount, and counts
//           each partner in an LDS counter indexed by its rank; heavy
//           vertex tails are cut into equal pieces across the wavefronts.
//   K4/5 threshold-and-emit for every s_k of the ensemble from the same
//       counters (the stored overlap is the largest s for which the pair
//       survives), compacted with wavefront ballots + prefix sums. The rank
//       order is the hyperedge-id order, so rows come out sorted.
//   K6  assembly: prefix sums of per-slot counts give each slot's output
//       offset and the CSR row pointers.
// Every step is exact integer work; no floating point is involved.
#include <limits.h>

#include "slg_internal.h"

namespace slg {
namespace {

// ---------------------------------------------------------------------------
// wavefront / workgroup primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

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
                                      uint8_t *__restrict__ flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    int32_t e = v_idx[p];
    uint8_t keep = 0;
    if (e >= 0 && e < m) keep = (he_ptr[e + 1] - he_ptr[e]) >= s_min;
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

// ---------------------------------------------------------------------------
// K2: per-row plan (one wavefront per hyperedge, grid-stride)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int light_class(int64_t w) {
    return w <= 64 ? 0 : (w <= 128 ? 1 : (w <= 256 ? 2 : 3));
}

__global__ __launch_bounds__(256) void row_plan_kernel(Pruned g, int32_t s_min,
                                                       int32_t *__restrict__ tail_beg,
                                                       int64_t *__restrict__ work,
                                                       int32_t *__restrict__ jmax_out,
                                                       int32_t *__restrict__ nslots,
                                                       uint8_t *__restrict__ rclass,
                                                       unsigned long long *__restrict__ class_count,
                                                       int *__restrict__ err) {
    __shared__ unsigned long long ccount[kNumLists];
    if (threadIdx.x < kNumLists) ccount[threadIdx.x] = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; i < g.m; i += nwaves) {
        const int64_t p0 = g.he_ptr[i], p1 = g.he_ptr[i + 1];
        int64_t w = 0;
        int jm = -1;
        int bad = 0;
        if (p0 < 0 || p1 > g.nnz || p1 < p0) {
            bad = 1;
        } else if (p1 - p0 >= s_min && p1 > p0) {
            for (int64_t p = p0 + lane; p < p1; p += 64) {
                const int v = g.he_idx[p];
                if (v < 0 || v >= g.n) {
                    bad = 1;
                    tail_beg[p] = 0;
                    continue;
                }
                const int64_t lo = g.vs_ptr[v], hi = g.vs_ptr[v + 1];
                if (lo < 0 || hi < lo || hi > g.nnz) {
                    bad = 1;
                    tail_beg[p] = 0;
                    continue;
                }
                int a = lower_bound_i32(g.vs_idx, (int)lo, (int)hi, (int)i);
                const bool found = a < hi && g.vs_idx[a] == (int)i;
                bad |= !found;  // the vertex CSR must be the transpose
                const int beg = found ? a + 1 : a;
                tail_beg[p] = beg;
                w += hi - beg;
                if (beg < hi) jm = max(jm, g.vs_idx[hi - 1]);
            }
        }
        w = wave_sum(w);
        jm = wave_max(jm);
        bad = wave_max(bad);
        if (lane == 0) {
            int cls = kNone;
            int64_t ns = 0;
            if (bad) {
                atomicOr(err, 1);
            } else if (w > 0) {
                if (w <= kLightMax) {
                    cls = kLight0 + light_class(w);
                    ns = 1;
                } else {
                    cls = kHeavy;
                    const int64_t range = (int64_t)jm - i;  // partners lie in [i+1, jm]
                    const int64_t by_range = (range + kRangeBits - 1) / kRangeBits;
                    const int64_t by_work = (w + kSlotWork - 1) / kSlotWork;
                    ns = by_range > by_work ? by_range : by_work;
                    if (ns > range) ns = range;
                }
            }
            work[i] = w;
            jmax_out[i] = jm;
            nslots[i] = (int32_t)ns;
            rclass[i] = (uint8_t)cls;
            if (cls != kNone) atomicAdd(&ccount[cls - 1], (unsigned long long)ns);
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumLists && ccount[threadIdx.x])
        atomicAdd(&class_count[threadIdx.x], ccount[threadIdx.x]);
}

// One thread per row: write the row's slots and append them to the tier lists.
__global__ __launch_bounds__(256) void fill_slots_kernel(
    int64_t m, const int64_t *__restrict__ slot_base, const int32_t *__restrict__ nslots,
    const int32_t *__restrict__ jmax, const uint8_t *__restrict__ rclass,
    int32_t *__restrict__ slot_row, int32_t *__restrict__ slot_ja, int32_t *__restrict__ slot_jb,
    int32_t *l0, int32_t *l1, int32_t *l2, int32_t *l3, int32_t *lh,
    unsigned long long *__restrict__ list_fill) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    int cls = kNone;
    int ns = 0;
    int64_t base = 0;
    int jm = 0;
    if (i < m) {
        cls = rclass[i];
        ns = nslots[i];
        base = slot_base[i];
        jm = jmax[i];
    }
    // light classes: wavefront-aggregated append, one slot per row
    int32_t *lists[kLightClasses] = {l0, l1, l2, l3};
#pragma unroll
    for (int c = 0; c < kLightClasses; ++c) {
        const bool mine = (cls == kLight0 + c);
        const unsigned long long mask = __ballot(mine);
        if (!mask) continue;
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long at = 0;
        if (lane == leader) at = atomicAdd(&list_fill[c], (unsigned long long)__popcll(mask));
        at = __shfl(at, leader);
        if (mine) {
            lists[c][at + bits_below(mask)] = (int32_t)base;
            slot_row[base] = (int32_t)i;
            slot_ja[base] = (int32_t)i + 1;
            slot_jb[base] = jm + 1;
        }
    }
    if (cls == kHeavy && ns > 0) {
        const unsigned long long at = atomicAdd(&list_fill[kLightClasses], (unsigned long long)ns);
        const int64_t range = (int64_t)jm - i;
        for (int t = 0; t < ns; ++t) {
            const int64_t s = base + t;
            slot_row[s] = (int32_t)i;
            slot_ja[s] = (int32_t)(i + 1 + range * t / ns);
            slot_jb[s] = (int32_t)(i + 1 + range * (t + 1) / ns);
            lh[at + t] = (int32_t)s;
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

template <int KPL, bool EMIT>
__global__ __launch_bounds__(256) void light_kernel(const int32_t *__restrict__ list, int64_t count,
                                                    Slots sl, Pruned g, EmitParams prm,
                                                    int64_t *__restrict__ slot_cnt,
                                                    const int64_t *__restrict__ slot_off,
                                                    int64_t out_base) {
    constexpr int P = 64 * KPL;
    __shared__ int32_t buf[4][P];
    __shared__ EmitParams sp;  // thresholds and outputs, indexed by a uniform k
    if (threadIdx.x == 0) sp = prm;
    __syncthreads();
    const EmitParams *ep = &sp;
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * 4 + wv;
    if (wid >= count) return;
    int32_t *kb = buf[wv];
    const int slot = list[wid];
    const int i = sl.row[slot];
    const int64_t p0 = g.he_ptr[i], p1 = g.he_ptr[i + 1];

    // gather the partners e_j of every 2-path (e_i, v, e_j), j > i
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
        const int excl = incl - len;
        const int tot = __shfl(incl, 63);
        for (int t = 0; t < len; ++t) {
            const int e = w + excl + t;
            if (e < P) kb[e] = g.vs_idx[beg + t];
        }
        w += tot;
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

    const int K = ep->k;
    const int64_t S = sl.count;
    for (int k = 0; k < K; ++k) {
        const int sk = ep->s[k];
        int64_t base = EMIT ? slot_off[(int64_t)k * (S + 1) + slot] - out_base : 0;
        int32_t *col = EMIT ? ep->col[k] : nullptr;
        int32_t *wo = EMIT ? ep->w[k] : nullptr;
        int32_t *ro = EMIT ? ep->row[k] : nullptr;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const bool surv = c[r] >= sk;  // sk >= 1, so only run heads
            const unsigned long long mask = __ballot(surv);
            if (EMIT && surv) {
                const int64_t pos = base + bits_below(mask);
                col[pos] = x[r];
                wo[pos] = c[r];
                if (ro) ro[pos] = i;
            }
            base += __popcll(mask);
        }
        if (!EMIT && lane == 0) slot_cnt[(int64_t)k * S + slot] = base;
    }
}

// ---------------------------------------------------------------------------
// K3-K5 heavy tier: one workgroup per slot, LDS bitmap + rank counters
// ---------------------------------------------------------------------------
constexpr int kHW = kHeavyThreads / 64;  // wavefronts per heavy workgroup

struct HeavySmem {
    uint32_t bitmap[kRangeWords];       // partner j present in the slot range
    uint32_t wpre[kRangeWords + 1];     // exclusive prefix popcount per word
    uint32_t cnt[kRankCap];             // overlap counter per rank in window
    int32_t keys[kRankCap];             // partner id per rank in window (emit)
    int32_t seg_a[kHeavyThreads];       // tail segment start per vertex batch
    int32_t seg_pre[kHeavyThreads + 1]; // flattened start per vertex batch
    int32_t wsum[kHW];
    int32_t wtot[SLG_MAX_S][kHW];
    unsigned long long acc[SLG_MAX_S];
    long long obase[SLG_MAX_S];
};

// Calls f(j) for every 2-path (e_i, v, e_j) with j in [ka, kb), over the
// incidences [p0, p1) of row i. Tails are clipped to the range by binary
// search; the flattened 2-path list of each batch of vertices is cut into
// equal pieces, one per wavefront, so a heavy vertex's tail is shared by all
// wavefronts of the workgroup. Ends with a workgroup barrier.
template <typename F>
__device__ __forceinline__ void for_each_2path(const Pruned &g, int64_t p0, int64_t p1, int ka,
                                               int kb, HeavySmem &sm, F &&f) {
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    for (int64_t vb = p0; vb < p1; vb += kHeavyThreads) {
        const int64_t p = vb + tid;
        int a = 0, len = 0;
        if (p < p1) {
            const int v = g.he_idx[p];
            int beg = g.tail_beg[p];
            int end = (int)g.vs_ptr[v + 1];
            if (beg < end) {
                if (g.vs_idx[beg] < ka) beg = lower_bound_i32(g.vs_idx, beg, end, ka);
                if (beg < end && g.vs_idx[end - 1] >= kb) end = lower_bound_i32(g.vs_idx, beg, end, kb);
                a = beg;
                len = end > beg ? end - beg : 0;
            }
        }
        int total;
        const int excl = block_excl_scan<kHeavyThreads>(len, sm.wsum, total);
        sm.seg_a[tid] = a;
        sm.seg_pre[tid] = excl;
        if (tid == 0) sm.seg_pre[kHeavyThreads] = total;
        __syncthreads();
        if (total > 0) {
            const int per = (total + kHW - 1) / kHW;
            const int c0 = wave * per;
            const int c1 = min(total, c0 + per);
            if (c0 < c1) {
                int lo = 0, hi = kHeavyThreads;  // seg_pre[lo] <= c0 < seg_pre[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (sm.seg_pre[mid] <= c0)
                        lo = mid;
                    else
                        hi = mid;
                }
                int u = lo, pos = c0;
                while (pos < c1) {
                    const int ue = min(c1, sm.seg_pre[u + 1]);
                    const int base = sm.seg_a[u] - sm.seg_pre[u];
                    for (int q = pos + lane; q < ue; q += 64) f(g.vs_idx[base + q]);
                    pos = ue;
                    ++u;
                }
            }
        }
        __syncthreads();
    }
}

template <bool EMIT>
__global__ __launch_bounds__(kHeavyThreads) void heavy_kernel(const int32_t *__restrict__ list,
                                                              int64_t count, Slots sl, Pruned g,
                                                              EmitParams prm,
                                                              int64_t *__restrict__ slot_cnt,
                                                              const int64_t *__restrict__ slot_off,
                                                              int64_t out_base) {
    __shared__ HeavySmem sm;
    __shared__ EmitParams sp;  // thresholds and outputs, indexed by a uniform k
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    if (tid == 0) sp = prm;
    __syncthreads();
    const EmitParams *ep = &sp;
    const int K = ep->k;
    const int64_t S = sl.count;
    const bool only_presence = !EMIT && K == 1 && ep->s[0] <= 1;

    for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
        const int slot = list[it];
        const int i = sl.row[slot], ja = sl.ja[slot], jb = sl.jb[slot];
        const int nw = (jb - ja + 31) >> 5;
        const int64_t p0 = g.he_ptr[i], p1 = g.he_ptr[i + 1];
        for (int x = tid; x < nw; x += kHeavyThreads) sm.bitmap[x] = 0u;
        if (tid < SLG_MAX_S) {
            sm.acc[tid] = 0;
            sm.obase[tid] = (EMIT && tid < K) ? slot_off[(int64_t)tid * (S + 1) + slot] - out_base : 0;
        }
        __syncthreads();

        // pass 1: mark every partner j of the slot's range
        const unsigned span = (unsigned)(jb - ja);
        for_each_2path(g, p0, p1, ja, jb, sm, [&](int j) {
            const unsigned off = (unsigned)(j - ja);
            if (off < span) atomicOr(&sm.bitmap[off >> 5], 1u << (off & 31));
        });

        // rank of a partner = number of marked partners below it
        constexpr int kWPT = kRangeWords / kHeavyThreads;
        int loc[kWPT];
        int mine = 0;
#pragma unroll
        for (int r = 0; r < kWPT; ++r) {
            const int x = tid * kWPT + r;
            loc[r] = x < nw ? __popc(sm.bitmap[x]) : 0;
            mine += loc[r];
        }
        int distinct;
        int run = block_excl_scan<kHeavyThreads>(mine, sm.wsum, distinct);
#pragma unroll
        for (int r = 0; r < kWPT; ++r) {
            const int x = tid * kWPT + r;
            if (x < nw) sm.wpre[x] = run;
            run += loc[r];
        }
        if (tid == 0) sm.wpre[nw] = distinct;
        __syncthreads();

        if (only_presence) {  // L_1 alone: every marked partner is an edge
            if (tid == 0) slot_cnt[slot] = distinct;
            __syncthreads();
            continue;
        }

        // windows of at most kRankCap ranks, cut at word boundaries
        int w0 = 0;
        while (w0 < nw) {
            const int r0 = sm.wpre[w0];
            int lo = w0 + 1, hi = nw;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int)sm.wpre[mid] - r0 <= kRankCap)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int w1 = lo;
            const int nr = (int)sm.wpre[w1] - r0;
            if (nr > 0) {
                const int ka = ja + 32 * w0;
                const int kb = min(jb, ja + 32 * w1);
                for (int x = tid; x < nr; x += kHeavyThreads) sm.cnt[x] = 0u;
                __syncthreads();
                // pass 2: count every 2-path into its partner's rank
                for_each_2path(g, p0, p1, ka, kb, sm, [&](int j) {
                    const unsigned off = (unsigned)(j - ja);
                    if (off >= span) return;
                    const int x = (int)(off >> 5);
                    const unsigned r = sm.wpre[x] + __popc(sm.bitmap[x] & ((1u << (off & 31)) - 1u)) - (unsigned)r0;
                    if (r < (unsigned)nr) atomicAdd(&sm.cnt[r], 1u);
                });
                if (EMIT) {
                    for (int x = w0 + tid; x < w1; x += kHeavyThreads) {
                        unsigned bits = sm.bitmap[x];
                        int r = (int)sm.wpre[x] - r0;
                        const int jbase = ja + 32 * x;
                        while (bits) {
                            sm.keys[r++] = jbase + __ffs(bits) - 1;
                            bits &= bits - 1u;
                        }
                    }
                    __syncthreads();
                }
                // threshold per s_k; ranks are in partner order
                for (int rb = 0; rb < nr; rb += kHeavyThreads) {
                    const int r = rb + tid;
                    const bool valid = r < nr;
                    const int c = valid ? (int)sm.cnt[r] : 0;
                    if (!EMIT) {
                        for (int k = 0; k < K; ++k) {
                            const unsigned long long mask = __ballot(c >= ep->s[k]);
                            if (lane == 0 && mask) atomicAdd(&sm.acc[k], (unsigned long long)__popcll(mask));
                        }
                    } else {
                        const int key = valid ? sm.keys[r] : 0;
                        for (int k = 0; k < K; ++k) {
                            const unsigned long long mask = __ballot(c >= ep->s[k]);
                            if (lane == 0) sm.wtot[k][wave] = __popcll(mask);
                        }
                        __syncthreads();
                        for (int k = 0; k < K; ++k) {
                            const bool surv = c >= ep->s[k];
                            const unsigned long long mask = __ballot(surv);
                            int pre = 0;
                            for (int w = 0; w < wave; ++w) pre += sm.wtot[k][w];
                            if (surv) {
                                const int64_t pos = sm.obase[k] + pre + bits_below(mask);
                                ep->col[k][pos] = key;
                                ep->w[k][pos] = c;
                                int32_t *ro = ep->row[k];
                                if (ro) ro[pos] = i;
                            }
                        }
                        __syncthreads();
                        if (tid < K) {
                            int tot = 0;
                            for (int w = 0; w < kHW; ++w) tot += sm.wtot[tid][w];
                            sm.obase[tid] += tot;
                        }
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
            w0 = w1;
        }
        __syncthreads();
        if (!EMIT && tid < K) slot_cnt[(int64_t)tid * S + slot] = (int64_t)sm.acc[tid];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K6: CSR row pointers from slot offsets
// ---------------------------------------------------------------------------
__global__ void row_ptr_kernel(int64_t row_lo, int64_t row_hi, const int64_t *__restrict__ slot_base,
                               const int64_t *__restrict__ slot_off, int64_t S, EmitParams prm,
                               int64_t out_base) {
    __shared__ EmitParams sp;
    if (threadIdx.x == 0) sp = prm;
    __syncthreads();
    const int64_t i = row_lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > row_hi) return;
    const int64_t sb = slot_base[i];
    for (int k = 0; k < sp.k; ++k) sp.row_ptr[k][i - row_lo] = slot_off[(int64_t)k * (S + 1) + sb] - out_base;
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

inline unsigned grid_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
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

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t value, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    fill_i64_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, n, value);
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
                                 int32_t s_min, uint8_t *flag, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    keep_incidence_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(nnz, v_idx, he_ptr, m, s_min, flag);
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

hipError_t launch_row_plan(const Pruned &g, int32_t s_min, int32_t *tail_beg, int64_t *work,
                           int32_t *jmax, int32_t *nslots, uint8_t *rclass,
                           unsigned long long *class_count, int *err, hipStream_t st) {
    if (g.m <= 0) return hipSuccess;
    row_plan_kernel<<<wave_grid(g.m, 4, 8192), 256, 0, st>>>(g, s_min, tail_beg, work, jmax, nslots,
                                                              rclass, class_count, err);
    return hipGetLastError();
}

hipError_t launch_fill_slots(int64_t m, const int64_t *slot_base, const int32_t *nslots,
                             const int32_t *jmax, const int64_t *work, const uint8_t *rclass,
                             int32_t *slot_row, int32_t *slot_ja, int32_t *slot_jb,
                             int32_t *const *lists, unsigned long long *list_fill,
                             hipStream_t st) {
    (void)work;
    if (m <= 0) return hipSuccess;
    fill_slots_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, slot_base, nslots, jmax, rclass, slot_row,
                                                         slot_ja, slot_jb, lists[0], lists[1],
                                                         lists[2], lists[3], lists[4], list_fill);
    return hipGetLastError();
}

hipError_t launch_light(int cls, bool emit, const int32_t *list, int64_t count, const Slots &sl,
                        const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, int64_t out_base, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned grid = grid_for(count, 4);
#define SLG_LIGHT(KPL)                                                                              \
    do {                                                                                           \
        if (emit)                                                                                  \
            light_kernel<KPL, true><<<grid, 256, 0, st>>>(list, count, sl, g, ep, slot_cnt,        \
                                                          slot_off, out_base);                     \
        else                                                                                       \
            light_kernel<KPL, false><<<grid, 256, 0, st>>>(list, count, sl, g, ep, slot_cnt,       \
                                                           slot_off, out_base);                    \
    } while (0)
    switch (cls) {
        case 0: SLG_LIGHT(1); break;
        case 1: SLG_LIGHT(2); break;
        case 2: SLG_LIGHT(4); break;
        case 3: SLG_LIGHT(8); break;
        default: return hipErrorInvalidValue;
    }
#undef SLG_LIGHT
    return hipGetLastError();
}

hipError_t launch_heavy(bool emit, const int32_t *list, int64_t count, const Slots &sl,
                        const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, int64_t out_base, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    if (emit)
        heavy_kernel<true><<<grid, kHeavyThreads, 0, st>>>(list, count, sl, g, ep, slot_cnt, slot_off,
                                                           out_base);
    else
        heavy_kernel<false><<<grid, kHeavyThreads, 0, st>>>(list, count, sl, g, ep, slot_cnt, slot_off,
                                                            out_base);
    return hipGetLastError();
}

hipError_t launch_row_ptr(int64_t row_lo, int64_t row_hi, const int64_t *slot_base,
                          const int64_t *slot_off, int64_t slots, const EmitParams &ep,
                          int64_t out_base, hipStream_t st) {
    const int64_t n = row_hi - row_lo + 1;
    if (n <= 0) return hipSuccess;
    row_ptr_kernel<<<grid_for(n, 256), 256, 0, st>>>(row_lo, row_hi, slot_base, slot_off, slots, ep,
                                                      out_base);
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
