// Internal interface between the host API (slg_api.cpp) and the gfx950
// kernels (slg_kernels.hip). Not installed; the public ABI is include/slg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "slg.h"

namespace slg {

// ---- tuning constants of the hot path ------------------------------------
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kLightMax = 2048;        // rows with <= this many 2-paths: wave-sort tier
constexpr int kTinyMax = 8;            // rows with <= this many 2-paths: one lane each
constexpr int kLightClasses = 7;       // tiny (lane per row), then 64 ... 2048 keys per wave
constexpr int kHeavyThreads = 256;     // workgroup of the bitmap-rank tier (4 per CU)
constexpr int kRangeBits = 1 << 16;    // hyperedge-id range of one heavy slot (bitmap bits)
constexpr int kRangeWords = kRangeBits / 32;
constexpr int kRankCap = 4096;         // overlap counters per rank window (LDS, u16)
constexpr int64_t kSlotWork = 4096;    // 2-paths per heavy slot before a row is split
constexpr int kWideMembers = 65535;    // rows this large need u32 overlap counters
// Dense tier: a row whose partners fill most of E_s (at least dense_ratio
// 2-paths per eight candidate partners) counts into direct LDS counters over
// aligned windows of kDenseWindow consecutive E_s positions.
constexpr int kDenseBits = 14;
constexpr int kDenseWindow = 1 << kDenseBits;  // E_s positions per dense slot (u32 counters, 64 KB)
constexpr int kDenseThreads = 512;            // workgroup of the dense tier (2 per CU)
constexpr int kDenseRatio = 4;                // default: 2-paths per 8 candidate partners to go dense
constexpr int kDenseMinRange = 8192;          // default: fewest candidate partners to go dense
constexpr int kDensePad = 1024;  // entries past the end of the E_s-position lists the dense walk may load
constexpr long long kDenseChunk = 1 << 16;  // dense-store entries a workgroup takes at a time

// Row classes written by the planning kernel.
enum RowClass : uint8_t {
    kNone = 0,
    kLight0 = 1,
    kHeavy = kLight0 + kLightClasses,  // bitmap-rank tier, u16 counters
    kHeavyWide = kHeavy + 1,           // bitmap-rank tier, u32 counters
    kDense = kHeavyWide + 1            // direct-counter tier over E_s windows
};
constexpr int kNumLists = kLightClasses + 3;  // light classes + heavy + heavy-wide + dense slots
constexpr int kNumHeavyLists = 3;             // heavy, heavy-wide, dense descriptor lists

// Per-call parameters, passed by value and staged in LDS by each kernel so
// that a runtime threshold index reads LDS, not a private copy.
struct EmitParams {
    int32_t k;                      // number of thresholds
    int32_t s[SLG_MAX_S];           // strictly increasing, s[0] = s_min
    int32_t slot_lo, slot_hi;       // emit only slots in [slot_lo, slot_hi)
    int32_t pad_;
    int32_t *row[SLG_MAX_S];        // COO i per threshold (may be null)
    int32_t *col[SLG_MAX_S];        // j per threshold
    int32_t *w[SLG_MAX_S];          // overlap per threshold
    int64_t *row_ptr[SLG_MAX_S];    // CSR offsets per threshold
    int64_t out_base[SLG_MAX_S];    // global edge offset of the buffers' first entry
    const int32_t *row_s;           // per-row threshold (batched form, k = 1), or null
    const int32_t *row_base;        // per-row id base subtracted on output, or null
};

// Device-side view of one hypergraph after pruning.
struct Pruned {
    int64_t m, n, nnz;
    const int64_t *he_ptr;
    const int32_t *he_idx;
    const int64_t *vs_ptr;    // vertex lists restricted to E_{s_min}
    const int32_t *vs_idx;
    const int32_t *tail_beg;  // per incidence (i, v): first position in v's list after i
    const int32_t *row_s;     // per-row threshold (batched form), or null for s_min
    // E_s positions (the dense tier; null when the plan has none): cid[i] =
    // rank of row i among the kept rows (-1 if pruned), cid_row[c] = the row
    // of rank c, and vs_cid = vs_idx with every id replaced by its rank
    // (ranks keep the id order, so the lists stay sorted). vs_win = vs_cid
    // modulo kDenseWindow: a rank's place in its (aligned) window, all that
    // the dense walk needs, in half the bytes.
    const int32_t *cid;
    const int32_t *cid_row;
    const int32_t *vs_cid;
    const uint16_t *vs_win;
};

// Slot table: a slot is (row i, hyperedge-id range) with its own output
// segment; a light row is one slot, a heavy row one or more.
struct Slots {
    int64_t count;
    const int32_t *row;
};

// One heavy slot, stored in processing order. The row's boundary table
// holds, for member q of e_i, bounds[bptr + q] = first position of q's tail
// with a partner >= ja, and bounds[bptr + k + q] = the same for jb (the next
// slot's start, or the tail end for the row's last slot). A dense slot's
// ja, jb are E_s positions: ja is a multiple of kDenseWindow and the slot's
// partners lie in [ja, ja + kDenseWindow).
struct HeavyDesc {
    int32_t row, ja, jb, k;  // row i, partner range [ja, jb), k = |e_i|
    int32_t slot, last;      // output segment; 1 on the row's last slot
    int64_t bptr;
};

// Overlaps kept by the counting pass for the emit pass: heavy slot t (its
// index in the heavy list) holds n[t] entries in rank order at off[t], each
// (partner - ja) | overlap << 16 (a slot spans at most 2^16 ids, and a
// non-wide row has fewer than 2^16 members); off is the exclusive prefix of
// the slots' 2-path counts, which bound their distinct partners.
// The dense tier's store holds only the partners whose overlap reaches the
// smallest threshold, each (position - window start) | overlap << 16 (a
// window spans 2^14 positions of E_s; its emit maps positions back to ids);
// a slot's room comes from a device cursor once it knows its count (off[t]),
// and n[t] = -1 marks a slot that found the store full (its emit walks the
// 2-paths again).
struct CountStore {
    uint32_t *ent;
    int64_t *off;
    int32_t *n;
};

// The same for the light rows (wavefront-sort tier): row i holds n[i]
// (partner id, overlap) pairs in partner order at off[i], the exclusive
// prefix of the light rows' 2-path counts.
struct LightStore {
    int32_t *key;
    uint16_t *cnt;
    int64_t *off;
    int32_t *n;
};

// ---- launchers (all enqueue on `st`, return hipError_t) -------------------
hipError_t launch_exclusive_scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *partials,
                                     hipStream_t st);
hipError_t launch_exclusive_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *partials,
                                     hipStream_t st);
hipError_t launch_exclusive_scan_u8(const uint8_t *in, int64_t n, int64_t *out, int64_t *partials,
                                    hipStream_t st);
int64_t scan_partials_size(int64_t n);
// Capacity of the large-row piece list of row planning.
int64_t plan_pieces_cap(int64_t nnz);

// K1: keep flags per incidence of the vertex CSR, then compaction.
hipError_t launch_keep_incidence(int64_t nnz, const int32_t *v_idx, const int64_t *he_ptr, int64_t m,
                                 int32_t s_min, const int32_t *row_s, uint8_t *flag, hipStream_t st);
hipError_t launch_compact_vertex_lists(int64_t n, int64_t nnz, const int64_t *v_ptr,
                                       const int32_t *v_idx, const uint8_t *flag,
                                       const int64_t *pos, int64_t *vs_ptr, int32_t *vs_idx,
                                       hipStream_t st);

// E_s positions: flag[i] = row i kept at s_min (or its own threshold), pre =
// its exclusive scan (int64[m+1]), then cid / cid_row, and vs_cid and vs_win
// over the pruned lists (vs_ptr[n] entries).
hipError_t launch_row_keep(int64_t m, const int64_t *he_ptr, int32_t s_min, const int32_t *row_s, uint8_t *flag,
                           hipStream_t st);
hipError_t launch_cid(int64_t m, const uint8_t *flag, const int64_t *pre, int32_t *cid, int32_t *cid_row,
                      hipStream_t st);
hipError_t launch_vs_cid(int64_t n, int64_t m, int64_t nnz, const int64_t *vs_ptr, const int32_t *vs_idx,
                         const int32_t *cid, int32_t *vs_cid, uint16_t *vs_win, hipStream_t st);

// K1/K2: per kept row, tail offsets, 2-path work, last partner, slot count.
// dense_ratio = 0 keeps every row off the dense tier (then g.cid may be
// null); dense_work gets the 2-paths of dense rows.
// Rows outside [row_lo, row_hi) are planned as pruned rows (no work, no
// slots); their member tails are not located.
hipError_t launch_row_plan(const Pruned &g, int32_t s_min, int32_t light_max, int64_t slot_work, int64_t row_lo,
                           int64_t row_hi, int32_t dense_ratio, int32_t dense_min, int32_t *tail_beg, int64_t *work,
                           int32_t *jmax, int32_t *nslots, uint8_t *rclass, int64_t *bsize,
                           unsigned long long *class_count, int *err, unsigned long long *heavy_work,
                           unsigned long long *dense_work, int64_t *pieces, unsigned long long *num_pieces,
                           hipStream_t st);
// Light lists and heavy descriptors (heavy lists in slot order). hat:
// int64[3 (m + 1)] and hcnt: int32[3 m] scratch, partials: scan_partials_size(m).
hipError_t launch_fill_slots(int64_t m, const int64_t *he_ptr, const int64_t *slot_base,
                             const int32_t *nslots, const int32_t *jmax, const uint8_t *rclass,
                             const int64_t *bbase, const int32_t *cid, int64_t *hat, int32_t *hcnt,
                             int64_t *partials, int32_t *slot_row, int32_t *const *lists, HeavyDesc *const *heavy,
                             const int64_t *caps, unsigned long long *list_fill, int *err, hipStream_t st);
// A row block [r0, r1): nslots / rclass / bsize of the other rows zeroed
// (from the *_all copies of every row), the block's list sizes and heavy /
// dense 2-paths added to class_count / heavy_work / dense_work.
hipError_t launch_block_mask(int64_t m, int64_t r0, int64_t r1, const int32_t *nslots_all, const uint8_t *rclass_all,
                             const int64_t *bsize_all, const int64_t *work, int32_t *nslots, uint8_t *rclass,
                             int64_t *bsize, unsigned long long *class_count, unsigned long long *heavy_work,
                             unsigned long long *dense_work, hipStream_t st);
// out[c] = position of the first slot >= slots[c] in a heavy list ordered by
// slot, c in [0, n).
hipError_t launch_list_cuts(const HeavyDesc *desc, int64_t count, const int64_t *slots, int64_t n, int64_t *out,
                            hipStream_t st);
// out[0..1] = positions of the first slot >= s0 and >= s1 in a heavy list.
hipError_t launch_heavy_range(const HeavyDesc *desc, int64_t count, int64_t s0, int64_t s1, int64_t *out,
                              hipStream_t st);
hipError_t launch_bounds(const Pruned &g, const HeavyDesc *desc, int64_t count, int32_t *bounds,
                         hipStream_t st);

// K3/K4/K5: count (EMIT=false) or emit (EMIT=true) per slot.
// store (counting pass of the wavefront-sort classes only, or null): keep
// the overlaps.
hipError_t launch_light(int cls, bool emit, const int32_t *list, int64_t count, const Slots &sl,
                        const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, const LightStore *store, hipStream_t st);
// Emit pass of a wavefront-sort class list from the light store.
hipError_t launch_light_store_emit(const int32_t *list, int64_t count, const Slots &sl, const LightStore &store,
                                   const EmitParams &ep, const int64_t *slot_off, hipStream_t st);
// lw[i] = 2-paths of row i if it is in a wavefront-sort class, else 0.
hipError_t launch_light_work(int64_t m, const uint8_t *rclass, const int64_t *work, int32_t *lw, hipStream_t st);
// Persistent launch: `resident` workgroups (0 = a default) take slots from
// the device counter `ticket`, which the caller zeroes before the launch.
// store (counting pass of non-wide slots only, or null): keep the overlaps.
hipError_t launch_heavy(bool emit, bool wide, const HeavyDesc *desc, int64_t count, int64_t slots,
                        const int32_t *bounds, const Pruned &g, const EmitParams &ep, int64_t *slot_cnt,
                        const int64_t *slot_off, int64_t *ticket, int resident, const CountStore *store,
                        hipStream_t st);
// work[t] = 2-paths of heavy slot t (from the boundary table).
hipError_t launch_slot_work(const HeavyDesc *desc, int64_t count, const int32_t *bounds, int64_t *work,
                            hipStream_t st);
// Emit pass of the heavy slots from the counting pass's store, or, with
// cid_row, of the dense slots from theirs (entries hold E_s positions, mapped
// to ids through cid_row; slots with n[t] < 0 are left to launch_dense(emit)).
hipError_t launch_heavy_store_emit(const HeavyDesc *desc, int64_t count, int64_t slots, const CountStore &store,
                                   const EmitParams &ep, const int64_t *slot_off, const int32_t *cid_row,
                                   hipStream_t st);
// Dense tier, persistent like launch_heavy. Counting pass (emit = false):
// slot_cnt gets every threshold's survivors and, with a store, the slot's
// survivors of the smallest threshold go to the store (room reserved from
// store_cursor, up to store_cap entries). Emit pass: writes the outputs by
// walking the 2-paths again, for every slot (store == null) or only those
// the store could not hold (n[t] < 0).
// order (or null: list order): the slots in the order the workgroups take
// them, as positions in desc.
hipError_t launch_dense(bool emit, const HeavyDesc *desc, int64_t count, const int32_t *order, int64_t slots,
                        const int32_t *bounds,
                        const Pruned &g, const EmitParams &ep, int64_t *slot_cnt, const int64_t *slot_off,
                        int64_t *ticket, int resident, const CountStore *store, int64_t *store_cursor,
                        int64_t store_cap, hipStream_t st);
// key[t] = the E_s window of dense slot t (its ja >> kDenseBits), id[t] = t.
hipError_t launch_dense_keys(const HeavyDesc *desc, int64_t count, int32_t *key, int32_t *id, hipStream_t st);
// Workgroups of the dense kernel that fit on the device at once.
int dense_resident(int device);
// *out += sum of n[0..count) (int32).
hipError_t launch_sum_i32(const int32_t *n, int64_t count, int64_t *out, hipStream_t st);
hipError_t launch_heavy_edges(const HeavyDesc *desc, int64_t count, const int64_t *slot_cnt, int64_t S,
                              int32_t K, int64_t *out, hipStream_t st);
// Workgroups of the heavy kernel that fit on the device at once.
int heavy_resident(int device);

// K6: row_ptr[k][i - row_lo] = slot_off[k][slot_base[i]] - out_base[k], i in [row_lo, row_hi].
hipError_t launch_row_ptr(int64_t row_lo, int64_t row_hi, const int64_t *slot_base,
                          const int64_t *slot_off, int64_t slots, const EmitParams &ep, hipStream_t st);
// Output bytes before row i (all thresholds; 12 B per edge + 8 B per row_ptr
// entry), i in [0, m]; and slot_off[k][slot_base[r]] gathered at rows[c].
hipError_t launch_row_bytes(int64_t m, const int64_t *slot_base, const int64_t *slot_off, int64_t slots,
                            int32_t K, int64_t *out, hipStream_t st);
hipError_t launch_gather_offsets(const int64_t *rows, int64_t count, const int64_t *slot_base,
                                 const int64_t *slot_off, int64_t slots, int32_t K, int64_t *out,
                                 hipStream_t st);
hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t value, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t st);

// Batched form: one graph of the disjoint union.
struct UnionPart {
    const int64_t *he_ptr, *v_ptr;
    const int32_t *he_idx, *v_idx;
    int64_t m, n, nnz, m_off, n_off, nnz_off;
    int32_t s, pad_;
};
// Concatenate `count` graphs into the union arrays (ids offset per graph);
// row_s/row_base get each row's threshold and first union row id.
hipError_t launch_union(const UnionPart *parts, int32_t count, int64_t max_elems, int64_t *he_ptr,
                        int32_t *he_idx, int64_t *v_ptr, int32_t *v_idx, int32_t *row_s, int32_t *row_base,
                        hipStream_t st);
// out[c] = src[idx[c]].
hipError_t launch_gather_i64(const int64_t *src, const int64_t *idx, int64_t count, int64_t *out,
                             hipStream_t st);

// s-connected components of L_s (hooking union-find over the edge list):
// label[i] = i for |e_i| >= s, else -1; then every edge (row, col) joins the
// trees of its ends (the larger root under the smaller); finally out[i] is
// the root of i, the smallest id of its component (or -1). count gets the
// number of roots; err is set if a bounded loop ran out (never expected).
hipError_t launch_cc_init(const int64_t *he_ptr, int64_t m, int32_t s, int32_t *label, hipStream_t st);
hipError_t launch_cc_hook(const int32_t *row, const int32_t *col, int64_t num_edges, int64_t m, int32_t *label,
                          int *err, hipStream_t st);
hipError_t launch_cc_finish(int64_t m, const int32_t *label, int32_t *out, unsigned long long *count,
                            hipStream_t st);
// ID squeezing: flag[i] = 1 for every end of an edge (ids outside [0, m):
// err |= 4, also in the hook).
hipError_t launch_mark_ends(const int32_t *row, const int32_t *col, int64_t num_edges, int64_t m, int32_t *flag,
                            int *err, hipStream_t st);
// new_id[i] = pre[i] when flag[i], else -1 (pre: exclusive scan of flag).
hipError_t launch_squeeze_ids(int64_t m, const int32_t *flag, const int64_t *pre, int32_t *new_id, hipStream_t st);
// row[e] = new_id[row[e]], col[e] = new_id[col[e]].
hipError_t launch_remap_edges(int32_t *row, int32_t *col, int64_t num_edges, const int32_t *new_id,
                              hipStream_t st);

// Stable LSD radix sort (slg_sort.hip): one pass orders items by the digit
// (key >> shift) & (2^bits - 1), bits <= kSortDigitBits, keeping the order of
// equal digits; a, b: optional int32 payloads (b only with a). hist:
// int32[2^bits * sort_chunks(n)], off: int64 of that count + 1, partials:
// scan_partials_size of that count.
constexpr int kSortDigitBits = 8;
int64_t sort_chunks(int64_t n);
int sort_passes(int key_bits);
hipError_t launch_sort_pass(const int32_t *key_in, const int32_t *a_in, const int32_t *b_in, int64_t n, int shift,
                            int bits, int32_t *hist, int64_t *off, int64_t *partials, int32_t *key_out,
                            int32_t *a_out, int32_t *b_out, hipStream_t st);
// out[0..2] += (edges, sum of w, sum of SplitMix64(i * 2^32 + j) ^ w) mod 2^64.
hipError_t launch_digest(const int32_t *row, const int32_t *col, const int32_t *w, int64_t n,
                         unsigned long long *out, hipStream_t st);
// lower_ptr[c] = number of ascending keys skey[0..n) below c, c in [0, m].
hipError_t launch_key_bounds(const int32_t *skey, int64_t n, int64_t m, int64_t *lower_ptr, hipStream_t st);
// err |= 1 unless (row_ptr, row, col) is an upper triangle in CSR order.
hipError_t launch_check_upper(const int64_t *row_ptr, const int32_t *row, const int32_t *col, int64_t n, int64_t m,
                              int *err, hipStream_t st);
// Symmetric CSR from the upper triangle (row_ptr, row, col, w) and the same
// edges sorted by column (skey = column, srow, sw); w / sw / sym_w may be
// null together. lower_ptr: int64[m+1] scratch.
hipError_t launch_symmetric(const int32_t *skey, const int32_t *srow, const int32_t *sw, const int64_t *row_ptr,
                            const int32_t *row, const int32_t *col, const int32_t *w, int64_t n, int64_t m,
                            int64_t *lower_ptr, int64_t *sym_ptr, int32_t *sym_col, int32_t *sym_w,
                            hipStream_t st);

// Preprocessing (slg_prep.hip). key[i] = |e_i| or n - |e_i|, id[i] = i.
hipError_t launch_size_keys(const int64_t *he_ptr, int64_t m, int64_t n, int descending, int32_t *key, int32_t *id,
                            hipStream_t st);
// size_out[k] = |e_order[k]|; err |= 1 for an id outside [0, m), 2 for a
// repeated id (seen: int32[m], zeroed).
hipError_t launch_select_sizes(const int32_t *order, int64_t count, const int64_t *he_ptr, int64_t m, int32_t *seen,
                               int64_t *size_out, int *err, hipStream_t st);
// Rows of the selection at new_ptr, with the new row id of every incidence.
hipError_t launch_select_rows(const int32_t *order, int64_t count, const int64_t *he_ptr, const int32_t *he_idx,
                              int64_t m, const int64_t *new_ptr, int32_t *new_idx, int32_t *row_of, hipStream_t st);
// keep[i] = 1 for a toplex, from the edges of L_1 (drop: int32[m] scratch);
// err |= 1 for an id outside [0, m) or a loop, 2 for an impossible overlap.
hipError_t launch_toplex_flags(const int32_t *row, const int32_t *col, const int32_t *w, int64_t num_edges,
                               const int64_t *he_ptr, int64_t m, int32_t *drop, int32_t *keep, int *err,
                               hipStream_t st);
// out[pre[i]] = i for every i with keep[i].
hipError_t launch_compact_ids(const int32_t *keep, const int64_t *pre, int64_t m, int32_t *out, hipStream_t st);

// Fixed device scratch of slg_components_noalloc: the largest m it takes,
// and the address of this device's copy of the array (looked up on first
// use with `device` current; then cached).
constexpr int64_t kNoAllocRows = int64_t(1) << 24;
hipError_t noalloc_scratch(int device, void **out);

// Validation kernels (SLG_VALIDATE).
hipError_t launch_validate_ptr(const int64_t *ptr, int64_t rows, int64_t nnz, int *err,
                               hipStream_t st);
hipError_t launch_validate_rows(const int64_t *ptr, const int32_t *idx, int64_t rows,
                                int64_t limit, int *err, hipStream_t st);
hipError_t launch_validate_transpose(const int64_t *he_ptr, const int32_t *he_idx, int64_t m,
                                     const int64_t *v_ptr, const int32_t *v_idx, int64_t n, int *err,
                                     hipStream_t st);

}  // namespace slg
