// gfx950 kernels for the optional preprocessing stages of the framework
// (Section IV, Stages 1 and 2):
//   - relabel-by-degree: hyperedge ids reassigned in order of size
//     (ascending or descending; equal sizes keep their id order);
//   - toplexes: the hyperedges no other hyperedge contains (the
//     simplification keeps only them), found from the overlaps of L_1: e_i
//     is inside e_j exactly when |e_i n e_j| = |e_i|;
//   - selection: the sub-hypergraph of an ordered list of hyperedges (both
//     CSRs rebuilt; the vertex lists by a stable sort of the new rows'
//     incidences by vertex, which keeps each list ascending).
// All of it is integer work with a deterministic result.
#include "slg_internal.h"

namespace slg {
namespace {

inline unsigned prep_grid(int64_t items, int threads, int64_t cap) {
    int64_t b = (items + threads - 1) / threads;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}

// key[i] = |e_i| (ascending) or n - |e_i| (descending); id[i] = i.
__global__ void size_key_kernel(const int64_t *__restrict__ he_ptr, int64_t m, int64_t n, int descending,
                                int32_t *__restrict__ key, int32_t *__restrict__ id) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t size = he_ptr[i + 1] - he_ptr[i];
        key[i] = (int32_t)(descending ? n - size : size);
        id[i] = (int32_t)i;
    }
}

// size_out[k] = |e_order[k]|; an id outside [0, m) or named twice sets err.
__global__ void select_sizes_kernel(const int32_t *__restrict__ order, int64_t count, const int64_t *__restrict__ he_ptr,
                                    int64_t m, int32_t *__restrict__ seen, int64_t *__restrict__ size_out,
                                    int *__restrict__ err) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = order[k];
        if (i < 0 || i >= m) {
            atomicOr(err, 1);
            size_out[k] = 0;
            continue;
        }
        if (atomicExch(&seen[i], 1) != 0) atomicOr(err, 2);
        size_out[k] = he_ptr[i + 1] - he_ptr[i];
    }
}

// One wavefront per new row k: the members of e_order[k] into the new row,
// and k beside every one of them (the row of each incidence, for the sort
// by vertex).
__global__ __launch_bounds__(256) void select_rows_kernel(const int32_t *__restrict__ order, int64_t count,
                                                          const int64_t *__restrict__ he_ptr,
                                                          const int32_t *__restrict__ he_idx, int64_t m,
                                                          const int64_t *__restrict__ new_ptr,
                                                          int32_t *__restrict__ new_idx,
                                                          int32_t *__restrict__ row_of) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; k < count; k += nwaves) {
        const int32_t i = order[k];
        if (i < 0 || i >= m) continue;  // flagged by select_sizes_kernel
        const int64_t a = he_ptr[i], b = he_ptr[i + 1], o = new_ptr[k];
        for (int64_t p = a + lane; p < b; p += 64) {
            new_idx[o + (p - a)] = he_idx[p];
            row_of[o + (p - a)] = (int32_t)k;
        }
    }
}

// Non-toplexes from the edges of L_1 (any order, any orientation): for an
// edge (a, b, w), e_a lies inside e_b when w = |e_a|; it is dropped when e_b
// is larger, or equal (the same set) with a smaller id, so one copy of a
// repeated maximal hyperedge stays. Empty hyperedges never have an edge and
// are dropped by toplex_init_kernel. An overlap above either size sets err.
__global__ void toplex_mark_kernel(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                                   const int32_t *__restrict__ w, int64_t num_edges,
                                   const int64_t *__restrict__ he_ptr, int64_t m, int32_t *__restrict__ drop,
                                   int *__restrict__ err) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < num_edges;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = row[e], b = col[e], x = w[e];
        if (a < 0 || a >= m || b < 0 || b >= m || a == b) {
            atomicOr(err, 1);
            continue;
        }
        const int64_t sa = he_ptr[a + 1] - he_ptr[a], sb = he_ptr[b + 1] - he_ptr[b];
        if (x < 1 || x > sa || x > sb) {
            atomicOr(err, 2);
            continue;
        }
        if (x == sa && (sb > sa || (sb == sa && b < a))) drop[a] = 1;
        if (x == sb && (sa > sb || (sa == sb && a < b))) drop[b] = 1;
    }
}

__global__ void toplex_init_kernel(const int64_t *__restrict__ he_ptr, int64_t m, int32_t *__restrict__ drop) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        drop[i] = he_ptr[i + 1] == he_ptr[i] ? 1 : 0;
}

// keep[i] = 1 - drop[i]; the kept ids in ascending order go to out[pre[i]].
__global__ void keep_flags_kernel(const int32_t *__restrict__ drop, int64_t m, int32_t *__restrict__ keep) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        keep[i] = 1 - drop[i];
}

__global__ void compact_ids_kernel(const int32_t *__restrict__ keep, const int64_t *__restrict__ pre, int64_t m,
                                   int32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (keep[i]) out[pre[i]] = (int32_t)i;
}

}  // namespace

hipError_t launch_size_keys(const int64_t *he_ptr, int64_t m, int64_t n, int descending, int32_t *key, int32_t *id,
                            hipStream_t st) {
    if (m <= 0) return hipSuccess;
    size_key_kernel<<<prep_grid(m, 256, 8192), 256, 0, st>>>(he_ptr, m, n, descending, key, id);
    return hipGetLastError();
}

hipError_t launch_select_sizes(const int32_t *order, int64_t count, const int64_t *he_ptr, int64_t m, int32_t *seen,
                               int64_t *size_out, int *err, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    select_sizes_kernel<<<prep_grid(count, 256, 8192), 256, 0, st>>>(order, count, he_ptr, m, seen, size_out, err);
    return hipGetLastError();
}

hipError_t launch_select_rows(const int32_t *order, int64_t count, const int64_t *he_ptr, const int32_t *he_idx,
                              int64_t m, const int64_t *new_ptr, int32_t *new_idx, int32_t *row_of, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    select_rows_kernel<<<prep_grid(count, 4, 8192), 256, 0, st>>>(order, count, he_ptr, he_idx, m, new_ptr, new_idx,
                                                                  row_of);
    return hipGetLastError();
}

hipError_t launch_toplex_flags(const int32_t *row, const int32_t *col, const int32_t *w, int64_t num_edges,
                               const int64_t *he_ptr, int64_t m, int32_t *drop, int32_t *keep, int *err,
                               hipStream_t st) {
    if (m <= 0) return hipSuccess;
    toplex_init_kernel<<<prep_grid(m, 256, 8192), 256, 0, st>>>(he_ptr, m, drop);
    if (num_edges > 0)
        toplex_mark_kernel<<<prep_grid(num_edges, 256, 16384), 256, 0, st>>>(row, col, w, num_edges, he_ptr, m, drop,
                                                                             err);
    keep_flags_kernel<<<prep_grid(m, 256, 8192), 256, 0, st>>>(drop, m, keep);
    return hipGetLastError();
}

hipError_t launch_compact_ids(const int32_t *keep, const int64_t *pre, int64_t m, int32_t *out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    compact_ids_kernel<<<prep_grid(m, 256, 8192), 256, 0, st>>>(keep, pre, m, out);
    return hipGetLastError();
}


}  // namespace slg
