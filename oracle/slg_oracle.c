/*
 * Brute-force CPU oracle for s-line graphs of hypergraphs.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header or constant with the GPU library and must never serve a product
 * call.
 *
 * What it computes is the plain definition, not the paper's algorithm:
 *   - E_s = { e in E : |e| >= s }                        (Section II-B)
 *   - e_i, e_j are s-incident when |e_i n e_j| >= s       (Section II-B)
 *   - L_s(H) = <E_s, F>, F = s-incident pairs; each edge carries the
 *     overlap |e_i n e_j| = (H^T H)[i, j]                 (Section II-B)
 * Pairs are reported once, as (i, j) with i < j (Section III-B, the upper
 * triangle), ordered by i then j.
 *
 * The intersection of two hyperedges is counted the slowest obvious way:
 * flag the members of e_i in a vertex-indexed array, then count the members
 * of e_j that carry the flag. Every pair (i, j) with j > i is visited; no
 * pruning beyond the definition of E_s, no hashing, no two-hop traversal.
 * Only the hyperedge->vertex CSR is read, so the oracle does not depend on
 * the vertex->hyperedge CSR the GPU path consumes.
 *
 * Two thresholds are exposed so that tests can reach every part of the
 * definition: `size_min` selects E_{size_min}; `s` is the overlap threshold.
 * The s-line graph itself is size_min = s.
 *
 * Parity pins (see tests/test_oracle.py): the worked example of Section I
 * (hand-enumerated fixture), the identity L = H^T H of Section II-B via a
 * scipy sparse product, the 2-path count sum_v C(d_s(v), 2), the textbook
 * line graph of 2-uniform hypergraphs (Section I), nestedness L_{s+1} c L_s,
 * permutation equivariance and Python-set brute force on tiny inputs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* 0 on success; 1 bad pointer array; 2 vertex id out of range; 3 row not
 * strictly increasing (a hyperedge is a set). */
int slgo_validate(int64_t m, int64_t n, const int64_t *he_ptr, const int32_t *he_idx)
{
    if (m < 0 || n < 0) return 1;
    if (m > 0 && he_ptr[0] != 0) return 1;
    for (int64_t i = 0; i < m; ++i)
        if (he_ptr[i + 1] < he_ptr[i]) return 1;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = he_ptr[i]; p < he_ptr[i + 1]; ++p) {
            if (he_idx[p] < 0 || he_idx[p] >= n) return 2;
            if (p > he_ptr[i] && he_idx[p] <= he_idx[p - 1]) return 3;
        }
    }
    return 0;
}

/* |e_j n e_i| with e_i's members flagged in `flag`. */
static int64_t overlap_with_flagged(const int64_t *he_ptr, const int32_t *he_idx,
                                    int64_t j, const unsigned char *flag)
{
    int64_t c = 0;
    for (int64_t p = he_ptr[j]; p < he_ptr[j + 1]; ++p) c += flag[he_idx[p]];
    return c;
}

/* Row i of L_s over E_{size_min}: all j > i with |e_j| >= size_min and
 * |e_i n e_j| >= s. Writes up to the count when j_out != NULL. */
static int64_t one_row(int64_t m, const int64_t *he_ptr, const int32_t *he_idx,
                       int64_t size_min, int64_t s, int64_t i, unsigned char *flag,
                       int32_t *j_out, int32_t *w_out)
{
    if (he_ptr[i + 1] - he_ptr[i] < size_min) return 0;
    for (int64_t p = he_ptr[i]; p < he_ptr[i + 1]; ++p) flag[he_idx[p]] = 1;
    int64_t count = 0;
    for (int64_t j = i + 1; j < m; ++j) {
        if (he_ptr[j + 1] - he_ptr[j] < size_min) continue;
        int64_t w = overlap_with_flagged(he_ptr, he_idx, j, flag);
        if (w >= s) {
            if (j_out) {
                j_out[count] = (int32_t)j;
                w_out[count] = (int32_t)w;
            }
            ++count;
        }
    }
    for (int64_t p = he_ptr[i]; p < he_ptr[i + 1]; ++p) flag[he_idx[p]] = 0;
    return count;
}

/* counts[r] = number of edges of L_s in row rows[r]. */
int slgo_rows_count(int64_t m, int64_t n, const int64_t *he_ptr, const int32_t *he_idx,
                    int64_t size_min, int64_t s, const int64_t *rows, int64_t nrows,
                    int64_t *counts, int threads)
{
    int bad = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
        if (!flag) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!flag) continue;
            counts[r] = one_row(m, he_ptr, he_idx, size_min, s, rows[r], flag, NULL, NULL);
        }
        free(flag);
    }
    return bad;
}

/* Writes row rows[r] of L_s at j_out/w_out[offsets[r] .. offsets[r+1]). */
int slgo_rows_emit(int64_t m, int64_t n, const int64_t *he_ptr, const int32_t *he_idx,
                   int64_t size_min, int64_t s, const int64_t *rows, int64_t nrows,
                   const int64_t *offsets, int32_t *j_out, int32_t *w_out, int threads)
{
    int bad = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
        if (!flag) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!flag) continue;
            int64_t c = one_row(m, he_ptr, he_idx, size_min, s, rows[r], flag,
                                j_out + offsets[r], w_out + offsets[r]);
            if (c != offsets[r + 1] - offsets[r]) {
#pragma omp atomic write
                bad = 2;
            }
        }
        free(flag);
    }
    return bad;
}

/* Number of 2-paths (e_i, v, e_j), i < j, both in E_{size_min}, v in both.
 * Grouping the triples by their middle vertex v: each v contributes
 * C(d(v), 2) where d(v) counts the hyperedges of E_{size_min} holding v. */
int64_t slgo_two_paths(int64_t m, int64_t n, const int64_t *he_ptr, const int32_t *he_idx,
                       int64_t size_min)
{
    int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!deg) return -1;
    for (int64_t i = 0; i < m; ++i) {
        if (he_ptr[i + 1] - he_ptr[i] < size_min) continue;
        for (int64_t p = he_ptr[i]; p < he_ptr[i + 1]; ++p) deg[he_idx[p]] += 1;
    }
    int64_t total = 0;
    for (int64_t v = 0; v < n; ++v) total += deg[v] * (deg[v] - 1) / 2;
    free(deg);
    return total;
}

/* Number of 2-paths whose first hyperedge is rows[r] (the work of row i in
 * the two-hop traversal, used to express oracle time in 2-paths/s). */
int slgo_row_two_paths(int64_t m, int64_t n, const int64_t *he_ptr, const int32_t *he_idx,
                       int64_t size_min, const int64_t *rows, int64_t nrows, int64_t *out,
                       int threads)
{
    /* Sum of |e_i n e_j| over kept j > i, by brute force per row. */
    if (threads > 0) omp_set_num_threads(threads);
    int bad = 0;
#pragma omp parallel
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
        if (!flag) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!flag) continue;
            int64_t i = rows[r];
            int64_t total = 0;
            if (he_ptr[i + 1] - he_ptr[i] >= size_min) {
                for (int64_t p = he_ptr[i]; p < he_ptr[i + 1]; ++p) flag[he_idx[p]] = 1;
                for (int64_t j = i + 1; j < m; ++j) {
                    if (he_ptr[j + 1] - he_ptr[j] < size_min) continue;
                    total += overlap_with_flagged(he_ptr, he_idx, j, flag);
                }
                for (int64_t p = he_ptr[i]; p < he_ptr[i + 1]; ++p) flag[he_idx[p]] = 0;
            }
            out[r] = total;
        }
        free(flag);
    }
    return bad;
}

/* s-connected components (Section II-B): the maximal subsets of E_s whose
 * members are pairwise joined by s-walks (sequences of s-incident
 * hyperedges). Breadth-first search from every unlabelled hyperedge of E_s
 * in increasing id order; the neighbours of e are found by counting
 * |e n f| for every unlabelled f of E_s. label[i] = the first (smallest) id
 * of its component, -1 when |e_i| < s. Returns the number of components,
 * or -1 when memory runs out. O(m^2 |e|): small inputs only. */
int64_t slgo_components_brute(int64_t m, int64_t n, const int64_t *he_ptr, const int32_t *he_idx,
                              int64_t s, int32_t *label)
{
    unsigned char *flag = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!flag || !queue) {
        free(flag);
        free(queue);
        return -1;
    }
    for (int64_t i = 0; i < m; ++i) label[i] = (he_ptr[i + 1] - he_ptr[i] >= s) ? -2 : -1;
    int64_t count = 0;
    for (int64_t r = 0; r < m; ++r) {
        if (label[r] != -2) continue;
        ++count;
        label[r] = (int32_t)r;
        int64_t head = 0, tail = 0;
        queue[tail++] = r;
        while (head < tail) {
            const int64_t e = queue[head++];
            for (int64_t p = he_ptr[e]; p < he_ptr[e + 1]; ++p) flag[he_idx[p]] = 1;
            for (int64_t f = 0; f < m; ++f) {
                if (label[f] != -2) continue;
                if (overlap_with_flagged(he_ptr, he_idx, f, flag) >= s) {
                    label[f] = (int32_t)r;
                    queue[tail++] = f;
                }
            }
            for (int64_t p = he_ptr[e]; p < he_ptr[e + 1]; ++p) flag[he_idx[p]] = 0;
        }
    }
    free(flag);
    free(queue);
    return count;
}

/* The same components from a given edge list of L_s (both ends in E_s):
 * breadth-first search over the undirected adjacency of the edges. Returns
 * the number of components, -1 when memory runs out, -2 when an edge names
 * an id outside [0, m) or a hyperedge with fewer than s vertices. */
int64_t slgo_components_edges(int64_t m, const int64_t *he_ptr, int64_t s, int64_t num_edges,
                              const int32_t *row, const int32_t *col, int32_t *label)
{
    for (int64_t e = 0; e < num_edges; ++e) {
        const int64_t a = row[e], b = col[e];
        if (a < 0 || a >= m || b < 0 || b >= m) return -2;
        if (he_ptr[a + 1] - he_ptr[a] < s || he_ptr[b + 1] - he_ptr[b] < s) return -2;
    }
    int64_t *ptr = (int64_t *)calloc((size_t)(m + 1), sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * num_edges > 0 ? 2 * num_edges : 1));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!ptr || !adj || !queue) {
        free(ptr);
        free(adj);
        free(queue);
        return -1;
    }
    for (int64_t e = 0; e < num_edges; ++e) {
        ++ptr[row[e] + 1];
        ++ptr[col[e] + 1];
    }
    for (int64_t i = 0; i < m; ++i) ptr[i + 1] += ptr[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!fill) {
        free(ptr);
        free(adj);
        free(queue);
        return -1;
    }
    for (int64_t i = 0; i < m; ++i) fill[i] = ptr[i];
    for (int64_t e = 0; e < num_edges; ++e) {
        adj[fill[row[e]]++] = col[e];
        adj[fill[col[e]]++] = row[e];
    }
    free(fill);
    for (int64_t i = 0; i < m; ++i) label[i] = (he_ptr[i + 1] - he_ptr[i] >= s) ? -2 : -1;
    int64_t count = 0;
    for (int64_t r = 0; r < m; ++r) {
        if (label[r] != -2) continue;
        ++count;
        label[r] = (int32_t)r;
        int64_t head = 0, tail = 0;
        queue[tail++] = r;
        while (head < tail) {
            const int64_t e = queue[head++];
            for (int64_t q = ptr[e]; q < ptr[e + 1]; ++q) {
                const int64_t f = adj[q];
                if (label[f] == -2) {
                    label[f] = (int32_t)r;
                    queue[tail++] = f;
                }
            }
        }
    }
    free(ptr);
    free(adj);
    free(queue);
    return count;
}
