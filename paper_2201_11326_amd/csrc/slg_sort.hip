// gfx950 kernels that turn an emitted s-line graph into a consumer-ready
// graph (Stage 4 of the framework, Section IV: the edge list becomes the
// graph's adjacency):
//   - a stable least-significant-digit radix sort of int32 keys carrying up
//     to two int32 payloads (used to transpose an edge list: sorting the
//     upper triangle by column keeps rows ascending inside every column);
//   - the symmetric CSR of L_s from its upper triangle.
// Every step is integer work and deterministic: the sort is stable, so the
// output does not depend on scheduling.
#include "slg_internal.h"

namespace slg {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRounds = 128;  // rounds of kSortThreads items per chunk
constexpr int64_t kSortChunk = (int64_t)kSortThreads * kSortRounds;
constexpr int kSortBins = 1 << kSortDigitBits;

__device__ __forceinline__ int lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Digit counts of every chunk: hist[d * nchunks + c] = items of chunk c whose
// digit (key >> shift) & (2^bits - 1) is d. Digit-major, so one exclusive
// scan gives every (digit, chunk) its first output position.
__global__ __launch_bounds__(kSortThreads) void sort_hist_kernel(const int32_t *__restrict__ key, int64_t n,
                                                                 int shift, int bits, int64_t nchunks,
                                                                 int32_t *__restrict__ hist) {
    __shared__ int h[kSortBins];
    const int nb = 1 << bits;
    const unsigned mask = (unsigned)nb - 1u;
    for (int d = threadIdx.x; d < nb; d += kSortThreads) h[d] = 0;
    __syncthreads();
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t base = c * kSortChunk, end = min(n, base + kSortChunk);
        for (int64_t q = base + threadIdx.x; q < end; q += kSortThreads)
            atomicAdd(&h[((unsigned)key[q] >> shift) & mask], 1);
        __syncthreads();
        for (int d = threadIdx.x; d < nb; d += kSortThreads) {
            hist[(int64_t)d * nchunks + c] = h[d];
            h[d] = 0;
        }
        __syncthreads();
    }
}

// Stable scatter of every chunk, a tile of kSortTile items at a time. An
// item's rank among the equal digits of its tile counts such items in
// earlier rounds (LDS running counts), in lower wavefronts of its round (LDS
// counts) and in lower lanes of its wavefront (ballots on the digit bits),
// so items keep their order. The tile is then reordered by digit in LDS and
// written out in runs, which keeps the HBM writes of a digit contiguous.
// `run` holds the next output position of every digit.
constexpr int kTileRounds = 16;
constexpr int kSortTile = kSortThreads * kTileRounds;
static_assert(kSortRounds % kTileRounds == 0, "a chunk is whole tiles");

template <int NP>
__global__ __launch_bounds__(kSortThreads) void sort_scatter_kernel(
    const int32_t *__restrict__ key_in, const int32_t *__restrict__ a_in, const int32_t *__restrict__ b_in,
    int64_t n, int shift, int bits, int64_t nchunks, const int64_t *__restrict__ off,
    int32_t *__restrict__ key_out, int32_t *__restrict__ a_out, int32_t *__restrict__ b_out) {
    __shared__ int64_t run[kSortBins];
    __shared__ int cnt[kSortBins];          // tile counts so far, then the tile's digit starts
    __shared__ int wcnt[kSortWaves][kSortBins];
    __shared__ int wsum[kSortWaves];
    __shared__ int32_t tk[kSortTile];
    __shared__ int32_t ta[NP > 0 ? kSortTile : 1];
    __shared__ int32_t tb[NP > 1 ? kSortTile : 1];
    const int nb = 1 << bits;
    const unsigned mask = (unsigned)nb - 1u;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int t = threadIdx.x; t < kSortWaves * kSortBins; t += kSortThreads) (&wcnt[0][0])[t] = 0;
    for (int t = threadIdx.x; t < kSortBins; t += kSortThreads) cnt[t] = 0;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        for (int d = threadIdx.x; d < nb; d += kSortThreads) run[d] = off[(int64_t)d * nchunks + c];
        __syncthreads();
        for (int64_t t0 = c * kSortChunk; t0 < min(n, (c + 1) * kSortChunk); t0 += kSortTile) {
            const int tn = (int)min((int64_t)kSortTile, n - t0);  // items in this tile
            unsigned key[kTileRounds];
            int32_t pa[kTileRounds], pb[kTileRounds];
            int rk[kTileRounds];
#pragma unroll
            for (int r = 0; r < kTileRounds; ++r) {
                const int i = r * kSortThreads + threadIdx.x;
                key[r] = i < tn ? (unsigned)key_in[t0 + i] : 0u;
                if (NP > 0) pa[r] = i < tn ? a_in[t0 + i] : 0;
                if (NP > 1) pb[r] = i < tn ? b_in[t0 + i] : 0;
            }
#pragma unroll
            for (int r = 0; r < kTileRounds; ++r) {
                const bool valid = r * kSortThreads + (int)threadIdx.x < tn;
                const unsigned d = (key[r] >> shift) & mask;
                unsigned long long peers = __ballot(valid);
                for (int i = 0; i < bits; ++i) {
                    const bool bit = (d >> i) & 1u;
                    const unsigned long long bb = __ballot(bit);
                    peers &= bit ? bb : ~bb;
                }
                const int rank = lanes_below(peers);
                if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
                __syncthreads();
                int pre = 0;
                for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
                rk[r] = cnt[d] + pre + rank;  // rank within the tile's digit d
                __syncthreads();
                for (int dd = threadIdx.x; dd < nb; dd += kSortThreads) {
                    int tot = 0;
#pragma unroll
                    for (int w = 0; w < kSortWaves; ++w) {
                        tot += wcnt[w][dd];
                        wcnt[w][dd] = 0;
                    }
                    cnt[dd] += tot;
                }
                __syncthreads();
            }
            // digit starts within the tile (exclusive scan of cnt)
            {
                int v[kSortBins / kSortThreads > 0 ? kSortBins / kSortThreads : 1];
                int mine = 0;
                constexpr int per = kSortBins / kSortThreads > 0 ? kSortBins / kSortThreads : 1;
#pragma unroll
                for (int j = 0; j < per; ++j) {
                    const int d = threadIdx.x * per + j;
                    v[j] = d < nb ? cnt[d] : 0;
                    mine += v[j];
                }
                int incl = mine;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                if (lane == 63) wsum[wave] = incl;
                __syncthreads();
                int base = incl - mine;
                for (int w = 0; w < wave; ++w) base += wsum[w];
#pragma unroll
                for (int j = 0; j < per; ++j) {
                    const int d = threadIdx.x * per + j;
                    if (d < nb) cnt[d] = base;  // start of digit d in the tile
                    base += v[j];
                }
                __syncthreads();
            }
            // reorder by digit in LDS
#pragma unroll
            for (int r = 0; r < kTileRounds; ++r) {
                if (r * kSortThreads + (int)threadIdx.x < tn) {
                    const unsigned d = (key[r] >> shift) & mask;
                    const int q = cnt[d] + rk[r];
                    tk[q] = (int32_t)key[r];
                    if (NP > 0) ta[q] = pa[r];
                    if (NP > 1) tb[q] = pb[r];
                }
            }
            __syncthreads();
            // runs of equal digits to their places
            for (int q = threadIdx.x; q < tn; q += kSortThreads) {
                const int32_t k = tk[q];
                const unsigned d = ((unsigned)k >> shift) & mask;
                const int64_t pos = run[d] + (q - cnt[d]);
                key_out[pos] = k;
                if (NP > 0) a_out[pos] = ta[q];
                if (NP > 1) b_out[pos] = tb[q];
            }
            __syncthreads();
            // next tile: advance the digit positions, clear the counts
            for (int d = threadIdx.x; d < nb; d += kSortThreads) {
                const int end = d + 1 < nb ? cnt[d + 1] : tn;
                run[d] += end - cnt[d];
            }
            __syncthreads();
            for (int d = threadIdx.x; d < kSortBins; d += kSortThreads) cnt[d] = 0;
            __syncthreads();
        }
    }
}

// The flat kernels below give every thread kFlat items per grid step, loaded
// before any is used, so that enough loads are in flight to cover HBM
// latency.
constexpr int kFlat = 4;

// Checks that (row_ptr, row, col) is the upper triangle of a graph on m
// vertices in CSR order: row[e] = r for e in [row_ptr[r], row_ptr[r+1]),
// r < col[e] < m, columns strictly increasing along a row. err |= 1 if not.
__global__ void check_upper_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ row,
                                   const int32_t *__restrict__ col, int64_t n, int64_t m, int *__restrict__ err) {
    bool bad = false;
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kFlat;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x * kFlat + threadIdx.x; e0 < n; e0 += step) {
        int32_t r[kFlat], c[kFlat], rp[kFlat], cp[kFlat];
#pragma unroll
        for (int j = 0; j < kFlat; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            const bool in = e < n;
            r[j] = in ? row[e] : 0;
            c[j] = in ? col[e] : 1;
            rp[j] = (in && e > 0) ? row[e - 1] : -1;
            cp[j] = (in && e > 0) ? col[e - 1] : -1;
        }
#pragma unroll
        for (int j = 0; j < kFlat; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            if (e >= n) continue;
            if (r[j] < 0 || r[j] >= m || c[j] <= r[j] || c[j] >= m) {
                bad = true;
                continue;
            }
            if (e < row_ptr[r[j]] || e >= row_ptr[r[j] + 1]) bad = true;
            if (rp[j] == r[j] && cp[j] >= c[j]) bad = true;
        }
    }
    if (bad) atomicOr(err, 1);
}

// row_ptr must start at 0, end at n and never decrease.
__global__ void check_ptr_kernel(const int64_t *__restrict__ row_ptr, int64_t m, int64_t n, int *__restrict__ err) {
    bool bad = false;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x)
        if (row_ptr[r] > row_ptr[r + 1]) bad = true;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (row_ptr[0] != 0 || row_ptr[m] != n)) bad = true;
    if (bad) atomicOr(err, 1);
}

// lower_ptr[c] = number of sorted keys below c, for c in [0, m].
__global__ void key_bounds_kernel(const int32_t *__restrict__ skey, int64_t n, int64_t m,
                                  int64_t *__restrict__ lower_ptr) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= m; c += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)skey[mid] < c)
                lo = mid + 1;
            else
                hi = mid;
        }
        lower_ptr[c] = lo;
    }
}

// Row r of the symmetric CSR is its partners below r (the transpose, rows
// ascending) followed by those above r (its own row): it starts at
// lower_ptr[r] + row_ptr[r].
__global__ void sym_ptr_kernel(const int64_t *__restrict__ lower_ptr, const int64_t *__restrict__ row_ptr,
                               int64_t m, int64_t *__restrict__ sym_ptr) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= m; r += (int64_t)gridDim.x * blockDim.x)
        sym_ptr[r] = lower_ptr[r] + row_ptr[r];
}

// Sorted entry p (column c, row i) lands at p + row_ptr[c]: the entries of
// columns below c, plus the upper entries of rows below c.
__global__ void sym_lower_kernel(const int32_t *__restrict__ skey, const int32_t *__restrict__ srow,
                                 const int32_t *__restrict__ sw, int64_t n, int64_t m,
                                 const int64_t *__restrict__ row_ptr, int32_t *__restrict__ sym_col,
                                 int32_t *__restrict__ sym_w) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kFlat;
    for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x * kFlat + threadIdx.x; p0 < n; p0 += step) {
        int32_t c[kFlat], r[kFlat], w[kFlat];
#pragma unroll
        for (int j = 0; j < kFlat; ++j) {
            const int64_t p = p0 + (int64_t)j * blockDim.x;
            const bool in = p < n;
            c[j] = in ? skey[p] : -1;
            r[j] = in ? srow[p] : 0;
            w[j] = (in && sw) ? sw[p] : 0;
        }
#pragma unroll
        for (int j = 0; j < kFlat; ++j) {
            const int64_t p = p0 + (int64_t)j * blockDim.x;
            if (c[j] < 0 || c[j] >= m) continue;  // past the end, or the input check has failed
            const int64_t q = p + row_ptr[c[j]];
            if (q < 0 || q >= 2 * n) continue;
            sym_col[q] = r[j];
            if (sw) sym_w[q] = w[j];
        }
    }
}

// Upper entry e of row r lands at e + lower_ptr[r + 1].
__global__ void sym_upper_kernel(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                                 const int32_t *__restrict__ w, int64_t n, int64_t m,
                                 const int64_t *__restrict__ lower_ptr, int32_t *__restrict__ sym_col,
                                 int32_t *__restrict__ sym_w) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kFlat;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x * kFlat + threadIdx.x; e0 < n; e0 += step) {
        int32_t r[kFlat], c[kFlat], ww[kFlat];
#pragma unroll
        for (int j = 0; j < kFlat; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            const bool in = e < n;
            r[j] = in ? row[e] : -1;
            c[j] = in ? col[e] : 0;
            ww[j] = (in && w) ? w[e] : 0;
        }
#pragma unroll
        for (int j = 0; j < kFlat; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            if (r[j] < 0 || r[j] >= m) continue;
            const int64_t q = e + lower_ptr[r[j] + 1];
            if (q < 0 || q >= 2 * n) continue;
            sym_col[q] = c[j];
            if (w) sym_w[q] = ww[j];
        }
    }
}

// Order-independent digest of an edge list: the number of edges, the sum
// of the overlaps, and the sum mod 2^64 of SplitMix64's output function
// (Steele, Lea and Flood's mixer as published by Vigna) applied to
// i * 2^32 + j, xor the overlap. Equal edge sets give equal digests in any
// order, and the digests of disjoint parts add up to the digest of their
// union, so a streamed result can be checked chunk by chunk.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void digest_kernel(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ w, int64_t n,
                                                     unsigned long long *__restrict__ out) {
    unsigned long long cnt = 0, sw = 0, h = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long i = (unsigned)row[e], j = (unsigned)col[e];
        const unsigned long long x = (unsigned long long)(unsigned)w[e];
        cnt += 1;
        sw += x;
        h += splitmix64((i << 32) | j) ^ x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o);
        sw += __shfl_xor(sw, o);
        h += __shfl_xor(h, o);
    }
    if ((threadIdx.x & 63) == 0 && cnt) {
        atomicAdd(&out[0], cnt);
        atomicAdd(&out[1], sw);
        atomicAdd(&out[2], h);
    }
}

inline unsigned sort_grid(int64_t items, int threads, int64_t cap) {
    int64_t b = (items + threads - 1) / threads;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int64_t sort_chunks(int64_t n) { return (n + kSortChunk - 1) / kSortChunk; }

int sort_passes(int key_bits) { return key_bits <= 0 ? 0 : (key_bits + kSortDigitBits - 1) / kSortDigitBits; }

hipError_t launch_sort_pass(const int32_t *key_in, const int32_t *a_in, const int32_t *b_in, int64_t n, int shift,
                            int bits, int32_t *hist, int64_t *off, int64_t *partials, int32_t *key_out,
                            int32_t *a_out, int32_t *b_out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (bits < 1 || bits > kSortDigitBits || shift < 0 || shift + bits > 32) return hipErrorInvalidValue;
    const int64_t nchunks = sort_chunks(n);
    const unsigned grid = (unsigned)(nchunks < 65536 ? nchunks : 65536);
    sort_hist_kernel<<<grid, kSortThreads, 0, st>>>(key_in, n, shift, bits, nchunks, hist);
    hipError_t e = launch_exclusive_scan_i32(hist, (int64_t)(1 << bits) * nchunks, off, partials, st);
    if (e != hipSuccess) return e;
    if (b_in)
        sort_scatter_kernel<2><<<grid, kSortThreads, 0, st>>>(key_in, a_in, b_in, n, shift, bits, nchunks, off,
                                                               key_out, a_out, b_out);
    else if (a_in)
        sort_scatter_kernel<1><<<grid, kSortThreads, 0, st>>>(key_in, a_in, nullptr, n, shift, bits, nchunks, off,
                                                               key_out, a_out, nullptr);
    else
        sort_scatter_kernel<0><<<grid, kSortThreads, 0, st>>>(key_in, nullptr, nullptr, n, shift, bits, nchunks,
                                                               off, key_out, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_digest(const int32_t *row, const int32_t *col, const int32_t *w, int64_t n,
                         unsigned long long *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    digest_kernel<<<sort_grid(n, 256, 8192), 256, 0, st>>>(row, col, w, n, out);
    return hipGetLastError();
}

hipError_t launch_key_bounds(const int32_t *skey, int64_t n, int64_t m, int64_t *lower_ptr, hipStream_t st) {
    key_bounds_kernel<<<sort_grid(m + 1, 256, 4096), 256, 0, st>>>(skey, n, m, lower_ptr);
    return hipGetLastError();
}

hipError_t launch_check_upper(const int64_t *row_ptr, const int32_t *row, const int32_t *col, int64_t n, int64_t m,
                              int *err, hipStream_t st) {
    check_ptr_kernel<<<sort_grid(m > 0 ? m : 1, 256, 4096), 256, 0, st>>>(row_ptr, m, n, err);
    if (n > 0) check_upper_kernel<<<sort_grid(n, 256 * kFlat, 16384), 256, 0, st>>>(row_ptr, row, col, n, m, err);
    return hipGetLastError();
}

hipError_t launch_symmetric(const int32_t *skey, const int32_t *srow, const int32_t *sw, const int64_t *row_ptr,
                            const int32_t *row, const int32_t *col, const int32_t *w, int64_t n, int64_t m,
                            int64_t *lower_ptr, int64_t *sym_ptr, int32_t *sym_col, int32_t *sym_w,
                            hipStream_t st) {
    key_bounds_kernel<<<sort_grid(m + 1, 256, 4096), 256, 0, st>>>(skey, n, m, lower_ptr);
    sym_ptr_kernel<<<sort_grid(m + 1, 256, 4096), 256, 0, st>>>(lower_ptr, row_ptr, m, sym_ptr);
    if (n > 0) {
        sym_lower_kernel<<<sort_grid(n, 256 * kFlat, 16384), 256, 0, st>>>(skey, srow, sw, n, m, row_ptr, sym_col, sym_w);
        sym_upper_kernel<<<sort_grid(n, 256 * kFlat, 16384), 256, 0, st>>>(row, col, w, n, m, lower_ptr, sym_col, sym_w);
    }
    return hipGetLastError();
}

}  // namespace slg
