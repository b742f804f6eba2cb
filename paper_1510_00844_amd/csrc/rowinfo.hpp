// Row analysis and binning (the work estimate of Section 2: flops(A,B)
// counts scalar multiplications; Gustavson's cost is O(flops + nnz + m + n),
// Section 3).  For each row i of A, restricted to the inner window
// [k_lo, k_hi):
//   a_beg[i], a_end[i]  index range of A's stored entries inside the window
//   flops[i]            sum over those entries k of nnz(B(k,:))
//   maxb[i]             max over those k of nnz(B(k,:))  (a lower bound of nnz(C(i,:)))
//   bin[i]              the accumulator class the row is sent to
// Rows with at most LONG_ROW entries are handled by 16-lane groups; longer
// rows are queued for a workgroup each so no wave walks a hub row alone.
#pragma once
#include "common.hpp"

namespace spg {

struct BinParams {
    int32_t small_max_flops;  // <= 64
    int32_t hash_max_flops;   // symbolic hash limit
    int32_t hash_max_nnz;     // numeric hash limit
    int32_t dense_ok;         // symbolic LDS bitmap allowed (n <= 2^19)
    int32_t rank_max_log2;    // numeric rank-space accumulator: largest capacity (log2), 0 = off
    int32_t chunk_counts;     // the bitmap pass records per-chunk counts for the numeric chunks
    int32_t chunk_min_nnz;    // rows with chunk counts and more outputs than this take rank chunks
    int32_t heap_max_lists;   // rows with at most this many A entries ...
    int32_t heap_max_flops;   // ... and products take the k-way merge (heap) bin; 0 = off
    int64_t ncols;            // n
};

constexpr int NBINS = 17;
constexpr int BIN_EMPTY = 0, BIN_TINY = 1, BIN_SMALL = 2, BIN_HASH0 = 3, BIN_DENSE = 12;
constexpr int BIN_DENSE_PAR = 11;  // numeric: column chunks of one row in parallel
constexpr int BIN_RANK0 = 13;  // rank-space accumulator, capacity 4096 << (b - BIN_RANK0)
constexpr int BIN_HEAP = 16;   // k-way merge of the row's few B rows (both passes)
constexpr int RANK_MIN_LOG2 = 12;
constexpr int LONG_ROW = 128;
constexpr int HASH_MIN_LOG2 = 7;  // 128 slots

__device__ inline int ceil_log2_i64(int64_t x) {
    return x <= 1 ? 0 : 64 - __clzll((unsigned long long)(x - 1));
}

// Symbolic bin from the row's work.
__device__ inline int sym_bin(int64_t flops, int64_t annz, const BinParams& bp) {
    if (flops == 0) return BIN_EMPTY;
    if (annz == 1) return BIN_TINY;
    if (flops <= bp.small_max_flops) return BIN_SMALL;
    if (annz <= bp.heap_max_lists && flops <= bp.heap_max_flops) return BIN_HEAP;
    // a bitmap over all n columns costs n/32 words to clear and count; use it
    // once the row's products outnumber that, or once a hash table would not fit
    bool bitmap_cheaper = bp.dense_ok && flops * 32 >= bp.ncols;
    if (flops <= bp.hash_max_flops && !bitmap_cheaper) {  // larger rows: bitmap, in blocks if n is large
        // at most 3/4 of the slots in use (the row's distinct columns are at most its products)
        int lg = ceil_log2_i64((4 * flops + 2) / 3);
        if (lg < HASH_MIN_LOG2) lg = HASH_MIN_LOG2;
        return BIN_HASH0 + (lg - HASH_MIN_LOG2);
    }
    return BIN_DENSE;
}

// Numeric bin from the exact output count.  Rows whose symbolic pass kept
// a full-width bitmap (sym_dense) reuse it: their values accumulate in LDS
// indexed by output rank when the count fits the largest capacity.
__device__ inline int num_bin(int64_t flops, int64_t annz, int64_t cnt, bool sym_dense,
                              const BinParams& bp) {
    if (cnt == 0) return BIN_EMPTY;
    if (annz == 1) return BIN_TINY;
    if (flops <= bp.small_max_flops) return BIN_SMALL;
    if (annz <= bp.heap_max_lists && flops <= bp.heap_max_flops) return BIN_HEAP;  // as in the symbolic pass
    if (sym_dense && bp.rank_max_log2 && cnt <= (1ll << bp.rank_max_log2)) {
        int lg = ceil_log2_i64(cnt);
        if (lg < RANK_MIN_LOG2) lg = RANK_MIN_LOG2;
        return BIN_RANK0 + (lg - RANK_MIN_LOG2);
    }
    // rows with a saved bitmap and chunk counts may take rank chunks before
    // the largest hash tables
    const bool chunks_ok = sym_dense && bp.chunk_counts;
    const int64_t hash_lim = chunks_ok ? bp.chunk_min_nnz : bp.hash_max_nnz;
    if (cnt <= hash_lim) {
        int lg = ceil_log2_i64((4 * cnt + 2) / 3);  // at most 3/4 of the slots in use
        if (lg < HASH_MIN_LOG2) lg = HASH_MIN_LOG2;
        return BIN_HASH0 + (lg - HASH_MIN_LOG2);
    }
    return chunks_ok ? BIN_DENSE_PAR : BIN_DENSE;
}

// The rows of one bin, located on the device: the per-bin row counts (the
// lists of the bins below b come first in `lists`).  Kernels launched this
// way stride over the bin's rows, so their launches need no host copy of
// the counts (the grid only sizes the parallelism).
struct BinRef {
    const int64_t* counts;
    const int32_t* lists;
    int32_t bin;
    __device__ inline void locate(const int32_t*& rows, int64_t& n) const {
        int64_t off = 0;
        for (int x = 0; x < bin; ++x) off += counts[x];
        rows = lists + off;
        n = counts[bin];
    }
};

// Rows of a bin over workgroups: row r goes to workgroup r mod gridDim.x.
// body(r, i) gets the position r in the bin list and the row i; it may use
// barriers (all threads call it).
template <class Body>
__device__ inline void for_each_bin_row(const BinRef& ref, Body body) {
    const int32_t* rows;
    int64_t n;
    ref.locate(rows, n);
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        body(r, (int64_t)rows[r]);
        __syncthreads();  // the row is done with the LDS
    }
}

struct RowInfoOut {
    int64_t* a_beg;
    int64_t* a_end;
    int64_t* flops;
    int32_t* maxb;
    uint8_t* bin;
    int64_t* cnt;        // symbolic counts (c_row_ptr + 1); EMPTY/TINY rows written here
    int64_t* bin_stats;  // [3][NBINS]: rows, flops, A entries
    int32_t* long_rows;  // queue of rows with more than LONG_ROW entries
    int32_t* long_count;
    unsigned long long* max_flops;  // largest flops_i over the rows (one value)
};

__device__ inline int64_t lower_bound_col(const int32_t* col, int64_t lo, int64_t hi, int64_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)col[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline void finish_row(int64_t i, int64_t beg, int64_t end, int64_t f, int32_t mb,
                                  const BinParams& bp, const RowInfoOut& o, int* s_hist,
                                  int64_t* s_flops, int64_t* s_annz, unsigned long long* s_fmax) {
    o.a_beg[i] = beg;
    o.a_end[i] = end;
    o.flops[i] = f;
    o.maxb[i] = mb;
    int b = sym_bin(f, end - beg, bp);
    o.bin[i] = (uint8_t)b;
    if (b == BIN_EMPTY) o.cnt[i] = 0;
    else if (b == BIN_TINY) o.cnt[i] = f;  // nnz(C(i,:)) = nnz(B(k,:)) exactly
    atomicAdd(&s_hist[b], 1);
    atomicAdd((unsigned long long*)&s_flops[b], (unsigned long long)f);
    atomicAdd((unsigned long long*)&s_annz[b], (unsigned long long)(end - beg));
    atomicMax(s_fmax, (unsigned long long)f);
}

__device__ inline void flush_stats(const RowInfoOut& o, int* s_hist, int64_t* s_flops,
                                   int64_t* s_annz, unsigned long long* s_fmax) {
    if (threadIdx.x == 0 && *s_fmax) atomicMax(o.max_flops, *s_fmax);
    if (threadIdx.x < NBINS) {
        int b = threadIdx.x;
        if (s_hist[b]) {
            atomicAdd((unsigned long long*)&o.bin_stats[b], (unsigned long long)s_hist[b]);
            atomicAdd((unsigned long long*)&o.bin_stats[NBINS + b], (unsigned long long)s_flops[b]);
            atomicAdd((unsigned long long*)&o.bin_stats[2 * NBINS + b], (unsigned long long)s_annz[b]);
        }
    }
}

__device__ inline void rowinfo_row(const Csr& A, const Csr& B, int64_t k_lo, int64_t k_hi, int full_window,
                                   const BinParams& bp, const RowInfoOut& o, int64_t i, int gl, int* s_hist,
                                   int64_t* s_flops, int64_t* s_annz, unsigned long long* s_fmax);

// 256 threads = 16 groups of 16 lanes, one row per group; the grid strides
// over groups of 16 rows (few workgroups, so few global statistics atomics).
__global__ void __launch_bounds__(256) k_rowinfo(Csr A, Csr B, int64_t k_lo, int64_t k_hi,
                                                 int full_window, BinParams bp, RowInfoOut o) {
    __shared__ int s_hist[NBINS];
    __shared__ int64_t s_flops[NBINS], s_annz[NBINS];
    __shared__ unsigned long long s_fmax;
    if (threadIdx.x < NBINS) {
        s_hist[threadIdx.x] = 0;
        s_flops[threadIdx.x] = 0;
        s_annz[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) s_fmax = 0;
    __syncthreads();
    const int g = threadIdx.x >> 4, gl = threadIdx.x & 15;
    for (int64_t i0 = (int64_t)blockIdx.x * 16; i0 < A.nrows; i0 += (int64_t)gridDim.x * 16)
        rowinfo_row(A, B, k_lo, k_hi, full_window, bp, o, i0 + g, gl, s_hist, s_flops, s_annz, &s_fmax);
    __syncthreads();
    flush_stats(o, s_hist, s_flops, s_annz, &s_fmax);
}

__device__ inline void rowinfo_row(const Csr& A, const Csr& B, int64_t k_lo, int64_t k_hi, int full_window,
                                   const BinParams& bp, const RowInfoOut& o, int64_t i, int gl, int* s_hist,
                                   int64_t* s_flops, int64_t* s_annz, unsigned long long* s_fmax) {
    bool active = i < A.nrows;
    int64_t beg = 0, end = 0;
    if (active) {
        beg = A.rp[i];
        end = A.rp[i + 1];
        if (!full_window) {
            // the A row is sorted by column: binary search the window edges
            beg = lower_bound_col(A.col, beg, end, k_lo);
            end = lower_bound_col(A.col, beg, end, k_hi);
        }
        if (end - beg > LONG_ROW) {
            if (gl == 0) {
                int slot = atomicAdd(o.long_count, 1);
                o.long_rows[slot] = (int32_t)i;
            }
            active = false;
        }
    }
    int64_t f = 0;
    int32_t mb = 0;
    if (active) {
        // two A entries per lane per step, so their dependent loads overlap
        for (int64_t p = beg + gl; p < end; p += 32) {
            const bool two = p + 16 < end;
            const int64_t k0 = A.col[p];
            const int64_t k1 = two ? (int64_t)A.col[p + 16] : k0;
            const int64_t l0 = B.rp[k0 + 1] - B.rp[k0];
            const int64_t l1 = two ? B.rp[k1 + 1] - B.rp[k1] : 0;
            f += l0 + l1;
            mb = l0 > mb ? (int32_t)l0 : mb;
            mb = l1 > mb ? (int32_t)l1 : mb;
        }
    }
    // reduce inside the 16-lane group (xor offsets < 16 stay in the group)
#pragma unroll
    for (int d = 8; d > 0; d >>= 1) {
        f += __shfl_xor(f, d, SPG_WAVE);
        int32_t o2 = __shfl_xor(mb, d, SPG_WAVE);
        mb = o2 > mb ? o2 : mb;
    }
    if (active && gl == 0) finish_row(i, beg, end, f, mb, bp, o, s_hist, s_flops, s_annz, s_fmax);
}

// One 256-thread workgroup per queued long row, grid-stride over the queue.
__global__ void __launch_bounds__(256) k_rowinfo_long(Csr A, Csr B, int64_t k_lo, int64_t k_hi,
                                                      int full_window, BinParams bp,
                                                      RowInfoOut o) {
    __shared__ int s_hist[NBINS];
    __shared__ int64_t s_flops[NBINS], s_annz[NBINS];
    __shared__ int64_t s_red[8];
    __shared__ int32_t s_redm[8];
    __shared__ unsigned long long s_fmax;
    if (threadIdx.x < NBINS) {
        s_hist[threadIdx.x] = 0;
        s_flops[threadIdx.x] = 0;
        s_annz[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) s_fmax = 0;
    __syncthreads();
    const int nq = *o.long_count;
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int64_t i = o.long_rows[q];
        int64_t beg = A.rp[i], end = A.rp[i + 1];
        if (!full_window) {
            beg = lower_bound_col(A.col, beg, end, k_lo);
            end = lower_bound_col(A.col, beg, end, k_hi);
        }
        int64_t f = 0;
        int32_t mb = 0;
        for (int64_t p = beg + threadIdx.x; p < end; p += 256) {
            int64_t k = A.col[p];
            int64_t len = B.rp[k + 1] - B.rp[k];
            f += len;
            mb = len > mb ? (int32_t)len : mb;
        }
        f = wave_reduce_add(f);
        mb = wave_reduce_max(mb);
        const int w = threadIdx.x / SPG_WAVE;
        if (lane_id() == 0) {
            s_red[w] = f;
            s_redm[w] = mb;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t tf = 0;
            int32_t tm = 0;
            for (int x = 0; x < 4; ++x) {
                tf += s_red[x];
                tm = s_redm[x] > tm ? s_redm[x] : tm;
            }
            finish_row(i, beg, end, tf, tm, bp, o, s_hist, s_flops, s_annz, &s_fmax);
        }
        __syncthreads();
    }
    flush_stats(o, s_hist, s_flops, s_annz, &s_fmax);
}

// Numeric classification from exact counts (after the symbolic scan).
// A bitmap row keeps its rank paths only if the symbolic pass saved its
// bitmap (heavy_idx >= 0; NULL = no bitmaps saved).
__global__ void __launch_bounds__(256) k_num_classify(int64_t m, const int64_t* c_rp,
                                                      const int64_t* a_beg, const int64_t* a_end,
                                                      const int64_t* flops, BinParams bp,
                                                      const int32_t* heavy_idx, uint8_t* bin, int64_t* bin_stats) {
    __shared__ int s_hist[NBINS];
    __shared__ int64_t s_flops[NBINS], s_annz[NBINS], s_cnnz[NBINS];
    if (threadIdx.x < NBINS) {
        s_hist[threadIdx.x] = 0;
        s_flops[threadIdx.x] = 0;
        s_annz[threadIdx.x] = 0;
        s_cnnz[threadIdx.x] = 0;
    }
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) {
        int64_t cnt = c_rp[i + 1] - c_rp[i];
        int64_t an = a_end[i] - a_beg[i];
        int64_t f = flops[i];
        const bool saved = bin[i] == BIN_DENSE && heavy_idx && heavy_idx[i] >= 0;
        int b = num_bin(f, an, cnt, saved, bp);
        bin[i] = (uint8_t)b;
        atomicAdd(&s_hist[b], 1);
        atomicAdd((unsigned long long*)&s_flops[b], (unsigned long long)f);
        atomicAdd((unsigned long long*)&s_annz[b], (unsigned long long)an);
        atomicAdd((unsigned long long*)&s_cnnz[b], (unsigned long long)cnt);
    }
    __syncthreads();
    if (threadIdx.x < NBINS) {
        int b = threadIdx.x;
        if (s_hist[b]) {
            atomicAdd((unsigned long long*)&bin_stats[b], (unsigned long long)s_hist[b]);
            atomicAdd((unsigned long long*)&bin_stats[NBINS + b], (unsigned long long)s_flops[b]);
            atomicAdd((unsigned long long*)&bin_stats[2 * NBINS + b], (unsigned long long)s_annz[b]);
            atomicAdd((unsigned long long*)&bin_stats[3 * NBINS + b], (unsigned long long)s_cnnz[b]);
        }
    }
}

// Counting-sort scatter of rows into per-bin lists.  bin_stats[0..NBINS)
// holds the per-bin row counts; list segment of bin b starts at the sum of
// the counts of bins < b.  cursor[NBINS] must be zero on entry.
__global__ void __launch_bounds__(256) k_bin_scatter(int64_t m, const uint8_t* bin,
                                                     const int64_t* bin_counts, int32_t* cursor,
                                                     int32_t* lists) {
    __shared__ int s_cnt[NBINS];
    __shared__ int s_base[NBINS];
    if (threadIdx.x < NBINS) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int b = -1, local = 0;
    if (i < m) {
        b = bin[i];
        local = atomicAdd(&s_cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < NBINS) {
        int bb = threadIdx.x;
        int64_t off = 0;
        for (int x = 0; x < bb; ++x) off += bin_counts[x];
        s_base[bb] = s_cnt[bb] ? (int)off + atomicAdd(&cursor[bb], s_cnt[bb]) : 0;
    }
    __syncthreads();
    if (b >= 0) lists[s_base[b] + local] = (int32_t)i;
}

// Longest-processing-time order of the row lists of a run of consecutive
// bins [b_lo, b_lo + nb): within each bin, rows with more products first,
// so that the heaviest workgroups start early and the end of a launch is not
// held up by a large row that started last.  The bins' lists are contiguous,
// so one counting sort over the run with key (bin - b_lo, work class) keeps
// every bin in place; 256 work classes per bin, 8 per power of two of the
// products (rows within about 12% of each other share a class).
constexpr int LPT_KEYS = 256;
constexpr int LPT_MAX_BINS = 8;
__device__ inline int lpt_class(int64_t w) {
    if (w < 1) w = 1;
    const int e = 63 - __clzll((unsigned long long)w);  // floor(log2 w)
    const int frac = e >= 3 ? (int)((w >> (e - 3)) & 7) : (int)((w << (3 - e)) & 7);
    const int k = e * 8 + frac;
    return LPT_KEYS - 1 - (k < LPT_KEYS - 1 ? k : LPT_KEYS - 1);  // more work: smaller class
}
__device__ inline int lpt_key(int32_t row, const uint8_t* bin, int b_lo, const int64_t* work) {
    return ((int)bin[row] - b_lo) * LPT_KEYS + lpt_class(work[row]);
}

// The rows of bins [b_lo, b_hi) in the lists: offset and count from the
// per-bin counts on the device.
__device__ inline void bin_run(const int64_t* counts, int b_lo, int b_hi, int64_t& off, int64_t& n) {
    off = 0;
    for (int x = 0; x < b_lo; ++x) off += counts[x];
    n = 0;
    for (int x = b_lo; x < b_hi; ++x) n += counts[x];
}

__global__ void __launch_bounds__(256) k_lpt_hist(const int32_t* lists, const int64_t* counts, int b_lo, int b_hi,
                                                  const uint8_t* bin, int nk, const int64_t* work, int32_t* hist) {
    __shared__ int32_t s_h[LPT_KEYS * LPT_MAX_BINS];
    int64_t off, n;
    bin_run(counts, b_lo, b_hi, off, n);
    if ((int64_t)blockIdx.x * 256 >= n) return;
    for (int k = threadIdx.x; k < nk; k += 256) s_h[k] = 0;
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256)
        atomicAdd(&s_h[lpt_key(lists[off + r], bin, b_lo, work)], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += 256)
        if (s_h[k]) atomicAdd(&hist[k], s_h[k]);
}

// one workgroup: counts -> exclusive offsets, in place (nk <= 256 * LPT_MAX_BINS;
// thread t owns keys [t * per, (t + 1) * per))
__global__ void __launch_bounds__(256) k_lpt_scan(int32_t* hist, int nk) {
    __shared__ int32_t tmp[256 / SPG_WAVE + 1];
    const int per = (nk + 255) / 256;
    const int k0 = threadIdx.x * per;
    int32_t part = 0;
    for (int k = k0; k < k0 + per && k < nk; ++k) part += hist[k];
    int32_t total;
    int32_t run = block_exclusive_scan<256, int32_t>(part, &total, tmp);
    for (int k = k0; k < k0 + per && k < nk; ++k) {
        const int32_t v = hist[k];
        hist[k] = run;
        run += v;
    }
}

// Scatter by key; each 256-row tile of a workgroup takes its key bases with
// one atomic per key.  tmp receives the ordered rows (n entries).
__global__ void __launch_bounds__(256) k_lpt_scatter(const int32_t* lists, const int64_t* counts, int b_lo, int b_hi,
                                                     const uint8_t* bin, int nk, const int64_t* work, int32_t* cursor,
                                                     int32_t* tmp) {
    __shared__ int32_t s_cnt[LPT_KEYS * LPT_MAX_BINS];
    int64_t off, n;
    bin_run(counts, b_lo, b_hi, off, n);
    for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < n; t0 += (int64_t)gridDim.x * 256) {
        for (int k = threadIdx.x; k < nk; k += 256) s_cnt[k] = 0;
        __syncthreads();
        const int64_t r = t0 + threadIdx.x;
        int key = 0, local = 0, row = 0;
        if (r < n) {
            row = lists[off + r];
            key = lpt_key(row, bin, b_lo, work);
            local = atomicAdd(&s_cnt[key], 1);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nk; k += 256)
            if (s_cnt[k]) s_cnt[k] = atomicAdd(&cursor[k], s_cnt[k]);  // now the tile's base for key k
        __syncthreads();
        if (r < n) tmp[s_cnt[key] + local] = row;
        __syncthreads();
    }
}

// The ordered rows back into the lists.
__global__ void __launch_bounds__(256) k_lpt_copy(int32_t* lists, const int64_t* counts, int b_lo, int b_hi,
                                                  const int32_t* tmp) {
    int64_t off, n;
    bin_run(counts, b_lo, b_hi, off, n);
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256)
        lists[off + r] = tmp[r];
}

}  // namespace spg
