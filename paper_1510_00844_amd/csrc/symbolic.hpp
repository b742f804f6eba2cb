// Symbolic phase: nnz(C(i,:)) = |union over stored A(i,k), k in window, of
// the column sets of B(k,:)|, the stored-set part of the product definition
// (Section 2; explicit zeros count, so values are never read).  Each bin of
// rows gets its own accumulator:
//   SMALL  (<= 64 products): one wave per row, the products' column keys
//          sit one per lane and are sorted across the wave; the count is
//          the number of run heads.
//   HASH   : workgroup per row, open-addressing table of int32 keys in LDS
//            (linear probing, >= 4/3 slots per product).
//   DENSE  : workgroup per row, an n-bit bitmap in LDS (n <= 2^19), the
//            structural part of the sparse accumulator of Section 3.
#pragma once
#include "products.hpp"
#include "rowinfo.hpp"

namespace spg {

constexpr int32_t EMPTY_KEY = -1;
constexpr int MAX_CHUNKS = 256;  // column chunks per row recorded by the bitmap pass

// Locate, for each lane, the product with flat index = lane among the row's
// products (<= 64 of them): returns the A index p and B index q.  The A row
// is walked in order, so flat order is ascending k, then ascending column.
__device__ inline bool wave_locate_product(const Csr& A, const Csr& B, int64_t beg, int64_t end,
                                           int64_t& p_out, int64_t& q_out) {
    // Lane f takes the f-th product of the row in (A entry, B entry) order.
    // Up to 64 A entries at a time: each lane loads one entry's B segment,
    // a wave scan gives the segment offsets, and each lane finds the segment
    // holding its product by a binary search over the scanned offsets.
    const int lane = lane_id();
    int pos = 0;  // products in earlier groups of A entries
    bool have = false;
    for (int64_t base = beg; base < end && pos < SPG_WAVE; base += SPG_WAVE) {
        const int64_t p = base + lane;
        int64_t bs = 0;
        int len = 0;
        if (p < end) {
            const int64_t k = A.col[p];
            bs = B.rp[k];
            len = (int)(B.rp[k + 1] - bs);
        }
        const int incl = wave_inclusive_scan_add(len);
        const int total = __shfl(incl, SPG_WAVE - 1, SPG_WAVE);
        const int f = lane - pos;
        int t = 0;  // first lane whose inclusive count exceeds f
#pragma unroll
        for (int step = SPG_WAVE / 2; step > 0; step >>= 1) {
            const int v = __shfl(incl, t + step - 1, SPG_WAVE);
            if (v <= f) t += step;
        }
        t = t < SPG_WAVE ? t : SPG_WAVE - 1;
        const int64_t bst = __shfl(bs, t, SPG_WAVE);
        const int excl = __shfl(incl - len, t, SPG_WAVE);
        if (f >= 0 && f < total) {
            p_out = base + t;
            q_out = bst + (f - excl);
            have = true;
        }
        pos += total;
    }
    return have;
}

// The same for SMALL_ROWS rows at once whose A windows hold at most 64
// entries (one group): each dependent load level (A columns, B extents, B
// entries) is issued for all rows before any is waited for, so a wave keeps
// that many rows' loads in flight.  Lane f takes product f of row u.
constexpr int SMALL_ROWS = 2;
__device__ inline void wave_locate_rows(const Csr& A, const Csr& B, const int64_t* beg, const int64_t* end,
                                        bool* have, int64_t* p_out, int64_t* q_out) {
    const int lane = lane_id();
    int64_t kk[SMALL_ROWS];
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u) {
        const int64_t p = beg[u] + lane;
        kk[u] = p < end[u] ? (int64_t)A.col[p] : -1;
    }
    int64_t bs[SMALL_ROWS];
    int len[SMALL_ROWS];
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u) {
        bs[u] = 0;
        len[u] = 0;
        if (kk[u] >= 0) {
            bs[u] = B.rp[kk[u]];
            len[u] = (int)(B.rp[kk[u] + 1] - bs[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u) {
        const int incl = wave_inclusive_scan_add(len[u]);
        const int total = __builtin_amdgcn_readlane(incl, SPG_WAVE - 1);
        int t = 0;  // first lane whose inclusive count exceeds this lane's product
#pragma unroll
        for (int step = SPG_WAVE / 2; step > 0; step >>= 1) {
            const int v = __shfl(incl, t + step - 1, SPG_WAVE);
            if (v <= lane) t += step;
        }
        t = t < SPG_WAVE ? t : SPG_WAVE - 1;
        const int64_t bst = __shfl(bs[u], t, SPG_WAVE);
        const int excl = __shfl(incl - len[u], t, SPG_WAVE);
        have[u] = lane < total;
        p_out[u] = beg[u] + t;
        q_out[u] = bst + (lane - excl);
    }
}

// The rows of one wave: SMALL_ROWS consecutive list entries.  locate(u, i,
// have, p, q) gets each row's products; rows past the list are skipped, and a
// row with more than 64 A entries in the window (empty B rows among them)
// falls back to the one-row search.
template <class Body>
__device__ inline void for_small_rows(const Csr& A, const Csr& B, const int32_t* rows, int64_t nrows, int64_t w,
                                      const int64_t* a_beg, const int64_t* a_end, Body body) {
    int64_t i[SMALL_ROWS], beg[SMALL_ROWS], end[SMALL_ROWS];
    bool ok[SMALL_ROWS];
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u) {
        const int64_t r = w * SMALL_ROWS + u;
        ok[u] = r < nrows;
        i[u] = ok[u] ? rows[r] : 0;
    }
    bool one_group = true;
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u) {
        beg[u] = ok[u] ? a_beg[i[u]] : 0;
        end[u] = ok[u] ? a_end[i[u]] : 0;
        one_group = one_group && end[u] - beg[u] <= SPG_WAVE;
    }
    bool have[SMALL_ROWS];
    int64_t p[SMALL_ROWS], q[SMALL_ROWS];
    if (one_group) {
        wave_locate_rows(A, B, beg, end, have, p, q);
    } else {
#pragma unroll
        for (int u = 0; u < SMALL_ROWS; ++u) {
            p[u] = q[u] = 0;
            have[u] = wave_locate_product(A, B, beg[u], end[u], p[u], q[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u)
        if (ok[u]) body(u, i[u], have[u], p[u], q[u]);
}

// 4 waves per block, SMALL_ROWS rows per wave, the waves striding over the
// bin's rows (located on the device).  A row's (at most 64) product columns
// are counted by inserting them into a per-row LDS set of SS_SLOTS int32
// keys (at most half full): one insertion per lane, no sort.
constexpr int SS_LOG2 = 7;
constexpr int SS_SLOTS = 1 << SS_LOG2;
static_assert(SS_SLOTS >= 2 * SPG_WAVE && SS_SLOTS % SPG_WAVE == 0, "a set holds a row's products at most half full");

__global__ void __launch_bounds__(256) k_sym_small(Csr A, Csr B, BinRef ref, const int64_t* a_beg,
                                                   const int64_t* a_end, int64_t* cnt) {
    __shared__ int32_t sets[4][SMALL_ROWS][SS_SLOTS];
    const int32_t* rows;
    int64_t nrows;
    ref.locate(rows, nrows);
    const int lane = lane_id();
    const int wv = (int)(threadIdx.x >> 6);
    for (int64_t w = (int64_t)blockIdx.x * 4 + wv; w * SMALL_ROWS < nrows; w += (int64_t)gridDim.x * 4) {
#pragma unroll
        for (int u = 0; u < SMALL_ROWS; ++u)
            for (int t = lane; t < SS_SLOTS; t += SPG_WAVE) sets[wv][u][t] = EMPTY_KEY;
        wave_lds_sync();
        int32_t mine[SMALL_ROWS];
        int64_t row[SMALL_ROWS];
        for_small_rows(A, B, rows, nrows, w, a_beg, a_end, [&](int u, int64_t i, bool have, int64_t, int64_t q) {
            row[u] = i;
            mine[u] = 0;
            if (have) {
                const int32_t j = B.col[q];
                int32_t* T = sets[wv][u];
                uint32_t h = hash_slot(j, SS_LOG2);
                while (true) {  // ends: the set is at most half full
                    const int32_t old = atomicCAS(&T[h], EMPTY_KEY, j);
                    if (old == EMPTY_KEY) {
                        mine[u] = 1;
                        break;
                    }
                    if (old == j) break;
                    h = (h + 1) & (SS_SLOTS - 1);
                }
            }
        });
#pragma unroll
        for (int u = 0; u < SMALL_ROWS; ++u) {
            if (w * SMALL_ROWS + u >= nrows) break;
            const int32_t tot = wave_reduce_add(mine[u]);
            if (lane == 0) cnt[row[u]] = tot;
        }
        wave_lds_sync();  // the sets are read before the next rows clear them
    }
}

// Workgroup per row (rows claimed one at a time).
template <int NT, int LOG2T>
__global__ void __launch_bounds__(NT) k_sym_hash(Csr A, Csr B, BinRef ref, const int64_t* a_beg, const int64_t* a_end,
                                                 int64_t* cnt) {
    constexpr int T = 1 << LOG2T;
    __shared__ int32_t tab[T];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    for_each_bin_row(ref, [&](int64_t, int64_t i) {
        for (int t = threadIdx.x; t < T; t += NT) tab[t] = EMPTY_KEY;
        __syncthreads();
        int32_t mine = 0;
        for_each_product_u<NT, 4>(
            a_beg[i], a_end[i], L,
            [&](int64_t p, int64_t& bs, int32_t& len) {
                int64_t k = A.col[p];
                bs = B.rp[k];
                len = (int32_t)(B.rp[k + 1] - bs);
            },
            [&](int, int64_t) {},
            [&](int64_t q) { return B.col[q]; },
            [&](int, int32_t j) {
                uint32_t h = hash_slot(j, LOG2T);
                while (true) {
                    int32_t cur = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (cur == j) break;
                    if (cur == EMPTY_KEY) {
                        int32_t old = atomicCAS(&tab[h], EMPTY_KEY, j);
                        if (old == EMPTY_KEY) {
                            ++mine;
                            break;
                        }
                        if (old == j) break;
                    }
                    h = (h + 1) & (T - 1);
                }
            });
        int32_t total = block_reduce_add<NT, int32_t>(mine, red);
        if (threadIdx.x == 0) cnt[i] = total;
    });
}

// HASH rows of at most 384 products (the 128-, 256- and 512-slot bins): one
// wave per row, four rows per workgroup, each wave with its own set of
// SW_SLOTS int32 keys (at most 3/8 full).  The row's A entries are taken 64
// at a time (wave_products): each lane holds one entry's B segment, a wave
// scan gives the segment offsets, and each product is placed by a binary
// search of the offsets across the lanes, its column inserted into the set.
// New columns are counted.  No block-wide product enumeration and no
// barriers: the rows of these bins are short.
constexpr int SW_LOG2 = 10;
constexpr int SW_SLOTS = 1 << SW_LOG2;

__global__ void __launch_bounds__(256) k_sym_hash_wave(Csr A, Csr B, BinRef ref, const int64_t* a_beg,
                                                       const int64_t* a_end, int64_t* cnt) {
    __shared__ int4 tab4[4][SW_SLOTS / 4];
    int4* T4 = tab4[threadIdx.x >> 6];
    int32_t* T = reinterpret_cast<int32_t*>(T4);
    const int lane = lane_id();
    const int32_t* rows;
    int64_t n;
    ref.locate(rows, n);
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[r];
        for (int t = lane; t < SW_SLOTS / 4; t += SPG_WAVE) T4[t] = make_int4(EMPTY_KEY, EMPTY_KEY, EMPTY_KEY, EMPTY_KEY);
        wave_lds_sync();
        int32_t mine = 0;
        wave_products<4, int32_t>(
            a_beg[i], a_end[i],
            [&](int64_t p, int64_t& bs, int32_t& len, int32_t&) {
                const int64_t k = A.col[p];
                bs = B.rp[k];
                len = (int32_t)(B.rp[k + 1] - bs);
            },
            [&](int64_t q) { return B.col[q]; },
            [&](int32_t, int32_t j) {
                uint32_t h = hash_slot(j, SW_LOG2);
                while (true) {  // ends: the set is at most 3/8 full
                    const int32_t old = atomicCAS(&T[h], EMPTY_KEY, j);
                    if (old == EMPTY_KEY) {
                        ++mine;
                        break;
                    }
                    if (old == j) break;
                    h = (h + 1) & (SW_SLOTS - 1);
                }
            });
        const int32_t tot = wave_reduce_add(mine);
        if (lane == 0) cnt[i] = tot;
        wave_lds_sync();  // the set is read before the next row clears it
    }
}

// Dynamic LDS: `nwords` 32-bit bitmap words covering columns [0, n).  Bits
// are set without reading them back; the count is the popcount at the end.
// The finished bitmap is the row's stored set; it is written to bm_save
// (slot = position in the bin list, recorded in heavy_idx) so the numeric
// pass can place values by rank without gathering the columns again.
// When n exceeds 32*nwords columns the row is counted in column blocks of
// that width, each block gathering all of the row's products and keeping
// those inside it; bitmaps are saved only in the single-block case.
template <int NT, int GM>
__global__ void __launch_bounds__(NT) k_sym_bitmap(Csr A, Csr B, BinRef ref,
                                                   const int64_t* a_beg, const int64_t* a_end,
                                                   int64_t* cnt, int32_t nwords, uint32_t* bm_save,
                                                   int32_t* heavy_idx, int32_t* chunk_save,
                                                   int32_t chunk_words, int32_t nchunks, int64_t slots) {
    extern __shared__ uint32_t bm[];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    __shared__ int32_t s_chunk[MAX_CHUNKS];
    const int64_t block_cols = (int64_t)nwords * 32;
    // r: the row's position in the bin list, also its slot among the saved bitmaps
    for_each_bin_row(ref, [&](int64_t r, int64_t i) {
    if (B.ncols > block_cols) {
        int64_t total = 0;
        for (int64_t cb = 0; cb < B.ncols; cb += block_cols) {
            for (int t = threadIdx.x; t < nwords; t += NT) bm[t] = 0u;
            __syncthreads();
            // each B row restricted to the block's columns by binary search:
            // a block gathers only its own products, and a segment never
            // exceeds block_cols entries (the batch sums stay in int32)
            for_each_product_gm<NT, GM>(
                a_beg[i], a_end[i], L,
                [&](int64_t p, int64_t& bs, int32_t& len) {
                    const int64_t k = A.col[p];
                    const int64_t rs = B.rp[k], re = B.rp[k + 1];
                    const int64_t lo = lower_bound_col(B.col, rs, re, cb);
                    const int64_t hi = lower_bound_col(B.col, lo, re, cb + block_cols);
                    bs = lo;
                    len = (int32_t)(hi - lo);
                },
                [&](int, int64_t) {},
                [&](int64_t q) { return (int64_t)B.col[q]; },
                [&](int, int64_t j) {
                    const int64_t jj = j - cb;
                    atomicOr(&bm[jj >> 5], 1u << (jj & 31));
                });
            int32_t mine = 0;
            for (int t = threadIdx.x; t < nwords; t += NT) mine += __popc(bm[t]);
            total += block_reduce_add<NT, int32_t>(mine, red);
        }
        if (threadIdx.x == 0) cnt[i] = total;
        return;
    }
    for (int t = threadIdx.x; t < nwords; t += NT) bm[t] = 0u;
    for (int t = threadIdx.x; t < MAX_CHUNKS; t += NT) s_chunk[t] = 0;
    __syncthreads();
    for_each_product_gm<NT, GM>(
        a_beg[i], a_end[i], L,
        [&](int64_t p, int64_t& bs, int32_t& len) {
            int64_t k = A.col[p];
            bs = B.rp[k];
            len = (int32_t)(B.rp[k + 1] - bs);
        },
        [&](int, int64_t) {},
        [&](int64_t q) { return (uint32_t)B.col[q]; },
        [&](int, uint32_t j) { atomicOr(&bm[j >> 5], 1u << (j & 31)); });
    int32_t mine = 0;
    // rows past the allocated slots are counted but not saved
    const bool keep = r < slots;
    uint32_t* dst = bm_save && keep ? bm_save + r * nwords : nullptr;
    // a wave's 64 consecutive words lie in one chunk (chunk_words is a
    // multiple of 64): the wave sums its counts and adds them once
    for (int t0 = threadIdx.x - lane_id(); t0 < nwords; t0 += NT) {
        const int t = t0 + lane_id();
        const uint32_t w = t < nwords ? bm[t] : 0u;
        const int pc = __popc(w);
        mine += pc;
        if (dst && t < nwords) dst[t] = w;
        if (chunk_save && keep) {
            const int cs = wave_reduce_add(pc);
            if (lane_id() == 0 && cs) atomicAdd(&s_chunk[t0 / chunk_words], cs);
        }
    }
    int32_t total = block_reduce_add<NT, int32_t>(mine, red);  // barriers: s_chunk complete
    if (threadIdx.x == 0) {
        cnt[i] = total;
        if (heavy_idx) heavy_idx[i] = keep ? (int32_t)r : -1;
    }
    if (chunk_save && keep)
        for (int c = threadIdx.x; c < nchunks; c += NT) chunk_save[r * nchunks + c] = s_chunk[c];
    });
}

}  // namespace spg
