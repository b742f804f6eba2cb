// Numeric phase: C(i,j) = (+)-sum over stored A(i,k), k in window, of
// A(i,k) (x) B(k,j), written as canonical CSR rows sorted by column
// (Section 5.1.1) at the offsets the symbolic phase produced.  Bins:
//   TINY   one A entry: C(i,:) = a (x) B(k,:), already sorted (no accumulator)
//   SMALL  <= 64 products: one wave per row; products sorted across the wave
//          by (column, product order), equal columns folded left to right,
//          which is ascending k (the order of Algorithm 1)
//   HASH   workgroup per row: LDS open-addressing table sized >= 4/3 slots per
//          output, semiring add by LDS atomics, then compaction and an LDS
//          bitonic sort by column
//   RANK   rows whose symbolic pass kept an n-bit bitmap: the bitmap is
//          reloaded, each word gets the count of set bits before it, c_col is
//          written straight from the bitmap, and values accumulate in LDS at
//          index rank(j) = set bits below column j, i.e. directly in output
//          order (a sparse accumulator compressed to the row's own columns)
//   DENSE  workgroup per row sweeping column chunks of W: an LDS dense
//          accumulator plus occupancy bitmap per chunk (the sparse
//          accumulator of Section 3, blocked by columns so it fits LDS);
//          the bitmap scan emits columns in order, so no sort is needed.
#pragma once
#include "products.hpp"
#include "rowinfo.hpp"
#include "symbolic.hpp"

namespace spg {

template <typename V>
struct BEntry {
    int32_t col;
    V val;
};

// Where a row's output goes: its count is rp[i+1] - rp[i]; it starts at
// pos[i] when pos is given (rows of a gathered sub-product written straight
// into the full product), else at rp[i].
struct OutRows {
    const int64_t* rp;
    const int64_t* pos;
    __host__ __device__ OutRows(const int64_t* r, const int64_t* p = nullptr) : rp(r), pos(p) {}
    __device__ int64_t off(int64_t i) const { return pos ? pos[i] : rp[i]; }
    __device__ int64_t count(int64_t i) const { return rp[i + 1] - rp[i]; }
};

// Rows of one A entry in the window: C(i,:) = a * B(k,:), a copy.  Each row
// takes G lanes (256 / G rows per workgroup): with G = 16 a wave keeps the
// dependent loads (row, A entry, B row extent) of four rows in flight, for
// bins whose B rows are short (most lanes of a whole wave would idle); G =
// 64 (a wave per row) for long B rows (R-MAT hubs), where 16 lanes would
// need four times the steps.
template <int SR, int G>
__global__ void __launch_bounds__(256) k_num_tiny(Csr A, Csr B, const int32_t* rows, int32_t nrows,
                                                  const int64_t* a_beg, OutRows c_rp,
                                                  int32_t* c_col, void* c_val) {
    typedef Sr<SR> S;
    static_assert(G == 16 || G == 32 || G == 64, "lanes per row");
    const int r = blockIdx.x * (256 / G) + (int)(threadIdx.x / G);
    if (r >= nrows) return;  // no barriers below
    const int g = (int)(threadIdx.x % G);
    const int64_t i = rows[r];
    const int64_t p = a_beg[i];
    const int64_t k = A.col[p];
    const typename S::acc_t a = S::load(A.val, p);
    const int64_t bs = B.rp[k], be = B.rp[k + 1];
    const int64_t off = c_rp.off(i) - bs;
    // four strides of the row loaded before any is stored, so the loads of
    // a long B row overlap instead of waiting one stride at a time
    constexpr int U = 4;
    for (int64_t q0 = bs; q0 < be; q0 += U * G) {
        int32_t cc[U];
        typename S::acc_t vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + u * G + g;
            cc[u] = 0;
            vv[u] = S::zero();
            if (q < be) {
                cc[u] = B.col[q];
                if (c_val) vv[u] = S::load(B.val, q);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + u * G + g;
            if (q < be) {
                c_col[off + q] = cc[u];
                if (c_val) S::store(c_val, off + q, S::mul(a, vv[u]));
            }
        }
    }
}

// cnt_out (optional) receives each row's output count.  4 waves per block,
// SMALL_ROWS rows per wave (their loads in flight together).
template <int SR>
__global__ void __launch_bounds__(256) k_num_small(Csr A, Csr B, const int32_t* rows, int32_t nrows,
                                                   const int64_t* a_beg, const int64_t* a_end,
                                                   OutRows c_rp, int32_t* c_col, void* c_val,
                                                   int64_t* cnt_out) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w * SMALL_ROWS >= nrows) return;  // whole wave leaves; no block barriers below
    const int lane = lane_id();
    V vals[SMALL_ROWS];
    uint64_t keys[SMALL_ROWS];
    int64_t row[SMALL_ROWS];
    for_small_rows(A, B, rows, nrows, w, a_beg, a_end, [&](int u, int64_t i, bool have, int64_t p, int64_t q) {
        row[u] = i;
        vals[u] = S::zero();
        keys[u] = ~0ull;
        if (have) {
            vals[u] = S::mul(S::load(A.val, p), S::load(B.val, q));
            keys[u] = ((uint64_t)(uint32_t)B.col[q] << 6) | (uint64_t)lane;  // (column, product order)
        }
    });
#pragma unroll
    for (int u = 0; u < SMALL_ROWS; ++u) {
        if (w * SMALL_ROWS + u >= nrows) break;
        const int64_t i = row[u];
        // (column, lane) fits 32 bits below 2^26 - 1 columns (the all-ones
        // key stays the empty lane's): the cheaper 32-bit sort
        uint64_t key;
        if (B.ncols < (1ll << 26) - 1) {
            const uint32_t k32 = wave_bitonic_sort_u32((uint32_t)keys[u]);
            key = k32 == 0xffffffffu ? ~0ull : (uint64_t)k32;
        } else {
            key = wave_bitonic_sort_u64(keys[u]);
        }
        const bool valid = key != ~0ull;
        const V v = __shfl(vals[u], (int)(key & 63), SPG_WAVE);  // value travels with its key
        const uint64_t col = key >> 6;
        const uint64_t prev = lane_prev(col);
        const bool head = valid && (lane == 0 || prev != col);
        // fold the run that starts at each head, left to right: at step s
        // every lane holds the entry s lanes above it (shifted one lane per step)
        V acc = v;
        bool open = head;
        uint64_t ncol = col;
        V nv = v;
        int nvalid = valid ? 1 : 0;
        for (int s = 1; s < SPG_WAVE; ++s) {
            if (!__any(open)) break;
            ncol = lane_next(ncol);
            nv = lane_next(nv);
            nvalid = lane_next(nvalid);
            open = open && (lane + s < SPG_WAVE) && nvalid != 0 && ncol == col;
            if (open) acc = S::add(acc, nv);
        }
        const uint64_t heads = __ballot(head);
        if (head) {
            const int64_t o = c_rp.off(i) + lanes_below(heads);
            c_col[o] = (int32_t)col;
            if (c_val) S::store(c_val, o, acc);
        }
        if (cnt_out && lane == 0) cnt_out[i] = __popcll(heads);
    }
}

// cnt_out (optional) receives each row's output count; a count above the
// slot c_rp.count(i) means the slot overflowed (only then is the output
// incomplete).
template <int SR, int NT, int LOG2T>
__global__ void __launch_bounds__(NT) k_num_hash(Csr A, Csr B, const int32_t* rows,
                                                 const int64_t* a_beg, const int64_t* a_end,
                                                 OutRows c_rp, int32_t* c_col, void* c_val,
                                                 int64_t* cnt_out) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    constexpr int T = 1 << LOG2T;
    constexpr int PER = T / NT;  // table slots owned by a thread during compaction
    static_assert(PER >= 1, "table smaller than block");
    __shared__ int32_t tkey[T];
    // 8 bytes a slot whatever the value type: the full sort below keeps up
    // to T keys of 8 bytes there
    __shared__ uint64_t tval_store[T];
    V* tval = reinterpret_cast<V*>(tval_store);
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    __shared__ int32_t mm[2 * (NT / SPG_WAVE)];
    __shared__ V s_av[NT];
    __shared__ int32_t s_bucket[NT];
    const int64_t i = rows[blockIdx.x];
    for (int t = threadIdx.x; t < T; t += NT) {
        tkey[t] = EMPTY_KEY;
        tval[t] = S::zero();
    }
    __syncthreads();
    // the table has >= 4/3 slots per output of the symbolic count, so a
    // probe ends within T steps; the cap only guards inputs that changed
    // between the two phases
    auto insert = [&](int32_t j, V v) {
        uint32_t h = hash_slot(j, LOG2T);
        for (int probes = 0; probes < T; ++probes) {
            int32_t cur = __hip_atomic_load(&tkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur == EMPTY_KEY) {
                int32_t old = atomicCAS(&tkey[h], EMPTY_KEY, j);
                cur = old == EMPTY_KEY ? j : old;
            }
            if (cur == j) {
                S::lds_add(&tval[h], v);
                break;
            }
            h = (h + 1) & (T - 1);
        }
    };
    if constexpr (NT == SPG_WAVE) {
        // one wave: the lane search needs no block-wide enumeration
        wave_products<4, V>(
            a_beg[i], a_end[i],
            [&](int64_t p, int64_t& bs, int32_t& len, V& av) {
                const int64_t k = A.col[p];
                bs = B.rp[k];
                len = (int32_t)(B.rp[k + 1] - bs);
                av = S::load(A.val, p);
            },
            [&](int64_t q) { return BEntry<V>{B.col[q], S::load(B.val, q)}; },
            [&](V av, const BEntry<V>& x) { insert(x.col, S::mul(av, x.val)); });
        __syncthreads();  // every insertion lands before the table is read
    } else {
        for_each_product_u<NT, 4>(
            a_beg[i], a_end[i], L,
            [&](int64_t p, int64_t& bs, int32_t& len) {
                int64_t k = A.col[p];
                bs = B.rp[k];
                len = (int32_t)(B.rp[k + 1] - bs);
            },
            [&](int t, int64_t p) { s_av[t] = S::load(A.val, p); },
            [&](int64_t q) { return BEntry<V>{B.col[q], S::load(B.val, q)}; },
            [&](int t, const BEntry<V>& x) { insert(x.col, S::mul(s_av[t], x.val)); });
    }
    // compaction: slots [t*PER, (t+1)*PER) -> registers
    int32_t rk[PER];
    V rv[PER];
    int32_t mine = 0;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        rk[s] = tkey[threadIdx.x * PER + s];
        rv[s] = tval[threadIdx.x * PER + s];
        mine += rk[s] != EMPTY_KEY;
    }
    __syncthreads();  // every slot is in registers before the table is reused
    int32_t cnt;
    int32_t pos = block_exclusive_scan<NT, int32_t>(mine, &cnt, red);
    const int64_t o = c_rp.off(i);
    const int32_t cnt_sym = (int32_t)c_rp.count(i);
    if (cnt_out && threadIdx.x == 0) cnt_out[i] = cnt;
    if (cnt_out && cnt > cnt_sym) return;  // slot overflow: the row is redone exactly
    // Output order.  When the row's columns span few enough bitmap words, the
    // rank of a column is the popcount of the bitmap below it (prefix of
    // per-word popcounts): no sort.  Otherwise sort (column, slot) keys.
    int32_t kmin = 0x7fffffff, kmax = -1;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        if (rk[s] != EMPTY_KEY) {
            kmin = rk[s] < kmin ? rk[s] : kmin;
            kmax = rk[s] > kmax ? rk[s] : kmax;
        }
    }
    block_min_max<NT, int32_t>(kmin, kmax, mm);
    const int32_t nw = kmax >= kmin ? ((kmax - kmin) >> 5) + 1 : 0;
    if (nw > 0 && nw <= T && nw <= 8 * cnt + 64) {
        uint32_t* bm = reinterpret_cast<uint32_t*>(tkey);
        int32_t* wp = reinterpret_cast<int32_t*>(tval);
        for (int w = threadIdx.x; w < nw; w += NT) bm[w] = 0u;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            if (rk[s] != EMPTY_KEY) {
                const int32_t j = rk[s] - kmin;
                atomicOr(&bm[j >> 5], 1u << (j & 31));
            }
        }
        __syncthreads();
        const int wpt = (nw + NT - 1) / NT;
        const int w0 = threadIdx.x * wpt;
        int32_t part = 0;
        for (int w = w0; w < w0 + wpt && w < nw; ++w) part += __popc(bm[w]);
        int32_t dummy;
        int32_t run = block_exclusive_scan<NT, int32_t>(part, &dummy, red);
        for (int w = w0; w < w0 + wpt && w < nw; ++w) {
            wp[w] = run;
            run += __popc(bm[w]);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            if (rk[s] != EMPTY_KEY) {
                const int32_t j = rk[s] - kmin;
                const int32_t w = j >> 5;
                const int32_t rank = wp[w] + __popc(bm[w] & ((1u << (j & 31)) - 1u));
                if (rank < cnt_sym) {
                    c_col[o + rank] = rk[s];
                    if (c_val) S::store(c_val, o + rank, rv[s]);
                }
            }
        }
        return;
    }
    // Wide spans: NT buckets of (nearly) equal column width, one per thread.
    // The entries are counted per bucket, placed bucket by bucket, and each
    // thread sorts its own bucket (insertion sort); then the row is written in
    // order.  Falls back to the full sort below when some bucket holds more
    // than 32.  The bucket of a column is (column - kmin) * NT / span in FP32,
    // truncated and clamped to NT - 1: every step of that is monotone, so the
    // buckets follow column order, and it costs a multiply where an integer
    // division by the width would cost a few dozen instructions per entry.
    if (cnt <= T) {
        const float bscale = (float)NT / (float)((int64_t)kmax - kmin + 1);
        auto bucket_of = [&](int32_t key) {
            const int32_t b = (int32_t)((float)(uint32_t)(key - kmin) * bscale);
            return b < NT - 1 ? b : NT - 1;
        };
        s_bucket[threadIdx.x] = 0;
        __syncthreads();
        int32_t bl[PER];
#pragma unroll
        for (int s = 0; s < PER; ++s)
            bl[s] = rk[s] != EMPTY_KEY ? atomicAdd(&s_bucket[bucket_of(rk[s])], 1) : 0;
        __syncthreads();
        const int32_t mycnt = s_bucket[threadIdx.x];
        int32_t bmin = mycnt, bmax = mycnt;
        block_min_max<NT, int32_t>(bmin, bmax, mm);
        if (bmax <= 32) {
            int32_t tot;
            const int32_t boff = block_exclusive_scan<NT, int32_t>(mycnt, &tot, red);
            s_bucket[threadIdx.x] = boff;
            __syncthreads();
            const int32_t nout = cnt < cnt_sym ? cnt : cnt_sym;
            // Columns that fit beside a slot index in 32 bits: each entry
            // becomes the key (column - kmin) << LOG2T | slot, the values stay
            // in the table, and every thread sorts its bucket's keys in
            // registers with a sorting network (two instructions per
            // comparator, no LDS round trips).  Buckets of 17 to 32 take a
            // network only in the kernels of 16 slots per thread, where they
            // are common; elsewhere its registers would cost waves.
            constexpr int NET_MAX = PER >= 16 ? 32 : 16;
            if (bmax <= NET_MAX && cnt > 0 && (int64_t)kmax - kmin < (1ll << (32 - LOG2T))) {
#pragma unroll
                for (int s = 0; s < PER; ++s) {
                    if (rk[s] != EMPTY_KEY) {
                        const int32_t q = s_bucket[bucket_of(rk[s])] + bl[s];
                        tkey[q] = (int32_t)(((uint32_t)(rk[s] - kmin) << LOG2T) | (uint32_t)(threadIdx.x * PER + s));
                    }
                }
                __syncthreads();
                uint32_t* pk = reinterpret_cast<uint32_t*>(tkey);
                if (bmax <= 8) bucket_sort_net<8>(pk, boff, mycnt, T);
                else if (NET_MAX == 16 || bmax <= 16) bucket_sort_net<16>(pk, boff, mycnt, T);
                else bucket_sort_net<NET_MAX>(pk, boff, mycnt, T);
                __syncthreads();
                for (int t = threadIdx.x; t < nout; t += NT) {
                    const uint32_t key = (uint32_t)tkey[t];
                    c_col[o + t] = kmin + (int32_t)(key >> LOG2T);
                    if (c_val) S::store(c_val, o + t, tval[key & (T - 1)]);
                }
                return;
            }
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                if (rk[s] != EMPTY_KEY) {
                    const int32_t q = s_bucket[bucket_of(rk[s])] + bl[s];
                    tkey[q] = rk[s];
                    tval[q] = rv[s];
                }
            }
            __syncthreads();
            for (int x = boff + 1; x < boff + mycnt; ++x) {
                const int32_t kx = tkey[x];
                const V vx = tval[x];
                int y = x - 1;
                while (y >= boff && tkey[y] > kx) {
                    tkey[y + 1] = tkey[y];
                    tval[y + 1] = tval[y];
                    --y;
                }
                tkey[y + 1] = kx;
                tval[y + 1] = vx;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < nout; t += NT) {
                c_col[o + t] = tkey[t];
                if (c_val) S::store(c_val, o + t, tval[t]);
            }
            return;
        }
        __syncthreads();
    }
    // Full sort: (column, compact index) keys sorted in the value storage
    // (up to T keys of 8 bytes); the sorted order gives each compact index
    // its rank (in tkey's bytes), and every thread writes its own entries,
    // whose values never left its registers, at their ranks.
    uint64_t* skey = tval_store;
    int32_t* rank_of = tkey;
    int32_t posv[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        posv[s] = -1;
        if (rk[s] != EMPTY_KEY) {
            posv[s] = pos;
            skey[pos] = ((uint64_t)(uint32_t)rk[s] << 32) | (uint64_t)pos;
            ++pos;
        }
    }
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int t = cnt + threadIdx.x; t < P; t += NT) skey[t] = ~0ull;
    __syncthreads();
    block_bitonic_sort_u64<NT>(skey, P);
    for (int t = threadIdx.x; t < cnt; t += NT) rank_of[(int32_t)(skey[t] & 0xffffffffu)] = t;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        if (posv[s] >= 0) {
            const int32_t rank = rank_of[posv[s]];
            if (rank < cnt_sym) {
                c_col[o + rank] = rk[s];
                if (c_val) S::store(c_val, o + rank, rv[s]);
            }
        }
    }
}

// Column split table for the dense sweep: split[k*(P+1)+c] = offset inside
// B(k,:) of the first entry with column >= c*W (c = 0..P).
__global__ void __launch_bounds__(256) k_split_table(Csr B, int32_t W, int32_t P, int32_t* split) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = B.nrows * (int64_t)(P + 1);
    if (idx >= total) return;
    const int64_t k = idx / (P + 1);
    const int c = (int)(idx - k * (P + 1));
    const int64_t rs = B.rp[k], re = B.rp[k + 1];
    int64_t r;
    if (c == 0) r = rs;
    else if (c == P) r = re;
    else r = lower_bound_col(B.col, rs, re, (int64_t)c * W);
    split[idx] = (int32_t)(r - rs);
}

// Rows without a saved bitmap (n above the LDS bitmap): one workgroup per
// row sweeps the P column chunks of W columns in order, accumulating each
// chunk densely in LDS and emitting it in column order.
template <int SR, int NT, int W, int GM>
__global__ void __launch_bounds__(NT) k_num_dense(Csr A, Csr B, const int32_t* rows, int64_t nrows,
                                                  const int64_t* a_beg, const int64_t* a_end,
                                                  const int32_t* split, int32_t P,
                                                  OutRows c_rp, int32_t* c_col, void* c_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    constexpr int NWD = W / 32;
    static_assert(NWD <= NT, "one bitmap word per thread at most");
    __shared__ V acc[W];
    __shared__ uint32_t bits[NWD];
    __shared__ V s_av[NT];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    // the accumulator is cleared once; emission resets exactly the slots it
    // reads, so later chunks (and later work items) start from zero again
    for (int t = threadIdx.x; t < W; t += NT) acc[t] = S::zero();
    for (int t = threadIdx.x; t < NWD; t += NT) bits[t] = 0u;
    // grid-stride over the rows, so the grid stays small
    for (int64_t item = blockIdx.x; item < nrows; item += gridDim.x) {
    const int64_t i = rows[item];
    const int64_t beg = a_beg[i], end = a_end[i];
    int64_t off = c_rp.off(i);
    const int64_t row_end = off + c_rp.count(i);
    const int c_first = 0, c_last = P;
    // Rows with at most NT entries in the window keep their A entry (column
    // k, start of B(k,:), position reached in B(k,:)) in registers across
    // the chunks, so each chunk costs one split-table load per entry.
    const bool single = end - beg <= NT;
    int64_t my_k = 0, my_rs = 0;
    int32_t my_cur = 0;
    if (single && beg + (int64_t)threadIdx.x < end) {
        const int64_t p = beg + threadIdx.x;
        my_k = A.col[p];
        my_rs = B.rp[my_k];
        s_av[threadIdx.x] = S::load(A.val, p);
    }
    __syncthreads();
    for (int c = c_first; c < c_last; ++c) {
        const int32_t cbase = c * W;
        for_each_product_gm<NT, GM>(
            beg, end, L,
            [&](int64_t p, int64_t& bs, int32_t& len) {
                if (single) {
                    const int32_t nxt = P > 1 ? split[my_k * (P + 1) + c + 1] : (int32_t)(B.rp[my_k + 1] - my_rs);
                    bs = my_rs + my_cur;
                    len = nxt - my_cur;
                    my_cur = nxt;
                } else {
                    const int64_t k = A.col[p];
                    const int64_t rs = B.rp[k];
                    if (P > 1) {
                        const int32_t* sp = split + k * (P + 1) + c;
                        bs = rs + sp[0];
                        len = sp[1] - sp[0];
                    } else {
                        bs = rs;
                        len = (int32_t)(B.rp[k + 1] - rs);
                    }
                }
            },
            [&](int t, int64_t p) {
                if (!single) s_av[t] = S::load(A.val, p);
            },
            [&](int64_t q) { return BEntry<V>{B.col[q], S::load(B.val, q)}; },
            [&](int t, const BEntry<V>& x) {
                const int32_t j = x.col - cbase;
                S::lds_add(&acc[j], S::mul(s_av[t], x.val));
                atomicOr(&bits[j >> 5], 1u << (j & 31));
            });
        // thread t owns bitmap word t: prefix of popcounts, then its set bits
        const uint32_t wbits = threadIdx.x < NWD ? bits[threadIdx.x] : 0u;
        int32_t chunk_total;
        int32_t pre = block_exclusive_scan<NT, int32_t>(__popc(wbits), &chunk_total, red);
        if (wbits) {
            int64_t o = off + pre;
            uint32_t wb = wbits;
            while (wb) {
                const int b = __ffs(wb) - 1;
                wb &= wb - 1;
                const int j = threadIdx.x * 32 + b;
                if (o < row_end) {
                    c_col[o] = cbase + j;
                    if (c_val) S::store(c_val, o, acc[j]);
                }
                acc[j] = S::zero();
                ++o;
            }
            bits[threadIdx.x] = 0u;
        }
        off += chunk_total;
        __syncthreads();
    }
    }
}

// Copy nw bitmap words from global memory into the low halves of the LDS
// words bw[] with coalesced loads, the first 8 per thread issued together.
template <int NT>
__device__ inline void stage_bitmap_words(const uint32_t* src, int nw, uint64_t* bw) {
    constexpr int K = 8;
    uint32_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int w = threadIdx.x + k * NT;
        v[k] = w < nw ? src[w] : 0u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int w = threadIdx.x + k * NT;
        if (w < nw) bw[w] = v[k];
    }
    for (int w = threadIdx.x + K * NT; w < nw; w += NT) bw[w] = src[w];
}

// Packs the staged bitmap words (low half: the bits; high half: the number
// of set bits in all earlier words) and writes the column cbase + 32 w + b of
// every set bit, in order, to out[0, cnt).  Each thread scans a contiguous
// run of words and drops its columns into `acc` (LDS, used as int32 staging:
// it holds at least cnt accumulators of 4 or 8 bytes); the block then copies
// them out with consecutive threads on consecutive positions, so the global
// stores are coalesced, and leaves acc[0, cnt) zero.  Contains barriers.
template <int NT, typename V>
__device__ inline void pack_words_write_cols(uint64_t* bw, int nw, int32_t cbase, int32_t cnt, V* acc,
                                             int32_t* out, int32_t* red) {
    int32_t* stage = reinterpret_cast<int32_t*>(acc);
    const int wpt = (nw + NT - 1) / NT;
    const int w0 = threadIdx.x * wpt;
    const int w1 = w0 + wpt < nw ? w0 + wpt : nw;
    int32_t part = 0;
    for (int w = w0; w < w1; ++w) part += __popc((uint32_t)bw[w]);
    int32_t dummy;
    int32_t run = block_exclusive_scan<NT, int32_t>(part, &dummy, red);
    for (int w = w0; w < w1; ++w) {
        uint32_t bits = (uint32_t)bw[w];
        bw[w] = ((uint64_t)(uint32_t)run << 32) | bits;
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            if (run < cnt) stage[run] = cbase + w * 32 + b;
            ++run;
        }
    }
    __syncthreads();
    // accumulator e holds staged positions [K e, K e + K): one thread reads
    // them, stores them and clears the accumulator
    constexpr int K = (int)(sizeof(V) / sizeof(int32_t));
    const int ne = (cnt + K - 1) / K;
    for (int e = threadIdx.x; e < ne; e += NT) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (K * e + k < cnt) out[K * e + k] = stage[K * e + k];
        acc[e] = V(0);
    }
    for (int e = ne + threadIdx.x; e < cnt; e += NT) acc[e] = V(0);
}

// Dynamic LDS: nwords 64-bit words (bits in the low half, count of set bits
// in all earlier words in the high half), then `cap` accumulators.
template <int SR, int NT, int GM>
__global__ void __launch_bounds__(NT) k_num_rank(Csr A, Csr B, const int32_t* rows,
                                                 const int64_t* a_beg, const int64_t* a_end,
                                                 const uint32_t* bm_save, const int32_t* heavy_idx,
                                                 int32_t nwords, OutRows c_rp, int32_t* c_col,
                                                 void* c_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    extern __shared__ uint64_t dyn[];
    uint64_t* bw = dyn;
    V* acc = reinterpret_cast<V*>(dyn + nwords);
    __shared__ V s_av[NT];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    const int64_t i = rows[blockIdx.x];
    const int64_t off = c_rp.off(i);
    const int32_t cnt = (int32_t)c_rp.count(i);
    const uint32_t* src = bm_save + (int64_t)heavy_idx[i] * nwords;
    stage_bitmap_words<NT>(src, nwords, bw);
    __syncthreads();
    pack_words_write_cols<NT>(bw, nwords, 0, cnt, acc, c_col + off, red);
    __syncthreads();
    for_each_product_gm<NT, GM>(
        a_beg[i], a_end[i], L,
        [&](int64_t p, int64_t& bs, int32_t& len) {
            int64_t k = A.col[p];
            bs = B.rp[k];
            len = (int32_t)(B.rp[k + 1] - bs);
        },
        [&](int t, int64_t p) { s_av[t] = S::load(A.val, p); },
        [&](int64_t q) { return BEntry<V>{B.col[q], S::load(B.val, q)}; },
        [&](int t, const BEntry<V>& x) {
            const uint32_t j = (uint32_t)x.col;
            const uint64_t wd = bw[j >> 5];
            const int32_t rank = (int32_t)(wd >> 32) + __popc((uint32_t)wd & ((1u << (j & 31)) - 1u));
            if (rank < cnt) S::lds_add(&acc[rank], S::mul(s_av[t], x.val));
        });
    if (c_val)
        for (int r = threadIdx.x; r < cnt; r += NT) S::store(c_val, off + r, acc[r]);
}

// Rank chunks: the rows of the bitmap pass that are too large for the
// per-row rank kernel.  A row's column chunks of W columns (counts recorded
// by the bitmap pass) are grouped greedily into items of at most RC outputs
// and at most G chunks; an item accumulates in LDS at index = rank inside
// the item, with its B segments taken from the split table.
struct RankItem {
    int32_t r;      // index into the bin's row list
    int32_t c0, c1; // chunk range [c0, c1)
    int32_t cnt;    // outputs of the item
    int64_t roff;   // outputs of the row before the item
};

// Chunks per rank-chunk item: about RC outputs at the bin's mean density
// (cnnz outputs over nr rows of `chunks` chunks), at most chunk_group and
// `chunks`, and no more than the LDS holds (G*W/32 packed words + RC
// values + static_lds <= max_lds).  Integer arithmetic, so the host (sizing
// the launch) and the device (forming the items) agree.
__host__ __device__ inline int32_t rankc_group(int64_t nr, int64_t cnnz, int32_t chunks, int32_t RC, int32_t chunk_group,
                                               int32_t W, int64_t static_lds, int64_t max_lds) {
    int64_t G = cnnz > 0 ? (2 * (int64_t)RC * nr * chunks + cnnz) / (2 * cnnz) : chunks;
    if (G > chunks) G = chunks;
    if (G > chunk_group) G = chunk_group;
    if (G < 1) G = 1;
    while (G > 1 && G * (W / 32) * 8 + (int64_t)RC * 8 + static_lds > max_lds) --G;
    return (int32_t)G;
}

// Work items of the rank-chunk bin, located on the device (counts of the
// numeric classification): each row's chunks grouped greedily into items
// of at most RC outputs and G chunks.
__global__ void __launch_bounds__(256) k_rank_items(BinRef ref, const int32_t* heavy_idx, const int32_t* chunk_cnt,
                                                    int32_t P, int32_t RC, int32_t chunk_group, int32_t W,
                                                    int64_t static_lds, int64_t max_lds, const int64_t* cnnz_of_bin,
                                                    RankItem* items, int32_t* nitems) {
    __shared__ int32_t tmp[256 / SPG_WAVE + 1];
    __shared__ int32_t s_base;
    const int32_t* rows;
    int64_t nrows;
    ref.locate(rows, nrows);
    const int32_t G = rankc_group(nrows, *cnnz_of_bin, P, RC, chunk_group, W, static_lds, max_lds);
    for (int64_t r0 = (int64_t)blockIdx.x * 256; r0 < nrows; r0 += (int64_t)gridDim.x * 256) {
        const int64_t r = r0 + threadIdx.x;
        const int32_t* cc = r < nrows ? chunk_cnt + (int64_t)heavy_idx[rows[r]] * P : nullptr;
        // the greedy grouping of the row's chunks, walked twice: to count the
        // items (one global add per workgroup reserves their slots), then to
        // write them
        auto walk = [&](auto emit) {
            int64_t roff = 0;
            int c0 = 0;
            while (c0 < P) {
                int c1 = c0;
                int32_t n = 0;
                while (c1 < P && c1 - c0 < G && n + cc[c1] <= RC) n += cc[c1++];
                if (c1 == c0) {  // a chunk above RC (the host keeps RC >= W): take it alone, always progress
                    n = cc[c0];
                    c1 = c0 + 1;
                }
                if (n > 0) emit(c0, c1, n, roff);
                roff += n;
                c0 = c1;
            }
        };
        int32_t mine = 0;
        if (cc) walk([&](int, int, int32_t, int64_t) { ++mine; });
        int32_t total;
        int32_t slot = block_exclusive_scan<256, int32_t>(mine, &total, tmp);
        if (threadIdx.x == 0) s_base = total ? atomicAdd(nitems, total) : 0;
        __syncthreads();
        slot += s_base;
        if (cc) walk([&](int c0, int c1, int32_t n, int64_t roff) { items[slot++] = RankItem{(int32_t)r, c0, c1, n, roff}; });
        __syncthreads();
    }
}

// Dynamic LDS: G*W/32 packed words (prefix << 32 | bits), then RC values.
template <int SR, int NT, int GM>
__global__ void __launch_bounds__(NT) k_num_rankc(Csr A, Csr B, int32_t W, const int32_t* rows, const int64_t* a_beg,
                                                  const int64_t* a_end, const uint32_t* bm_save,
                                                  const int32_t* heavy_idx, int32_t nwords, const int32_t* split,
                                                  int32_t P, const RankItem* items, const int32_t* nitems,
                                                  int32_t RC, int32_t G, OutRows c_rp, int32_t* c_col,
                                                  void* c_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    const int WPC = W / 32;  // bitmap words per chunk
    extern __shared__ uint64_t dyn[];
    uint64_t* bw = dyn;
    V* acc = reinterpret_cast<V*>(dyn + (int64_t)G * WPC);
    __shared__ V s_av[NT];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    for (int t = threadIdx.x; t < RC; t += NT) acc[t] = S::zero();
    __syncthreads();
    const int32_t total_items = *nitems;
    for (int32_t it = blockIdx.x; it < total_items; it += gridDim.x) {
        const RankItem item = items[it];
        const int64_t i = rows[item.r];
        const uint32_t* src = bm_save + (int64_t)heavy_idx[i] * nwords + (int64_t)item.c0 * WPC;
        // the last chunk of a row may be partial (n not a multiple of W): the
        // saved bitmap ends at nwords, so stage no word past it (columns of
        // the missing words are >= n and never looked up)
        const int nw_full = (item.c1 - item.c0) * WPC, nw_left = nwords - item.c0 * WPC;
        const int nw = nw_full < nw_left ? nw_full : nw_left;
        const int64_t off = c_rp.off(i) + item.roff;
        const int32_t cbase = item.c0 * W;
        // packed words and columns
        stage_bitmap_words<NT>(src, nw, bw);
        __syncthreads();
        pack_words_write_cols<NT>(bw, nw, cbase, item.cnt < RC ? item.cnt : RC, acc, c_col + off, red);
        __syncthreads();
        const int c0 = item.c0, c1 = item.c1;
        for_each_product_gm<NT, GM>(
            a_beg[i], a_end[i], L,
            [&](int64_t p, int64_t& bs, int32_t& len) {
                const int64_t k = A.col[p];
                const int64_t rs = B.rp[k];
                if (split) {
                    const int32_t* sp = split + k * (P + 1);
                    bs = rs + sp[c0];
                    len = sp[c1] - sp[c0];
                } else {  // one chunk covers all columns: the whole B row (no split table)
                    bs = rs;
                    len = (int32_t)(B.rp[k + 1] - rs);
                }
            },
            [&](int t, int64_t p) { s_av[t] = S::load(A.val, p); },
            [&](int64_t q) { return BEntry<V>{B.col[q], S::load(B.val, q)}; },
            [&](int t, const BEntry<V>& x) {
                const uint32_t j = (uint32_t)(x.col - cbase);
                const uint64_t wd = bw[j >> 5];
                const int32_t rank = (int32_t)(wd >> 32) + __popc((uint32_t)wd & ((1u << (j & 31)) - 1u));
                if (rank < RC) S::lds_add(&acc[rank], S::mul(s_av[t], x.val));
            });
        const int32_t nout = item.cnt < RC ? item.cnt : RC;
        for (int r = threadIdx.x; r < nout; r += NT) {
            if (c_val) S::store(c_val, off + r, acc[r]);
            acc[r] = S::zero();
        }
        __syncthreads();
    }
}

}  // namespace spg
