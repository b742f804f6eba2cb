// Multiway merge with reduction (Section 4.3; LocalMerge of Algorithm 2):
// out = entry-wise semiring sum of c layers of equal shape.  Row i of the
// output is the sorted union of the c sorted segments layer_l(i,:), with
// values of equal columns combined in ascending layer order.  The paper
// merges with a heap per thread over a split of the column range; here:
//   SORT   (more than 8 layers) rows of 65 ... MS_LMAX entries whose columns
//          span less than 2^(32 - MS_XBITS): one wave per row; every entry
//          becomes a 32-bit key (column - min, then its index in the
//          layer-major order), the keys go to 64 column buckets (one per
//          lane) and each lane sorts its bucket in registers; equal columns
//          are then adjacent in ascending layer order
//   WAVE   rows of at most KW_LMAX entries over at most 8 layers: one
//          wave per row, the column range split over the 64 lanes and each
//          lane merging its range of the c segments (kway.hpp), staged in LDS
//   SMALL  (more layers than the wave merge takes) rows of <= 64 entries:
//          a wave sort of (column, position)
//   RANK   65 ... 4096 entries: a workgroup places each entry by binary
//          searches in the other layers' segments, staged in LDS
//   DENSE  longer rows: a workgroup sweeping column chunks with an LDS dense
//          accumulator, each layer's chunk range found by binary search (the
//          column-range split of Section 4.3)
#pragma once
#include "kway.hpp"
#include "products.hpp"
#include "rowinfo.hpp"

namespace spg {

struct LayerDesc {
    const int64_t* rp;
    const int32_t* col;
    const void* val;
};

constexpr int MERGE_MAX_LAYERS = 64;

// The layers, passed by value as a kernel argument (no device copy).
struct LayerSet {
    LayerDesc d[MERGE_MAX_LAYERS];
};

// merge bins by total row length L over the layers
constexpr int MBIN_EMPTY = 0, MBIN_WAVE = 1, MBIN_SMALL = 2, MBIN_R256 = 3, MBIN_R1K = 4, MBIN_R4K = 5,
              MBIN_DENSE = 6, MBIN_SORT = 7;
constexpr int MBINS = 8;

// the bucket-sort bin: entries per row, bits of a staged index, column span
constexpr int MS_LMAX = 512;
constexpr int MS_XBITS = 9;
constexpr int64_t MS_SPAN_MAX = 1ll << (32 - MS_XBITS);
static_assert((MS_LMAX & (MS_LMAX - 1)) == 0 && MS_LMAX <= (1 << MS_XBITS),
              "the whole-row sort pads to a power of two inside the key array");
constexpr int MERGE_LDS_MAX = 4096;

// The wave k-way merge costs O(c) instructions per output (the smallest of c
// heads each step): it wins for few layers (with 4 layers it is 1.6 times
// as fast as the bucket sort); more layers take the bucket sort and rank
// paths.
constexpr int MERGE_KWAY_MAX_LAYERS = 8;

__device__ inline int merge_bin(int64_t L, int c) {
    if (L == 0) return MBIN_EMPTY;
    if (L <= KW_LMAX && c <= MERGE_KWAY_MAX_LAYERS) return MBIN_WAVE;
    if (L <= SPG_WAVE) return MBIN_SMALL;
    if (L <= 256) return MBIN_R256;
    if (L <= 1024) return MBIN_R1K;
    if (L <= MERGE_LDS_MAX) return MBIN_R4K;
    return MBIN_DENSE;
}

__global__ void __launch_bounds__(256) k_merge_rowinfo(int64_t m, int32_t c, LayerSet layers,
                                                       int64_t* total_len, uint8_t* bin,
                                                       int64_t* bin_stats) {
    __shared__ int s_hist[NBINS];
    __shared__ int64_t s_len[NBINS];
    if (threadIdx.x < NBINS) {
        s_hist[threadIdx.x] = 0;
        s_len[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        int64_t L = 0;
        for (int l = 0; l < c; ++l) L += layers.d[l].rp[i + 1] - layers.d[l].rp[i];
        total_len[i] = L;
        int b = merge_bin(L, c);
        if (c > MERGE_KWAY_MAX_LAYERS && L > SPG_WAVE && L <= MS_LMAX) {  // the bucket sort, if the columns pack
            int32_t mn = 0x7fffffff, mx = -1;
            for (int l = 0; l < c; ++l) {
                const int64_t rs = layers.d[l].rp[i], re = layers.d[l].rp[i + 1];
                if (re > rs) {
                    const int32_t a = layers.d[l].col[rs], z = layers.d[l].col[re - 1];
                    mn = a < mn ? a : mn;
                    mx = z > mx ? z : mx;
                }
            }
            if ((int64_t)mx - mn < MS_SPAN_MAX) b = MBIN_SORT;
        }
        bin[i] = (uint8_t)b;
        atomicAdd(&s_hist[b], 1);
        atomicAdd((unsigned long long*)&s_len[b], (unsigned long long)L);
    }
    __syncthreads();
    if (threadIdx.x < NBINS && s_hist[threadIdx.x]) {
        atomicAdd((unsigned long long*)&bin_stats[threadIdx.x], (unsigned long long)s_hist[threadIdx.x]);
        atomicAdd((unsigned long long*)&bin_stats[NBINS + threadIdx.x], (unsigned long long)s_len[threadIdx.x]);
    }
}

// One wave per row (4 per workgroup), the rows of the bin located on the
// device.  cnt != nullptr: count pass; otherwise fill pass at out_rp.
template <int SR, int KMAX, bool FILL>
__global__ void __launch_bounds__(256) k_merge_kway(int32_t c, LayerSet layers, BinRef ref, int64_t* cnt,
                                                    const int64_t* out_rp, int32_t* out_col, void* out_val) {
    typedef typename Sr<SR>::acc_t V;
    __shared__ KwLds<V, FILL> lds[4];
    KwLds<V, FILL>& W = lds[threadIdx.x >> 6];
    const int32_t* rows;
    int64_t n;
    ref.locate(rows, n);
    const int lane = lane_id();
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[r];
        KwList<V> lst{nullptr, nullptr, 0, 0, Sr<SR>::zero()};
        if (lane < c) {
            const int64_t rs = layers.d[lane].rp[i];
            lst.colp = layers.d[lane].col;
            lst.valp = layers.d[lane].val;
            lst.start = rs;
            lst.len = (int32_t)(layers.d[lane].rp[i + 1] - rs);
        }
        const int32_t L = wave_reduce_add(lst.len);
        const int32_t got = kway_merge_wave<SR, KMAX, FILL, false>(lst, c, L, W, out_col, out_val,
                                                                   FILL ? out_rp[i] : 0);
        if (!FILL && lane == 0) cnt[i] = got;
        wave_lds_sync();  // the staged row is read before the next one overwrites it
    }
}

// Count pass of the WAVE and SORT bins (rows of at most MS_LMAX entries):
// counting needs no order, so the row's columns are inserted into an LDS
// hash set of MC_SLOTS slots (at most half full), one wave per row, and
// each new column counts once.  Every lane then clears the slots it
// filled, so the set is empty again for the wave's next row.
constexpr int MC_LOG2 = 10;
constexpr int MC_SLOTS = 1 << MC_LOG2;
static_assert(MC_SLOTS >= 2 * MS_LMAX && MS_LMAX >= KW_LMAX, "the hash count takes both bins' rows");

__global__ void __launch_bounds__(256) k_merge_count_hash(int32_t c, LayerSet layers, BinRef ref, int64_t* cnt) {
    constexpr int NU = MS_LMAX / SPG_WAVE;
    __shared__ int32_t tab[4][MC_SLOTS];
    int32_t* T = tab[threadIdx.x >> 6];
    const int lane = lane_id();
    for (int t = lane; t < MC_SLOTS; t += SPG_WAVE) T[t] = -1;
    wave_lds_sync();
    const int32_t* rows;
    int64_t n;
    ref.locate(rows, n);
    int top = 1;  // search width over the layers
    while (top < c) top <<= 1;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[r];
        int64_t rs = 0;
        int32_t len = 0;
        const int32_t* colp = nullptr;
        if (lane < c) {
            colp = layers.d[lane].col;
            rs = layers.d[lane].rp[i];
            len = (int32_t)(layers.d[lane].rp[i + 1] - rs);
        }
        const int32_t incl = wave_inclusive_scan_add(len);
        const int32_t soff = incl - len;
        const int32_t L = __builtin_amdgcn_readlane(incl, SPG_WAVE - 1);
        int32_t mine = 0;
        int32_t used[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) used[u] = -1;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            if (u * SPG_WAVE >= L) break;
            const int32_t x = u * SPG_WAVE + lane;
            int l = 0;
            for (int step = top >> 1; step > 0; step >>= 1) {
                const int cand = l + step;
                const int32_t so = __shfl(soff, cand < SPG_WAVE ? cand : SPG_WAVE - 1, SPG_WAVE);
                if (cand < c && so <= x) l = cand;
            }
            const int32_t lo = __shfl(soff, l, SPG_WAVE);
            const int64_t st = __shfl((long long)rs, l, SPG_WAVE);
            const int32_t* cp = (const int32_t*)__shfl((long long)(intptr_t)colp, l, SPG_WAVE);
            if (x < L) {
                const int32_t col = cp[st + (x - lo)];
                uint32_t h = hash_slot(col, MC_LOG2);
                while (true) {  // ends: the set is at most half full
                    const int32_t old = atomicCAS(&T[h], -1, col);
                    if (old == -1) {
                        ++mine;
                        used[u] = (int32_t)h;
                        break;
                    }
                    if (old == col) break;
                    h = (h + 1) & (MC_SLOTS - 1);
                }
            }
        }
        const int32_t tot = wave_reduce_add(mine);
        if (lane == 0) cnt[i] = tot;
        wave_lds_sync();  // every insertion is done before the set is cleared
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (used[u] >= 0) T[used[u]] = -1;
        wave_lds_sync();
    }
}

// Per-wave LDS of the bucket-sort merge: the row's keys, its values by
// staged index (fill pass), the bucket counters.
template <typename V, bool FILL>
struct MsLds {
    uint32_t key[MS_LMAX];
    V val[FILL ? MS_LMAX : 1];
    int32_t bcnt[SPG_WAVE];
};

// One wave per row of the SORT bin (4 per workgroup).  Entry x of the flat
// order (layer 0's segment, then layer 1's, ...) gets the key
// (column - cmin) << MS_XBITS | x, so keys order by column and equal columns
// by layer.  The keys are counted into 64 buckets of equal column width
// (bucket = (column - cmin) * 64 / span in FP32, monotone), placed bucket by
// bucket, and every lane sorts its own bucket with a register network; a
// row whose largest bucket holds more than 16 is sorted whole by the wave
// (a larger network would cost registers, and so waves, on every row).
// Runs of equal columns are then folded in key order.  cnt != nullptr: count
// pass; otherwise fill pass at out_rp.
template <int SR, bool FILL>
__global__ void __launch_bounds__(256) k_merge_sort(int32_t c, LayerSet layers, BinRef ref, int64_t* cnt,
                                                    const int64_t* out_rp, int32_t* out_col, void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    constexpr int NU = MS_LMAX / SPG_WAVE;
    constexpr uint32_t XMASK = (1u << MS_XBITS) - 1;
    __shared__ MsLds<V, FILL> lds[4];
    MsLds<V, FILL>& W = lds[threadIdx.x >> 6];
    const int32_t* rows;
    int64_t n;
    ref.locate(rows, n);
    const int lane = lane_id();
    int top = 1;  // search width over the layers
    while (top < c) top <<= 1;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[r];
        // lane l < c: layer l's segment, its first and last column
        int64_t rs = 0;
        int32_t len = 0, cmin = 0x7fffffff, cmax = -1;
        const int32_t* colp = nullptr;
        const void* valp = nullptr;
        if (lane < c) {
            colp = layers.d[lane].col;
            valp = layers.d[lane].val;
            rs = layers.d[lane].rp[i];
            len = (int32_t)(layers.d[lane].rp[i + 1] - rs);
            if (len > 0) {
                cmin = colp[rs];
                cmax = colp[rs + len - 1];
            }
        }
        const int32_t incl = wave_inclusive_scan_add(len);
        const int32_t soff = incl - len;
        const int32_t L = __builtin_amdgcn_readlane(incl, SPG_WAVE - 1);
#pragma unroll
        for (int d = SPG_WAVE / 2; d > 0; d >>= 1) {
            const int32_t a = lane_xor(cmin, d), b = lane_xor(cmax, d);
            cmin = a < cmin ? a : cmin;
            cmax = b > cmax ? b : cmax;
        }
        const float bscale = (float)SPG_WAVE / (float)((int64_t)cmax - cmin + 1);
        W.bcnt[lane] = 0;
        wave_lds_sync();
        // stage: entry x = u * 64 + lane lies in the last layer whose
        // segment starts at or before x (empty segments share the start of
        // the next one)
        uint32_t ck[NU];
        int32_t cbs[NU];  // bucket << 16 | place in the bucket
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            if (u * SPG_WAVE >= L) break;
            const int32_t x = u * SPG_WAVE + lane;
            int l = 0;
            for (int step = top >> 1; step > 0; step >>= 1) {
                const int cand = l + step;
                const int32_t so = __shfl(soff, cand < SPG_WAVE ? cand : SPG_WAVE - 1, SPG_WAVE);
                if (cand < c && so <= x) l = cand;
            }
            const int32_t lo = __shfl(soff, l, SPG_WAVE);
            const int64_t st = __shfl((long long)rs, l, SPG_WAVE);
            const int32_t* cp = (const int32_t*)__shfl((long long)(intptr_t)colp, l, SPG_WAVE);
            const void* vp = FILL ? (const void*)__shfl((long long)(intptr_t)valp, l, SPG_WAVE) : nullptr;
            if (x < L) {
                const int64_t q = st + (x - lo);
                const uint32_t rel = (uint32_t)(cp[q] - cmin);
                int32_t b = (int32_t)((float)rel * bscale);
                b = b < SPG_WAVE - 1 ? b : SPG_WAVE - 1;
                ck[u] = (rel << MS_XBITS) | (uint32_t)x;
                cbs[u] = (b << 16) | atomicAdd(&W.bcnt[b], 1);
                if constexpr (FILL) {
                    // no value array: structure-only output (booleans: all true)
                    W.val[x] = (vp || SR == SR_BOOL) ? S::load(vp, q) : S::zero();
                }
            }
        }
        wave_lds_sync();
        const int32_t mycnt = W.bcnt[lane];
        const int32_t bmax = wave_reduce_max(mycnt);
        const int32_t boff = wave_inclusive_scan_add(mycnt) - mycnt;
        wave_lds_sync();  // every lane has read its count
        W.bcnt[lane] = boff;
        wave_lds_sync();
        if (bmax <= 16) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                if (u * SPG_WAVE >= L) break;
                if (u * SPG_WAVE + lane < L) W.key[W.bcnt[cbs[u] >> 16] + (cbs[u] & 0xffff)] = ck[u];
            }
            wave_lds_sync();
            if (bmax <= 8) bucket_sort_net<8>(W.key, boff, mycnt, MS_LMAX);
            else bucket_sort_net<16>(W.key, boff, mycnt, MS_LMAX);
        } else {
            int P = SPG_WAVE;
            while (P < L) P <<= 1;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int32_t x = u * SPG_WAVE + lane;
                if (x < L) W.key[x] = ck[u];
                else if (x < P) W.key[x] = 0xffffffffu;
            }
            wave_lds_sync();
            wave_lds_bitonic_u32(W.key, P);
        }
        wave_lds_sync();
        // runs of equal columns: each lane takes a contiguous range of
        // sorted positions and owns the runs that start there
        const int per = (L + SPG_WAVE - 1) / SPG_WAVE;
        const int q0 = lane * per < L ? lane * per : L;
        const int q1 = q0 + per < L ? q0 + per : L;
        int32_t heads = 0;
        for (int q = q0; q < q1; ++q) heads += (q == 0 || (W.key[q] >> MS_XBITS) != (W.key[q - 1] >> MS_XBITS)) ? 1 : 0;
        if constexpr (!FILL) {
            const int32_t tot = wave_reduce_add(heads);
            if (lane == 0) cnt[i] = tot;
        } else {
            int64_t o = out_rp[i] + (wave_inclusive_scan_add(heads) - heads);
            for (int q = q0; q < q1; ++q) {
                const uint32_t kq = W.key[q];
                if (q == 0 || (kq >> MS_XBITS) != (W.key[q - 1] >> MS_XBITS)) {
                    V acc = W.val[kq & XMASK];
                    for (int y = q + 1; y < L && (W.key[y] >> MS_XBITS) == (kq >> MS_XBITS); ++y)
                        acc = S::add(acc, W.val[W.key[y] & XMASK]);
                    out_col[o] = cmin + (int32_t)(kq >> MS_XBITS);
                    if (out_val) S::store(out_val, o, acc);
                    ++o;
                }
            }
        }
        wave_lds_sync();  // the row's LDS is read before the next row overwrites it
    }
}

// cnt != nullptr: count pass; otherwise fill pass into out_rp/out_col/out_val.
template <int SR>
__global__ void __launch_bounds__(256) k_merge_small(int32_t c, LayerSet layers_, BinRef ref, int64_t* cnt,
                                                     const int64_t* out_rp, int32_t* out_col,
                                                     void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    const LayerDesc* layers = layers_.d;
    const int32_t* rows;
    int64_t nrows;
    ref.locate(rows, nrows);
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nrows; r += (int64_t)gridDim.x * 4) {
    const int64_t i = rows[r];
    const int lane = lane_id();
    int pos = 0, my_l = -1;
    int64_t my_q = 0;
    for (int l = 0; l < c; ++l) {
        const int64_t rs = layers[l].rp[i];
        const int len = (int)(layers[l].rp[i + 1] - rs);
        if (lane >= pos && lane < pos + len) {
            my_l = l;
            my_q = rs + (lane - pos);
        }
        pos += len;
    }
    uint64_t key = ~0ull;
    V v = S::zero();
    if (my_l >= 0) {
        key = ((uint64_t)(uint32_t)layers[my_l].col[my_q] << 6) | (uint64_t)lane;
        if (!cnt) v = S::load(layers[my_l].val, my_q);
    }
    key = wave_bitonic_sort_u64(key);
    const bool valid = key != ~0ull;
    const uint64_t col = key >> 6;
    const uint64_t prev = lane_prev(col);
    const bool head = valid && (lane == 0 || prev != col);
    const uint64_t heads = __ballot(head);
    if (cnt) {
        if (lane == 0) cnt[i] = __popcll(heads);
        continue;
    }
    v = __shfl(v, (int)(key & 63), SPG_WAVE);
    V acc = v;
    bool open = head;
    uint64_t ncol = col;
    V nv = v;
    int nvalid = valid ? 1 : 0;
    for (int s = 1; s < SPG_WAVE; ++s) {  // entry s lanes above, one lane per step
        if (!__any(open)) break;
        ncol = lane_next(ncol);
        nv = lane_next(nv);
        nvalid = lane_next(nvalid);
        open = open && (lane + s < SPG_WAVE) && nvalid != 0 && ncol == col;
        if (open) acc = S::add(acc, nv);
    }
    if (head) {
        const int64_t o = out_rp[i] + lanes_below(heads);
        out_col[o] = (int32_t)col;
        if (out_val) S::store(out_val, o, acc);
    }
    }
}

// first index in [lo, hi) of the sorted s with s[idx] >= x (lower) or > x (upper)
__device__ inline int seg_lower(const int32_t* s, int lo, int hi, int32_t x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ inline int seg_upper(const int32_t* s, int lo, int hi, int32_t x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// layer of staged entry x: largest l < c with soff[l] <= x
__device__ inline int layer_of(const int32_t* soff, int c, int x) {
    int lo = 0, hi = c;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (soff[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// One workgroup per row of 65..cap entries.  The row's c segments are
// staged back to back in LDS (scol).  Count pass: an entry opens a new
// column unless an earlier layer holds the same column.  Fill pass: the
// entry's place in the merged order is its index in its own segment plus,
// for every other layer, the entries of that layer with smaller columns
// (and, for earlier layers, equal ones), so equal columns end up adjacent in
// ascending layer order; the runs are then folded left to right.
// Dynamic LDS: cap values (fill pass), cap staged columns, cap merged
// columns (fill pass).
template <int SR, int NT>
__global__ void __launch_bounds__(NT) k_merge_rank(int32_t c, LayerSet layers_, BinRef ref,
                                                   const int64_t* total_len, int32_t cap, int64_t* cnt,
                                                   const int64_t* out_rp, int32_t* out_col, void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    const LayerDesc* layers = layers_.d;
    extern __shared__ uint64_t dyn[];
    V* mval = reinterpret_cast<V*>(dyn);
    int32_t* scol = cnt ? reinterpret_cast<int32_t*>(dyn) : reinterpret_cast<int32_t*>(mval + cap);
    int32_t* mcol = scol + cap;
    __shared__ int32_t soff[MERGE_MAX_LAYERS + 1];
    __shared__ int64_t srs[MERGE_MAX_LAYERS];
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    for_each_bin_row(ref, [&](int64_t, int64_t i) {
    const int L = (int)total_len[i];
    if (threadIdx.x < SPG_WAVE) {  // c <= 64 segment lengths, scanned by one wave
        const int l = threadIdx.x;
        int len = 0;
        if (l < c) {
            const int64_t rs = layers[l].rp[i];
            len = (int)(layers[l].rp[i + 1] - rs);
            srs[l] = rs;
        }
        const int incl = wave_inclusive_scan_add(len);
        if (l < c) soff[l + 1] = incl;
        if (l == 0) soff[0] = 0;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < L; x += NT) {
        const int l = layer_of(soff, c, x);
        scol[x] = layers[l].col[srs[l] + (x - soff[l])];
    }
    __syncthreads();
    if (cnt) {
        int32_t mine = 0;
        for (int x = threadIdx.x; x < L; x += NT) {
            const int l = layer_of(soff, c, x);
            const int32_t col = scol[x];
            bool fresh = true;
            for (int l2 = 0; l2 < l && fresh; ++l2) {
                const int q = seg_lower(scol, soff[l2], soff[l2 + 1], col);
                fresh = !(q < soff[l2 + 1] && scol[q] == col);
            }
            mine += fresh ? 1 : 0;
        }
        const int32_t tot = block_reduce_add<NT, int32_t>(mine, red);
        if (threadIdx.x == 0) cnt[i] = tot;
        return;
    }
    for (int x = threadIdx.x; x < L; x += NT) {
        const int l = layer_of(soff, c, x);
        const int32_t col = scol[x];
        int pos = x - soff[l];
        for (int l2 = 0; l2 < c; ++l2) {
            if (l2 == l) continue;
            const int lo = soff[l2], hi = soff[l2 + 1];
            pos += (l2 < l ? seg_upper(scol, lo, hi, col) : seg_lower(scol, lo, hi, col)) - lo;
        }
        mcol[pos] = col;
        if (out_val) mval[pos] = S::load(layers[l].val, srs[l] + (x - soff[l]));
    }
    __syncthreads();
    // heads over a contiguous range of merged positions per thread
    const int per = (L + NT - 1) / NT;
    const int q0 = threadIdx.x * per;
    const int q1 = q0 + per < L ? q0 + per : L;
    int32_t mine = 0;
    for (int q = q0; q < q1; ++q) mine += (q == 0 || mcol[q - 1] != mcol[q]) ? 1 : 0;
    int32_t total;
    int32_t rank = block_exclusive_scan<NT, int32_t>(mine, &total, red);
    const int64_t o = out_rp[i];
    for (int q = q0; q < q1; ++q) {
        if (q == 0 || mcol[q - 1] != mcol[q]) {
            const int32_t col = mcol[q];
            out_col[o + rank] = col;
            if (out_val) {
                V acc = mval[q];
                for (int y = q + 1; y < L && mcol[y] == col; ++y) acc = S::add(acc, mval[y]);
                S::store(out_val, o + rank, acc);
            }
            ++rank;
        }
    }
    });
}

// Rows above the rank path: a workgroup sweeps column chunks of W; within a
// chunk the layers are added one after the other (a layer holds a column
// at most once, so its entries go to distinct accumulators without atomics,
// and a barrier orders the layers), so equal columns combine in ascending
// layer order.  Each layer's chunk range is found by binary search (the
// column-range split of Section 4.3).
template <int SR, int NT, int W>
__global__ void __launch_bounds__(NT) k_merge_dense(int32_t c, LayerSet layers_, BinRef ref, int64_t ncols, int64_t* cnt,
                                                    const int64_t* out_rp, int32_t* out_col,
                                                    void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    constexpr int NWD = W / 32;
    const LayerDesc* layers = layers_.d;
    __shared__ V acc[W];
    __shared__ uint32_t bits[NWD];
    __shared__ int32_t wpre[NWD];
    __shared__ int64_t s_lo[MERGE_MAX_LAYERS], s_hi[MERGE_MAX_LAYERS];
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    const int P = (int)((ncols + W - 1) / W);
    for_each_bin_row(ref, [&](int64_t, int64_t i) {
    int64_t off = cnt ? 0 : out_rp[i];
    int64_t count = 0;
    for (int ch = 0; ch < P; ++ch) {
        for (int t = threadIdx.x; t < W; t += NT) acc[t] = S::zero();
        for (int t = threadIdx.x; t < NWD; t += NT) bits[t] = 0u;
        const int64_t cbase = (int64_t)ch * W;
        if (threadIdx.x < c) {  // each layer's entries inside the chunk
            const int l = threadIdx.x;
            const int64_t rs = layers[l].rp[i], re = layers[l].rp[i + 1];
            const int64_t lo = lower_bound_col(layers[l].col, rs, re, cbase);
            s_lo[l] = lo;
            s_hi[l] = lower_bound_col(layers[l].col, lo, re, cbase + W);
        }
        __syncthreads();
        for (int l = 0; l < c; ++l) {
            for (int64_t q = s_lo[l] + threadIdx.x; q < s_hi[l]; q += NT) {
                const int32_t j = (int32_t)(layers[l].col[q] - cbase);
                const uint32_t b = 1u << (j & 31);
                if (!cnt) {
                    const V v = S::load(layers[l].val, q);
                    acc[j] = (bits[j >> 5] & b) ? S::add(acc[j], v) : v;
                }
                atomicOr(&bits[j >> 5], b);
            }
            __syncthreads();  // layer l complete before layer l + 1
        }
        constexpr int WPT = (NWD + NT - 1) / NT;
        int32_t wc[WPT];
        int32_t sum = 0;
#pragma unroll
        for (int x = 0; x < WPT; ++x) {
            int w = threadIdx.x * WPT + x;
            wc[x] = w < NWD ? __popc(bits[w]) : 0;
            sum += wc[x];
        }
        int32_t chunk_total;
        int32_t pre = block_exclusive_scan<NT, int32_t>(sum, &chunk_total, red);
#pragma unroll
        for (int x = 0; x < WPT; ++x) {
            int w = threadIdx.x * WPT + x;
            if (w < NWD) wpre[w] = pre;
            pre += wc[x];
        }
        __syncthreads();
        if (!cnt && chunk_total) {
            for (int j = threadIdx.x; j < W; j += NT) {
                const uint32_t wbits = bits[j >> 5];
                const uint32_t b = 1u << (j & 31);
                if (wbits & b) {
                    const int64_t o = off + wpre[j >> 5] + __popc(wbits & (b - 1));
                    out_col[o] = (int32_t)(cbase + j);
                    if (out_val) S::store(out_val, o, acc[j]);
                }
            }
        }
        off += chunk_total;
        count += chunk_total;
        __syncthreads();
    }
    if (cnt && threadIdx.x == 0) cnt[i] = count;
    });
}

}  // namespace spg
