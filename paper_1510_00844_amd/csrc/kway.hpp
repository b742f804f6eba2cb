// k-way merge of sorted lists by one wave, with the column-range split of
// Section 4.3: the union of a row's k sorted lists (the layer rows of the
// multiway merge, or the B rows B(k,:) of a row of A in HeapSpGEMM, Section
// 4.2) is cut into 64 equal column ranges, one per lane, and every lane
// merges its range of all k lists sequentially, taking the smallest head
// column each step (the heap of HeapSpGEMM, its k heads held in registers).
// Equal columns are combined in ascending list order, so a list order of
// ascending k (or ascending layer) gives exactly the oracle's fold.  The
// output is sorted by construction: no hash table and no sort.
//
// The row's entries are staged in LDS once (coalesced loads, list by list
// in the flat order of a wave scan of the list lengths); each lane then finds
// where its column range starts in every list by a binary search (all lists
// in lockstep, so the searches' LDS reads overlap), and takes the end of its
// range from the next lane's starts.  Count mode runs one sweep (distinct
// columns); fill mode runs a counting sweep, a wave scan for the lanes'
// output offsets, and a second sweep that writes.
#pragma once
#include "common.hpp"

namespace spg {

constexpr int KW_LMAX = 384;  // entries of one row a wave stages
constexpr int KW_KMAX = 32;   // lists of one row
constexpr int32_t KW_INF = 0x7fffffff;

// Per-wave LDS: the staged columns and (fill mode) values of one row.
template <typename V, bool FILL>
struct KwLds {
    int32_t col[KW_LMAX];
    V val[FILL ? KW_LMAX : 1];
};

// Value of lane l (wave-uniform l) of a 64-bit quantity, as a scalar.
__device__ inline int64_t readlane_i64_(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline const void* readlane_ptr(const void* p, int l) {
    return (const void*)(intptr_t)readlane_i64_((int64_t)(intptr_t)p, l);
}
template <typename V>
__device__ inline V readlane_val(V v, int l) {
    if constexpr (sizeof(V) == 8) {
        int64_t u;
        __builtin_memcpy(&u, &v, 8);
        u = readlane_i64_(u, l);
        __builtin_memcpy(&v, &u, 8);
    } else {
        int u;
        __builtin_memcpy(&u, &v, 4);
        u = __builtin_amdgcn_readlane(u, l);
        __builtin_memcpy(&v, &u, 4);
    }
    return v;
}

// One list per lane (lanes l < k): its entries are col[start, start + len)
// of the arrays colp / valp, values taken times `scale` (fill mode; a NULL
// valp means all-true booleans).  scaled: multiply by scale (the B rows of
// a product) or take the values as they are (layer rows).
template <typename V>
struct KwList {
    const int32_t* colp;
    const void* valp;
    int64_t start;
    int32_t len;
    V scale;
};

// Merges the k lists held by lanes 0..k-1 of the calling wave (k <= KMAX,
// sum of lengths L <= KW_LMAX, both wave-uniform; the caller checks).
// UNIFORM: every list's colp and valp are the same (wave-uniform) arrays.
// Count mode (FILL = false): returns the number of distinct columns
// (wave-uniform).  Fill mode: writes the merged row to out_col/out_val
// starting at out_off (wave-uniform) and returns the count.
template <int SR, int KMAX, bool FILL, bool SCALED, bool UNIFORM = false>
__device__ inline int32_t kway_merge_wave(const KwList<typename Sr<SR>::acc_t>& lst, int k, int32_t L,
                                          KwLds<typename Sr<SR>::acc_t, FILL>& W, int32_t* out_col, void* out_val,
                                          int64_t out_off) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    const int lane = lane_id();
    const int32_t len = lane < k ? lst.len : 0;
    const int32_t soff = wave_inclusive_scan_add(len) - len;  // flat offset of this lane's list
    // list l's offset and length (wave-uniform, scalar registers)
    auto LB = [&](int l) { return __builtin_amdgcn_readlane(soff, l); };
    auto LN = [&](int l) { return __builtin_amdgcn_readlane(len, l); };
    // stage the entries: up to KW_LMAX / 64 per lane, all their loads issued
    // before any is stored (flat index x = u*64 + lane belongs to the last
    // list starting at or before x; empty lists share their successor's
    // start).  Lists in one pair of arrays (UNIFORM: the B rows of a
    // product) skip the pointer shuffles.
    constexpr int NU = KW_LMAX / SPG_WAVE;
    int32_t rc[NU];
    V rv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        if (u * SPG_WAVE >= L) break;
        const int32_t x = u * SPG_WAVE + lane;
        int l = 0;
#pragma unroll
        for (int step = KMAX / 2; step > 0; step >>= 1) {
            const int cand = l + step;
            const int32_t so = __shfl(soff, cand < SPG_WAVE ? cand : SPG_WAVE - 1, SPG_WAVE);
            if (cand < k && so <= x) l = cand;
        }
        const int32_t lo = __shfl(soff, l, SPG_WAVE);
        const int64_t st = __shfl(lst.start, l, SPG_WAVE);
        const int32_t* cp = UNIFORM ? lst.colp : (const int32_t*)__shfl((long long)(intptr_t)lst.colp, l, SPG_WAVE);
        const void* vp = !FILL ? nullptr
                               : (UNIFORM ? lst.valp : (const void*)__shfl((long long)(intptr_t)lst.valp, l, SPG_WAVE));
        V sc = S::zero();
        if constexpr (FILL && SCALED) sc = __shfl(lst.scale, l, SPG_WAVE);
        if (x < L) {
            const int64_t q = st + (x - lo);
            rc[u] = cp[q];
            if constexpr (FILL) {
                // no value array: structure-only output (booleans: all true)
                V v = (vp || SR == SR_BOOL) ? S::load(vp, q) : S::zero();
                rv[u] = v;
                if constexpr (SCALED) rv[u] = S::mul(sc, v);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        if (u * SPG_WAVE >= L) break;
        const int32_t x = u * SPG_WAVE + lane;
        if (x < L) {
            W.col[x] = rc[u];
            if constexpr (FILL) W.val[x] = rv[u];
        }
    }
    wave_lds_sync();
    // column span of the row: first and last entries of every list
    int32_t cmin = KW_INF, cmax = -1;
    if (lane < k && len > 0) {
        cmin = W.col[soff];
        cmax = W.col[soff + len - 1];
    }
#pragma unroll
    for (int d = SPG_WAVE / 2; d > 0; d >>= 1) {
        const int32_t a = lane_xor(cmin, d), b = lane_xor(cmax, d);
        cmin = a < cmin ? a : cmin;
        cmax = b > cmax ? b : cmax;
    }
    if (cmax < 0) return 0;  // no entries
    const int64_t span = (int64_t)cmax - cmin + 1;
    const int64_t width = (span + SPG_WAVE - 1) / SPG_WAVE;
    const int64_t key64 = (int64_t)cmin + (int64_t)lane * width;  // this lane's range starts here
    const int32_t key = key64 > (int64_t)cmax ? cmax + 1 : (int32_t)key64;
    // Per list l < KMAX (lists past k are empty: s = e, head INF): s[l] the
    // first entry at column >= key, e[l] the end of this lane's range, h[l]
    // the head column.  Straight-line code over all KMAX lists, every LDS read
    // unconditional (clamped inside the staged row) and results selected, so
    // each step's KMAX reads are in flight together.
    auto col_at = [&](int32_t x) { return W.col[x < KW_LMAX - 1 ? x : KW_LMAX - 1]; };
    int32_t s[KMAX], e[KMAX], h[KMAX], ln[KMAX];
    int32_t maxlen = 0;
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
        ln[l] = l < k ? LN(l) : 0;  // wave-uniform
        s[l] = l < k ? LB(l) : 0;
        maxlen = ln[l] > maxlen ? ln[l] : maxlen;
    }
    // uniform-step lower bound: at step t list l's n is ceil(len_l / 2^t);
    // the answer stays in [s, s + n]
    for (int t = 0; ((maxlen + (1 << t) - 1) >> t) > 1; ++t) {
        int32_t probe[KMAX];
#pragma unroll
        for (int l = 0; l < KMAX; ++l) {
            const int32_t n = (ln[l] + (1 << t) - 1) >> t;
            const int32_t half = n > 1 ? n >> 1 : 0;
            probe[l] = col_at(s[l] + half);
        }
#pragma unroll
        for (int l = 0; l < KMAX; ++l) {
            const int32_t n = (ln[l] + (1 << t) - 1) >> t;
            const int32_t half = n > 1 ? n >> 1 : 0;
            s[l] += probe[l] < key ? half : 0;
        }
    }
    {
        int32_t probe[KMAX];
#pragma unroll
        for (int l = 0; l < KMAX; ++l) probe[l] = col_at(s[l]);
#pragma unroll
        for (int l = 0; l < KMAX; ++l) s[l] += (ln[l] > 0 && probe[l] < key) ? 1 : 0;
    }
    // this lane's range ends where the next lane's begins
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
        const int32_t nxt = lane_next(s[l]);
        e[l] = l < k ? (lane == SPG_WAVE - 1 ? LB(l) + LN(l) : nxt) : s[l];  // lists past k: empty
    }
    auto load_heads = [&]() {
        int32_t probe[KMAX];
#pragma unroll
        for (int l = 0; l < KMAX; ++l) probe[l] = col_at(s[l]);
#pragma unroll
        for (int l = 0; l < KMAX; ++l) h[l] = s[l] < e[l] ? probe[l] : KW_INF;
    };
    // one merge step: the smallest head; every list holding it advances
    // (equal columns are one output); on_list(l) sees them in ascending l
    auto step = [&](auto on_list) -> int32_t {
        int32_t mn = KW_INF;
#pragma unroll
        for (int l = 0; l < KMAX; ++l) mn = h[l] < mn ? h[l] : mn;
        if (mn == KW_INF) return mn;
#pragma unroll
        for (int l = 0; l < KMAX; ++l) {
            const bool adv = h[l] == mn;
            on_list(l, adv);
            s[l] += adv ? 1 : 0;
        }
        int32_t probe[KMAX];
#pragma unroll
        for (int l = 0; l < KMAX; ++l) probe[l] = col_at(s[l]);
#pragma unroll
        for (int l = 0; l < KMAX; ++l) h[l] = h[l] == mn ? (s[l] < e[l] ? probe[l] : KW_INF) : h[l];
        return mn;
    };
    // counting sweep
    load_heads();
    int32_t cnt = 0;
    while (step([](int, bool) {}) != KW_INF) ++cnt;
    if constexpr (!FILL) {
        return wave_reduce_add(cnt);
    } else {
        const int32_t incl = wave_inclusive_scan_add(cnt);
        const int32_t total = __builtin_amdgcn_readlane(incl, SPG_WAVE - 1);
        // the writing sweep restarts where the previous lane's range ended
#pragma unroll
        for (int l = 0; l < KMAX; ++l) {
            const int32_t prv = lane_prev(e[l]);
            if (l < k) s[l] = lane == 0 ? LB(l) : prv;
        }
        load_heads();
        int64_t o = out_off + (incl - cnt);
        while (true) {
            V acc = S::zero();
            bool first = true;
            // the values of the lists holding the smallest head, in ascending
            // list order (the oracle's fold); read before the lists advance
            const int32_t mn = step([&](int l, bool adv) {
                const V v = W.val[s[l] < KW_LMAX - 1 ? s[l] : KW_LMAX - 1];
                if (adv) {
                    acc = first ? v : S::add(acc, v);
                    first = false;
                }
            });
            if (mn == KW_INF) break;
            out_col[o] = mn;
            if (out_val) S::store(out_val, o, acc);
            ++o;
        }
        return total;
    }
}

}  // namespace spg
