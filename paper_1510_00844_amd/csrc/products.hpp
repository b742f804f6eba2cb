// Enumerating the scalar products of one output row inside a workgroup.
//
// Row i of C gathers, for every stored A(i,k) in the window, the stored
// entries of B(k,:) (the row form of Algorithm 1).  B rows differ wildly in
// length (R-MAT hubs), so a batch of NT A entries is turned into a flat index
// space of products with a workgroup prefix sum of their B-segment lengths,
// and every thread takes an equal contiguous range of that space (a merge
// path over the segment offsets): one binary search over the NT offsets in
// LDS finds its first segment, after which it walks forward.  No thread walks
// a long B row alone and no product pays for a search.
#pragma once
#include <cstdint>
#include "common.hpp"

namespace spg {

template <int NT>
struct ProductLds {
    int32_t off[NT + 1];        // exclusive prefix of segment lengths
    int64_t bstart[NT];         // first B index of each segment
    int32_t tmp[NT / SPG_WAVE + 1];
};

// seg(p, &bstart, &len): B index range [bstart, bstart+len) for A entry p.
// visit(t, p, q): product of A entry p (slot t of the batch) and B entry q.
// pre(t, p): called once per A entry of the batch before the products (for
// staging per-entry data in LDS).  All threads of the block must call this.
template <int NT, class Seg, class Pre, class Visit>
__device__ inline void for_each_product(int64_t a_beg, int64_t a_end, ProductLds<NT>& L, Seg seg,
                                        Pre pre, Visit visit) {
    for (int64_t base = a_beg; base < a_end; base += NT) {
        const int64_t p = base + threadIdx.x;
        int64_t bs = 0;
        int32_t len = 0;
        if (p < a_end) {
            seg(p, bs, len);
            pre((int)threadIdx.x, p);
        }
        int32_t total;
        int32_t off = block_exclusive_scan<NT, int32_t>(len, &total, L.tmp);
        L.off[threadIdx.x] = off;
        L.bstart[threadIdx.x] = bs;
        if (threadIdx.x == 0) L.off[NT] = total;
        __syncthreads();
        const int32_t per = (total + NT - 1) / NT;
        int32_t f = (int32_t)threadIdx.x * per;
        const int32_t fend = f + per < total ? f + per : total;
        if (f < fend) {
            // largest t with off[t] <= f  (off[0] = 0 <= f < off[NT] = total)
            int t = 0, hi = NT;
            while (hi - t > 1) {
                int mid = (t + hi) >> 1;
                if (L.off[mid] <= f) t = mid; else hi = mid;
            }
            int32_t seg_end = L.off[t + 1];
            int64_t q = L.bstart[t] + (f - L.off[t]);
            for (; f < fend; ++f, ++q) {
                while (f >= seg_end) {  // next non-empty segment
                    ++t;
                    seg_end = L.off[t + 1];
                    q = L.bstart[t];
                }
                visit(t, base + t, q);
            }
        }
        __syncthreads();
    }
}

// Thread-contiguous variant: thread t walks products [t*per, (t+1)*per).
template <int NT, int U, class Seg, class Pre, class Load, class Apply>
__device__ inline void for_each_product_t(int64_t a_beg, int64_t a_end, ProductLds<NT>& L, Seg seg,
                                          Pre pre, Load load, Apply apply) {
    typedef decltype(load((int64_t)0)) X;
    for (int64_t base = a_beg; base < a_end; base += NT) {
        const int64_t p = base + threadIdx.x;
        int64_t bs = 0;
        int32_t len = 0;
        if (p < a_end) {
            seg(p, bs, len);
            pre((int)threadIdx.x, p);
        }
        int32_t total;
        int32_t off = block_exclusive_scan<NT, int32_t>(len, &total, L.tmp);
        L.off[threadIdx.x] = off;
        L.bstart[threadIdx.x] = bs;
        if (threadIdx.x == 0) L.off[NT] = total;
        __syncthreads();
        const int32_t per = (total + NT - 1) / NT;
        int32_t f = (int32_t)threadIdx.x * per;
        const int32_t fend = f + per < total ? f + per : total;
        if (f < fend) {
            int t = 0, hi = NT;
            while (hi - t > 1) {
                int mid = (t + hi) >> 1;
                if (L.off[mid] <= f) t = mid; else hi = mid;
            }
            int32_t seg_end = L.off[t + 1];
            int64_t q = L.bstart[t] + (f - L.off[t]);
            for (; f < fend; f += U) {
                int64_t qq[U];
                int tt[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (f + u < fend) {
                        while (f + u >= seg_end) {
                            ++t;
                            seg_end = L.off[t + 1];
                            q = L.bstart[t];
                        }
                        qq[u] = q++;
                        tt[u] = t;
                    }
                }
                X x[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (f + u < fend) x[u] = load(qq[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (f + u < fend) apply(tt[u], x[u]);
            }
        }
        __syncthreads();
    }
}

// 64-bit value of lane l (l wave-uniform).
__device__ inline int64_t readlane_i64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Same enumeration, mapped for coalesced gathers: each wave takes an equal
// contiguous range of the batch's products and its lanes take consecutive
// products, 64 at a time, so one load instruction reads 64 neighbouring B
// entries.  The segment the wave is in is kept in scalar registers (its
// index, its end, and the offset that turns a product number into a B
// index), so a step of 64 products that lies inside it costs no LDS access.
// A step that crosses segment ends reads the offsets of the next 64
// segments once (lane j: segment ta+j); the non-empty segments starting
// inside the step form a ballot mask, and each of them, in order, is taken
// by the lanes at or past its start (a scalar loop over the set bits, no
// LDS round trips).  Steps with many starts (short B rows) use a binary
// search over the lanes (shuffles) instead.
// U steps are gathered (`load(q)`) before any is applied (`apply(t, x)`), so
// each lane keeps U loads in flight.
// With COAL = false each thread instead takes its own contiguous range of
// products (one search per thread, U consecutive products per step): lanes
// then touch different segments, which spreads LDS atomics over more
// addresses at the price of uncoalesced gathers.
template <int NT, int U, bool COAL = true, bool DB = false, class Seg, class Pre, class Load, class Apply>
__device__ inline void for_each_product_u(int64_t a_beg, int64_t a_end, ProductLds<NT>& L, Seg seg,
                                          Pre pre, Load load, Apply apply) {
    typedef decltype(load((int64_t)0)) X;
    if (!COAL) {
        for_each_product_t<NT, U>(a_beg, a_end, L, seg, pre, load, apply);
        return;
    }
    // segment starts inside one step up to which the scalar loop is used
    constexpr int LOOP_MAX = 12;
    constexpr int NW = NT / SPG_WAVE;
    const int lane = lane_id();
    // wave-uniform values live in scalar registers (readfirstlane), so the
    // step bookkeeping below is scalar work and scalar branches
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SPG_WAVE));
    for (int64_t base = a_beg; base < a_end; base += NT) {
        const int64_t p = base + threadIdx.x;
        int64_t bs = 0;
        int32_t len = 0;
        if (p < a_end) {
            seg(p, bs, len);
            pre((int)threadIdx.x, p);
        }
        int32_t total;
        int32_t off = block_exclusive_scan<NT, int32_t>(len, &total, L.tmp);
        L.off[threadIdx.x] = off;
        L.bstart[threadIdx.x] = bs;
        if (threadIdx.x == 0) L.off[NT] = total;
        __syncthreads();
        const int32_t tot = __builtin_amdgcn_readfirstlane(total);
        const int32_t span = (tot + NW - 1) / NW;
        const int32_t f0 = wid * span;
        const int32_t f1 = f0 + span < tot ? f0 + span : tot;
        if (f0 < f1) {
            // segment of the range start (non-empty: the last one starting
            // at or before f0)
            int ta = 0;
            {
                int hi = NT;
                while (hi - ta > 1) {
                    int mid = (ta + hi) >> 1;
                    if (__builtin_amdgcn_readfirstlane(L.off[mid]) <= f0) ta = mid; else hi = mid;
                }
            }
            // product f of segment ta is B entry ta_rel + f; ta ends at ta_end
            int64_t ta_rel = readlane_i64(L.bstart[ta] - L.off[ta], 0);
            int32_t ta_end = __builtin_amdgcn_readfirstlane(L.off[ta + 1]);
            // The step search is written out twice, inline here and as the
            // locate lambda of the double-buffered form: folding this loop
            // onto the lambda cost the rank kernels 4 to 11 more VGPRs (one
            // workgroup fewer per CU), measured.
            if constexpr (!DB) {
                for (int32_t fb = f0; fb < f1; fb += SPG_WAVE * U) {
                    int64_t qq[U];
                    int tt[U];
                    bool ok[U];
    #pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int32_t fs = fb + u * SPG_WAVE;  // first product of this step
                        const int32_t f = fs + lane;
                        ok[u] = f < f1;
                        const int32_t flast = (fs + SPG_WAVE - 1 < f1 ? fs + SPG_WAVE - 1 : f1 - 1);
                        int t = ta;
                        int64_t rel = ta_rel;
                        if (fs < f1 && flast >= ta_end) {
                            // lane j: start (relative to fs), end and B offset of segment ta+j
                            const int j = ta + lane;
                            int32_t oj = INT32_MAX, oj1 = INT32_MAX;
                            int64_t bj = 0;
                            if (j < NT) {
                                oj = L.off[j];
                                oj1 = L.off[j + 1];
                                bj = L.bstart[j];
                            }
                            const int32_t dj = oj - fs;
                            const int64_t rj = bj - oj;
                            uint64_t starts = __ballot(lane > 0 && dj >= 0 && dj < SPG_WAVE && oj1 > oj);
                            if (__popcll(starts) <= LOOP_MAX) {
                                while (starts) {
                                    const int l = __builtin_ctzll(starts);
                                    starts &= starts - 1;
                                    const int32_t dl = __builtin_amdgcn_readlane(dj, l);
                                    const int64_t rl = readlane_i64(rj, l);
                                    if (lane >= dl) {
                                        t = ta + l;
                                        rel = rl;
                                    }
                                }
                            } else {
                                // last of the 64 starts at or before this lane
                                // (empty segments share the start of the next)
                                int lo = 0;
    #pragma unroll
                                for (int step = SPG_WAVE / 2; step > 0; step >>= 1) {
                                    const int32_t v = __shfl(dj, lo + step, SPG_WAVE);
                                    if (v <= lane) lo += step;
                                }
                                t = ta + lo;
                                rel = __shfl(rj, lo, SPG_WAVE);
                            }
                            // more than 64 segments start in the step (empty B
                            // rows): the lanes past the 64th search all segments
                            const int32_t o64 =
                                ta + SPG_WAVE <= NT ? __builtin_amdgcn_readfirstlane(L.off[ta + SPG_WAVE]) : INT32_MAX;
                            if (o64 <= flast && f >= o64) {
                                int hi = NT;
                                t = ta + SPG_WAVE;
                                while (hi - t > 1) {
                                    int mid = (t + hi) >> 1;
                                    if (L.off[mid] <= f) t = mid; else hi = mid;
                                }
                                rel = L.bstart[t] - L.off[t];
                            }
                            // the next step starts in the segment of this step's
                            // last product
                            const int tn = __builtin_amdgcn_readlane(t, SPG_WAVE - 1);
                            const int dn = tn - ta;
                            ta_end = dn < SPG_WAVE ? __builtin_amdgcn_readlane(oj1, dn)
                                                   : __builtin_amdgcn_readfirstlane(L.off[tn + 1]);
                            ta_rel = readlane_i64(rel, SPG_WAVE - 1);
                            ta = tn;
                        }
                        tt[u] = t;
                        qq[u] = rel + f;
                    }
                    X x[U];
    #pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (ok[u]) x[u] = load(qq[u]);
    #pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (ok[u]) apply(tt[u], x[u]);
                }
            } else {
                // segment t and B entry q of this lane's product in the step that
                // starts at product fs; moves the scalar segment state forward
                auto locate = [&](int32_t fs, int& t, int64_t& q) {
                    const int32_t f = fs + lane;
                    const int32_t flast = (fs + SPG_WAVE - 1 < f1 ? fs + SPG_WAVE - 1 : f1 - 1);
                    t = ta;
                    int64_t rel = ta_rel;
                    if (fs < f1 && flast >= ta_end) {
                        // lane j: start (relative to fs), end and B offset of segment ta+j
                        const int j = ta + lane;
                        int32_t oj = INT32_MAX, oj1 = INT32_MAX;
                        int64_t bj = 0;
                        if (j < NT) {
                            oj = L.off[j];
                            oj1 = L.off[j + 1];
                            bj = L.bstart[j];
                        }
                        const int32_t dj = oj - fs;
                        const int64_t rj = bj - oj;
                        uint64_t starts = __ballot(lane > 0 && dj >= 0 && dj < SPG_WAVE && oj1 > oj);
                        if (__popcll(starts) <= LOOP_MAX) {
                            while (starts) {
                                const int l = __builtin_ctzll(starts);
                                starts &= starts - 1;
                                const int32_t dl = __builtin_amdgcn_readlane(dj, l);
                                const int64_t rl = readlane_i64(rj, l);
                                if (lane >= dl) {
                                    t = ta + l;
                                    rel = rl;
                                }
                            }
                        } else {
                            // last of the 64 starts at or before this lane
                            // (empty segments share the start of the next)
                            int lo = 0;
    #pragma unroll
                            for (int step = SPG_WAVE / 2; step > 0; step >>= 1) {
                                const int32_t v = __shfl(dj, lo + step, SPG_WAVE);
                                if (v <= lane) lo += step;
                            }
                            t = ta + lo;
                            rel = __shfl(rj, lo, SPG_WAVE);
                        }
                        // more than 64 segments start in the step (empty B
                        // rows): the lanes past the 64th search all segments
                        const int32_t o64 =
                            ta + SPG_WAVE <= NT ? __builtin_amdgcn_readfirstlane(L.off[ta + SPG_WAVE]) : INT32_MAX;
                        if (o64 <= flast && f >= o64) {
                            int hi = NT;
                            t = ta + SPG_WAVE;
                            while (hi - t > 1) {
                                int mid = (t + hi) >> 1;
                                if (L.off[mid] <= f) t = mid; else hi = mid;
                            }
                            rel = L.bstart[t] - L.off[t];
                        }
                        // the next step starts in the segment of this step's
                        // last product
                        const int tn = __builtin_amdgcn_readlane(t, SPG_WAVE - 1);
                        const int dn = tn - ta;
                        ta_end = dn < SPG_WAVE ? __builtin_amdgcn_readlane(oj1, dn)
                                               : __builtin_amdgcn_readfirstlane(L.off[tn + 1]);
                        ta_rel = readlane_i64(rel, SPG_WAVE - 1);
                        ta = tn;
                    }
                    q = rel + f;
                };
                // a round: U steps located and their gathers issued
                auto fetch = [&](int32_t fb, X* x, int* tt, bool* ok) {
    #pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int32_t fs = fb + u * SPG_WAVE;
                        ok[u] = fs + lane < f1;
                        int64_t q;
                        locate(fs, tt[u], q);
                        if (ok[u]) x[u] = load(q);
                    }
                };
                auto drain = [&](const X* x, const int* tt, const bool* ok) {
    #pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (ok[u]) apply(tt[u], x[u]);
                };
                constexpr int32_t R = SPG_WAVE * U;
                X xa[U];
                int ta_[U];
                bool oa[U];
                // two rounds in flight: the gathers of the next round are
                // issued before the products of the current one are applied
                // (more registers, fewer waves: pays when the gathers miss L2)
                X xb[U];
                int tb_[U];
                bool ob[U];
                fetch(f0, xa, ta_, oa);
                for (int32_t fb = f0; fb < f1; fb += 2 * R) {
                    if (fb + R < f1) fetch(fb + R, xb, tb_, ob);
                    drain(xa, ta_, oa);
                    if (fb + R >= f1) break;
                    if (fb + 2 * R < f1) fetch(fb + 2 * R, xa, ta_, oa);
                    drain(xb, tb_, ob);
                }
            }
        }
        __syncthreads();
    }
}

// Gather mode of the heavy-row kernels (a tuning choice):
//   0: coalesced, 4 steps in flight   1: coalesced, 8 steps in flight
//   2: per-thread ranges, 4 in flight 3: per-thread ranges, 8 in flight
//   4: coalesced, two rounds of 4 steps in flight (double-buffered)
template <int NT, int GM, class Seg, class Pre, class Load, class Apply>
__device__ inline void for_each_product_gm(int64_t a_beg, int64_t a_end, ProductLds<NT>& L, Seg seg,
                                           Pre pre, Load load, Apply apply) {
    if constexpr (GM == 0) for_each_product_u<NT, 4, true>(a_beg, a_end, L, seg, pre, load, apply);
    else if constexpr (GM == 1) for_each_product_u<NT, 8, true>(a_beg, a_end, L, seg, pre, load, apply);
    else if constexpr (GM == 2) for_each_product_u<NT, 4, false>(a_beg, a_end, L, seg, pre, load, apply);
    else if constexpr (GM == 4) for_each_product_u<NT, 4, true, true>(a_beg, a_end, L, seg, pre, load, apply);
    else for_each_product_u<NT, 8, false>(a_beg, a_end, L, seg, pre, load, apply);
}

// The products of one row by one wave, for rows whose products are few or
// whose B rows are short (no workgroup-wide enumeration, no barriers).  The
// row's A entries are taken 64 at a time: seg(p, bs, len, pa) gives lane
// p - base its B segment and a per-entry payload pa (the A value); a wave
// scan of the lengths gives the segment offsets, and product x of the batch
// (x = 64 (U s + u) + lane) lies in the last lane's segment starting at or
// before x (a binary search across the lanes; empty segments share the
// start of the next one).  Each lane issues its U gathers (load(q)) before
// applying any (apply(pa, x)), so U loads are in flight.
template <int U, typename PA, class Seg, class Load, class Apply>
__device__ inline void wave_products(int64_t beg, int64_t end, Seg seg, Load load, Apply apply) {
    typedef decltype(load((int64_t)0)) X;
    const int lane = lane_id();
    for (int64_t base = beg; base < end; base += SPG_WAVE) {
        const int64_t p = base + lane;
        int64_t bs = 0;
        int32_t len = 0;
        PA pa{};
        if (p < end) seg(p, bs, len, pa);
        const int32_t incl = wave_inclusive_scan_add(len);
        const int32_t soff = incl - len;
        const int32_t nb = __builtin_amdgcn_readlane(incl, SPG_WAVE - 1);
        for (int32_t x0 = 0; x0 < nb; x0 += SPG_WAVE * U) {
            int64_t q[U];
            PA a[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t x = x0 + u * SPG_WAVE + lane;
                int l = 0;
#pragma unroll
                for (int step = SPG_WAVE / 2; step > 0; step >>= 1) {
                    const int32_t so = __shfl(soff, l + step, SPG_WAVE);
                    if (so <= x) l += step;
                }
                q[u] = lane_get(bs, l) + (x - __shfl(soff, l, SPG_WAVE));
                a[u] = lane_get(pa, l);
                ok[u] = x < nb;
            }
            X v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) v[u] = load(q[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) apply(a[u], v[u]);
        }
    }
}

}  // namespace spg
