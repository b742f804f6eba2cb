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

// Same enumeration, with the gathers of U consecutive products of a thread
// issued back to back before any of them is applied: `load(q)` reads what
// the product needs from B, `apply(t, x)` consumes it.  Keeping U loads in
// flight per thread is what hides the gather latency.
template <int NT, int U, class Seg, class Pre, class Load, class Apply>
__device__ inline void for_each_product_u(int64_t a_beg, int64_t a_end, ProductLds<NT>& L, Seg seg,
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

}  // namespace spg
