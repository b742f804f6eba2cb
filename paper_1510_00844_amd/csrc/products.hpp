// Enumerating the scalar products of one output row inside a workgroup.
//
// Row i of C gathers, for every stored A(i,k) in the window, the stored
// entries of B(k,:) (the row form of Algorithm 1).  B rows differ wildly in
// length (R-MAT hubs), so instead of giving each thread one A entry, a batch
// of NT A entries is turned into a flat index space of products with a
// workgroup prefix sum of their B-segment lengths; thread f then finds its
// A entry by binary search over the NT offsets held in LDS.  Neighbouring
// threads read neighbouring B entries, so gathers stay coalesced and no
// thread walks a long B row alone.
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
        for (int32_t f = threadIdx.x; f < total; f += NT) {
            // largest t with off[t] <= f  (off[0] = 0 <= f < off[NT] = total)
            int lo = 0, hi = NT;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (L.off[mid] <= f) lo = mid; else hi = mid;
            }
            visit(lo, base + lo, L.bstart[lo] + (f - L.off[lo]));
        }
        __syncthreads();
    }
}

}  // namespace spg
