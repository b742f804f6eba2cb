// Heap accumulator bin (HeapSpGEMM, Section 4.2): a row of C whose window of
// A holds few entries is the k-way merge of the k scaled rows B(k,:), one per
// stored A(i,k), each already sorted by column.  The heap of the paper keeps
// one head per B row and pops the smallest column; here one wave merges the
// row (kway.hpp): its products are staged in LDS, the column range is split
// over the 64 lanes and each lane pops the smallest of its k heads until its
// range is done.  The output comes out sorted with no hash table and no sort,
// and equal columns add in ascending k, the oracle's order, so FP64 values
// match the ascending-k sum bit for bit.
//
// Rows qualify when their window holds at most heap_max_lists A entries and
// at most KW_LMAX products.  The symbolic pass counts distinct columns (one
// sweep); the numeric pass writes the row at its offset.
#pragma once
#include "kway.hpp"
#include "numeric.hpp"

namespace spg {

// The k B rows of row i as the lanes' lists (lane l: A entry a_beg + l).
template <typename V, int SR, bool FILL>
__device__ inline KwList<V> heap_lists(const Csr& A, const Csr& B, int64_t beg, int k) {
    typedef Sr<SR> S;
    KwList<V> lst{B.col, B.val, 0, 0, S::zero()};
    const int lane = lane_id();
    if (lane < k) {
        const int64_t p = beg + lane;
        const int64_t kk = A.col[p];
        const int64_t bs = B.rp[kk];
        lst.start = bs;
        lst.len = (int32_t)(B.rp[kk + 1] - bs);
        if (FILL) lst.scale = (A.val || SR == SR_BOOL) ? S::load(A.val, p) : S::zero();
    }
    return lst;
}

// Symbolic: rows of the heap bin located on the device, one wave per row.
template <int KMAX>
__global__ void __launch_bounds__(256) k_sym_heap(Csr A, Csr B, BinRef ref, const int64_t* a_beg, const int64_t* a_end,
                                                  const int64_t* flops, int64_t* cnt) {
    __shared__ KwLds<uint32_t, false> lds[4];
    KwLds<uint32_t, false>& W = lds[threadIdx.x >> 6];
    const int32_t* rows;
    int64_t n;
    ref.locate(rows, n);
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[r];
        const int64_t beg = a_beg[i];
        const int k = (int)(a_end[i] - beg);
        const KwList<uint32_t> lst = heap_lists<uint32_t, SR_BOOL, false>(A, B, beg, k);
        const int32_t c = kway_merge_wave<SR_BOOL, KMAX, false, false, true>(lst, k, (int32_t)flops[i], W, nullptr, nullptr, 0);
        if (lane_id() == 0) cnt[i] = c;
        wave_lds_sync();  // the staged row is read before the next one overwrites it
    }
}

// Numeric: one wave per row of the list (rows, count from the host).
template <int SR, int KMAX>
__global__ void __launch_bounds__(256) k_num_heap(Csr A, Csr B, const int32_t* rows, int64_t nrows, const int64_t* a_beg,
                                                  const int64_t* a_end, const int64_t* flops, OutRows c_rp,
                                                  int32_t* c_col, void* c_val) {
    typedef typename Sr<SR>::acc_t V;
    __shared__ KwLds<V, true> lds[4];
    KwLds<V, true>& W = lds[threadIdx.x >> 6];
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nrows; r += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[r];
        const int64_t beg = a_beg[i];
        const int k = (int)(a_end[i] - beg);
        const KwList<V> lst = heap_lists<V, SR, true>(A, B, beg, k);
        kway_merge_wave<SR, KMAX, true, true, true>(lst, k, (int32_t)flops[i], W, c_col, c_val, c_rp.off(i));
        wave_lds_sync();
    }
}

}  // namespace spg
