// Row-compressed hypersparse matrices (DCSR) and the cut of A's rows into
// the pieces of the Sparse SUMMA stage blocks.
//
// DCSR is the row-wise counterpart of DCSC (Section 4.2): only the rows that
// hold entries are kept, each with its row index, so the arrays are O(nnz)
// whatever the row dimension.  Its pointer, column and value arrays are an
// ordinary CSR over the kept rows (the "compressed view").
//
// One process's Sparse SUMMA stages (Section 4.1, Algorithm 2) multiply A's
// columns and B's rows of each block of b inner indices and keep every
// block product; a multiway merge sums them at the end (Section 4.3).  With
// all of the process's blocks resident on one GPU, the block products are
// one product: each compressed row of A is cut where its columns cross into
// the next block, every piece becomes a row of its own ("piece rows"), and
// the product of the piece rows by B holds each block product's rows side
// by side, a row's stage rows next to each other in stage order.  The merge
// then sums, for every row of A, the contiguous run of its piece rows.
#pragma once
#include "common.hpp"

namespace spg {

// flags[1 + i] = 1 when row i holds an entry; the in-place scan of
// flags[1..m] then gives each kept row its slot.
__global__ void __launch_bounds__(256) k_nonempty_flags(const int64_t* rp, int64_t m, int64_t* flags) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) flags[1 + i] = rp[i + 1] > rp[i] ? 1 : 0;
}

// Kept rows to their slots: pos is the scan of the flags above (pos[i] =
// kept rows before i, pos[m] = all kept rows).  ids_in gives the row index
// to record (NULL: i itself).
__global__ void __launch_bounds__(256) k_compress_rows(const int64_t* rp, int64_t m, const int64_t* pos,
                                                       const int32_t* ids_in, int32_t* row_ids, int64_t* row_ptr) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) {
        const int64_t p = pos[i];
        if (pos[i + 1] > p) {
            row_ids[p] = ids_in ? ids_in[i] : (int32_t)i;
            row_ptr[p] = rp[i];
        }
    } else if (i == m) {
        row_ptr[pos[m]] = rp[m];
    }
}

// CSR row pointers of a DCSR matrix: row i starts where the first kept row
// with index >= i starts (absent rows are empty).
__global__ void __launch_bounds__(256) k_expand_rows(const int32_t* row_ids, const int64_t* row_ptr, int64_t nzr,
                                                     int64_t m, int64_t* out_rp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > m) return;
    int64_t lo = 0, hi = nzr;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row_ids[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    out_rp[i] = row_ptr[lo];
}

// Checks of the row index array of a DCSR matrix: strictly increasing, in
// [0, nrows), every kept row non-empty.
__global__ void __launch_bounds__(256) k_validate_rows(const int32_t* row_ids, const int64_t* row_ptr, int64_t nzr,
                                                       int64_t nrows, int32_t* bad) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= nzr) return;
    const int64_t r = row_ids[u];
    bool ok = r >= 0 && r < nrows && row_ptr[u + 1] > row_ptr[u];
    if (u > 0 && (int64_t)row_ids[u - 1] >= r) ok = false;
    if (!ok) atomicOr(bad, 1);
}

// flags[1 + e] = 1 where entry e opens a piece: its column lies in another
// block of b inner indices than the previous entry's.  Row starts are
// flagged by k_piece_row_starts, launched after this kernel.
__global__ void __launch_bounds__(256) k_piece_flags(const int32_t* col, int64_t nnz, uint32_t b, int64_t* flags) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nnz) return;
    const uint32_t blk = (uint32_t)col[e] / b;
    flags[1 + e] = (e == 0 || (uint32_t)col[e - 1] / b != blk) ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_piece_row_starts(const int64_t* rp, int64_t nzr, int64_t* flags) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= nzr) return;
    const int64_t s = rp[u];
    if (rp[u + 1] > s) flags[1 + s] = 1;
}

// Piece rows: piece g starts at the entry whose flag made pos step to g + 1.
__global__ void __launch_bounds__(256) k_piece_rows(const int64_t* pos, int64_t nnz, int64_t* piece_rp) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < nnz) {
        if (pos[e + 1] > pos[e]) piece_rp[pos[e]] = e;
    } else if (e == nnz) {
        piece_rp[pos[nnz]] = nnz;
    }
}

// The merge as a product by a selection matrix S (nzr x pieces): row u of S
// holds a unit entry at each of row u's pieces, which are consecutive, so
// (S P)(u,:) sums row u's stage rows in stage order.
template <int SR>
__global__ void __launch_bounds__(256) k_selection(const int64_t* rp, int64_t nzr, const int64_t* pos,
                                                   int64_t npieces, int64_t* s_rp, int32_t* s_col, void* s_val) {
    typedef typename Sr<SR>::acc_t V;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i <= nzr) s_rp[i] = pos[rp[i]];
    if (i < npieces) {
        s_col[i] = (int32_t)i;
        Sr<SR>::store(s_val, i, (V)1);
    }
}

}  // namespace spg
