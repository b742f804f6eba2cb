// Batched products: many independent instances are multiplied as one
// block-diagonal product.  The instances' CSR matrices are copied side by
// side into one CSR (row pointers shifted by the entries before the
// instance, column indices shifted by the columns before it), so every
// row-binned launch covers the rows of all instances at once and the
// binning balances uneven instances.  Results are split back per instance.
// Used for the Galerkin products R^T A R of multigrid restriction (the
// restriction experiments of Section 5.3), one instance per grid.
#pragma once
#include "common.hpp"

namespace spg {

struct BatchDesc {
    const int64_t* rp;
    const int32_t* col;
    const void* val;
    int64_t nrows;
    int64_t row_off;  // first row of the instance in the batch
    int64_t nz_off;   // first entry of the instance in the batch
    int64_t col_off;  // first column of the instance in the batch
};

__device__ inline int find_instance(const BatchDesc* d, int32_t nb, int64_t r) {
    int lo = 0, hi = nb;  // largest b with row_off <= r
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (d[mid].row_off <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// One thread per batch row: shifted row pointer and the row's entries.
// vw = value bytes (8 or 1; 0 = no values).
__global__ void __launch_bounds__(256) k_batch_assemble(const BatchDesc* d, int32_t nb, int64_t rows, int64_t nnz,
                                                        int32_t vw, int64_t* rp, int32_t* col, void* val) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r > rows) return;
    if (r == rows) {
        rp[rows] = nnz;
        return;
    }
    const int b = find_instance(d, nb, r);
    const BatchDesc& D = d[b];
    const int64_t i = r - D.row_off;
    const int64_t s = D.rp[i], e = D.rp[i + 1];
    const int64_t o = D.nz_off - D.rp[0];
    rp[r] = o + s;
    for (int64_t p = s; p < e; ++p) {
        col[o + p] = (int32_t)(D.col[p] + D.col_off);
        if (vw == 8) ((uint64_t*)val)[o + p] = ((const uint64_t*)D.val)[p];
        else if (vw == 1) ((uint8_t*)val)[o + p] = D.val ? ((const uint8_t*)D.val)[p] : (uint8_t)1;
    }
}

// Split the batch product back: per-instance row pointers starting at 0
// (instance b's rows at out_rp[row_off_b + b ...]) and column indices made
// local to the instance (in place).
__global__ void __launch_bounds__(256) k_batch_split(const BatchDesc* d, int32_t nb, int64_t rows, const int64_t* rp,
                                                     int32_t* col, int64_t* out_rp) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int b = find_instance(d, nb, r);
    const BatchDesc& D = d[b];
    const int64_t i = r - D.row_off;
    const int64_t base = rp[D.row_off];
    out_rp[D.row_off + b + i] = rp[r] - base;
    if (i == D.nrows - 1) out_rp[D.row_off + b + i + 1] = rp[r + 1] - base;
    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) col[p] = (int32_t)(col[p] - D.col_off);
}

}  // namespace spg
