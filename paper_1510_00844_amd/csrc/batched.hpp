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

// Largest b with d[b].row_off <= r (instances with no rows share the
// offset of the next instance and are skipped).
__device__ inline int find_instance(const BatchDesc* d, int32_t nb, int64_t r) {
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (d[mid].row_off <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// Largest b with d[b].nz_off <= e: the instance holding batch entry e.
__device__ inline int find_instance_nz(const BatchDesc* d, int32_t nb, int64_t e) {
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (d[mid].nz_off <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// Grid-stride over x < max(rows + 1, nnz): row pointer x (shifted by the
// entries before its instance) and entry x (column shifted by the columns
// before its instance, value copied), so reads and writes are coalesced.
// The instances' first rows and entries are staged in LDS for the searches.
// vw = value bytes (8 or 1; 0 = no values).
constexpr int BATCH_LDS_MAX = 1024;  // instances whose offsets fit the LDS tables

__device__ inline int find_sorted(const int64_t* off, int32_t nb, int64_t x) {
    int lo = 0, hi = nb;  // largest b with off[b] <= x
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_batch_assemble(const BatchDesc* d, int32_t nb, int64_t rows, int64_t nnz,
                                                        int32_t vw, int32_t structure, int64_t* rp, int32_t* col,
                                                        void* val) {
    __shared__ int64_t s_row[BATCH_LDS_MAX], s_nz[BATCH_LDS_MAX];
    const bool lds = nb <= BATCH_LDS_MAX;
    if (lds)
        for (int b = threadIdx.x; b < nb; b += 256) {
            s_row[b] = d[b].row_off;
            s_nz[b] = d[b].nz_off;
        }
    __syncthreads();
    // structure = 0: the row pointers and columns are in place from an
    // earlier call with the same instances; only the values are copied
    const int64_t n = structure ? (rows + 1 > nnz ? rows + 1 : nnz) : nnz;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t x = base + threadIdx.x;
        if (structure && x < rows) {
            const BatchDesc& D = d[lds ? find_sorted(s_row, nb, x) : find_instance(d, nb, x)];
            rp[x] = D.nz_off + (D.rp[x - D.row_off] - D.rp[0]);
        } else if (structure && x == rows) {
            rp[rows] = nnz;
        }
        if (base < nnz) {
            // the instance of the block's first entry (one search, the same
            // address for every thread), then forward to this thread's entry
            int b = lds ? find_sorted(s_nz, nb, base) : find_instance_nz(d, nb, base);
            while (b + 1 < nb && (lds ? s_nz[b + 1] : d[b + 1].nz_off) <= x) ++b;
            if (x < nnz) {
                const BatchDesc& D = d[b];
                const int64_t e = x - D.nz_off + D.rp[0];
                if (structure) col[x] = (int32_t)(D.col[e] + D.col_off);
                if (vw == 8) ((uint64_t*)val)[x] = ((const uint64_t*)D.val)[e];
                else if (vw == 1) ((uint8_t*)val)[x] = D.val ? ((const uint8_t*)D.val)[e] : (uint8_t)1;
            }
        }
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
