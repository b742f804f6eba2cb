/*
 * CPU oracle for the local SpGEMM hot path and the multiway layer merge.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may link, load or call this file; it exists so tests, the
 * smoke check and the CPU baseline of the benchmark can compare against a
 * plain, slow, obviously correct computation.  It shares no code with the
 * GPU path.
 *
 * What it computes (paper: Section 2 notation, Section 3 and Algorithm 1):
 *   C = A * B over a semiring S, with A (m x K) and B (K x n) in CSR.  Only
 *   inner indices k in the window [k_lo, k_hi) take part, which is how one
 *   layer's product A(:,K_l) * B(K_l,:) of the split 3D distribution
 *   (Section 4, Algorithm 2) is expressed on one process.
 *   Structure: (i,j) is stored iff some k in the window has A(i,k) and B(k,j)
 *   stored.  Values are never inspected for the structure: explicit zeros are
 *   nonzeros (Section 5), so entries whose value is zero stay.
 *   Value: C(i,j) = fold of (+) over those k in ascending k of A(i,k) (x) B(k,j),
 *   the first term taken as is.
 *   Rows are emitted with increasing column index (Section 5.1.1 keeps the
 *   output sorted so the later merge is cheap).
 *
 * The product is Gustavson's algorithm written by rows: Algorithm 1 walks
 * columns of B and scatters scaled columns of A into a sparse accumulator;
 * the row form used here walks row i of A and scatters scaled rows of B into
 * a dense accumulator (the SPA of Section 3) of length n, then sorts the list
 * of touched columns.  Both forms produce the same matrix.
 *
 * The merge (Section 4.3, LocalMerge of Algorithm 2) adds c matrices of the
 * same shape entry by entry: the stored set is the union of the c stored
 * sets and equal (i,j) are combined with (+) in ascending layer order.
 *
 * Semirings (Section 2 allows any semiring):
 *   0  plus-times over double
 *   1  plus-times over 64-bit integers, two's-complement wrap-around
 *   2  or-and over booleans stored as uint8 0/1 (a NULL value array means
 *      every stored entry is true)
 *
 * Rows are independent, so the row loops may run on several OpenMP threads;
 * each thread owns its accumulator.  Compile with -ffp-contract=off so that
 * a*b+c is always two roundings.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { SR_F64 = 0, SR_I64 = 1, SR_BOOL = 2 };

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/* flops_i = sum over stored A(i,k), k in window, of nnz(B(k,:)): the number of
 * scalar multiplications row i needs (Section 2 counts them for any
 * semiring). */
int oracle_row_flops(int64_t m, const int64_t* a_rp, const int32_t* a_col,
                     const int64_t* b_rp, int64_t k_lo, int64_t k_hi,
                     int64_t* flops_out) {
    for (int64_t i = 0; i < m; ++i) {
        int64_t f = 0;
        for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
            int64_t k = a_col[p];
            if (k < k_lo || k >= k_hi) continue;
            f += b_rp[k + 1] - b_rp[k];
        }
        flops_out[i] = f;
    }
    return 0;
}

/* One row of the product.  spa_* are per-thread arrays of length n with
 * mark[] all zero on entry and on exit.  If out_col is NULL only the count is
 * produced. */
static int64_t product_row(int sr, int64_t i, const int64_t* a_rp, const int32_t* a_col,
                           const void* a_val, const int64_t* b_rp, const int32_t* b_col,
                           const void* b_val, int64_t k_lo, int64_t k_hi,
                           uint8_t* mark, double* spa_f, uint64_t* spa_u,
                           int32_t* touched, int32_t* out_col, void* out_val) {
    int64_t nt = 0;
    for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
        int64_t k = a_col[p];
        if (k < k_lo || k >= k_hi) continue;
        for (int64_t q = b_rp[k]; q < b_rp[k + 1]; ++q) {
            int32_t j = b_col[q];
            if (sr == SR_F64) {
                double t = ((const double*)a_val)[p] * ((const double*)b_val)[q];
                if (!mark[j]) { mark[j] = 1; spa_f[j] = t; touched[nt++] = j; }
                else spa_f[j] = spa_f[j] + t;
            } else if (sr == SR_I64) {
                uint64_t t = (uint64_t)((const int64_t*)a_val)[p] *
                             (uint64_t)((const int64_t*)b_val)[q];
                if (!mark[j]) { mark[j] = 1; spa_u[j] = t; touched[nt++] = j; }
                else spa_u[j] = spa_u[j] + t;
            } else {
                uint64_t av = a_val ? (((const uint8_t*)a_val)[p] != 0) : 1;
                uint64_t bv = b_val ? (((const uint8_t*)b_val)[q] != 0) : 1;
                uint64_t t = av & bv;
                if (!mark[j]) { mark[j] = 1; spa_u[j] = t; touched[nt++] = j; }
                else spa_u[j] = spa_u[j] | t;
            }
        }
    }
    if (out_col) qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t j = touched[t];
        if (out_col) {
            out_col[t] = j;
            if (out_val) {
                if (sr == SR_F64) ((double*)out_val)[t] = spa_f[j];
                else if (sr == SR_I64) ((int64_t*)out_val)[t] = (int64_t)spa_u[j];
                else ((uint8_t*)out_val)[t] = (uint8_t)spa_u[j];
            }
        }
        mark[j] = 0;
    }
    return nt;
}

/* Count (out_col == NULL) or fill pass over a set of rows.
 * rows == NULL means rows 0..nsel-1.  For the fill pass out_ptr[r] gives the
 * offset of selected row r in out_col/out_val (out_ptr has nsel+1 entries).
 * Returns 0, or -1 when scratch memory cannot be allocated. */
static int spgemm_rows(int sr, int64_t n, const int64_t* a_rp, const int32_t* a_col,
                       const void* a_val, const int64_t* b_rp, const int32_t* b_col,
                       const void* b_val, int64_t k_lo, int64_t k_hi, int64_t nsel,
                       const int64_t* rows, int64_t* cnt_out, const int64_t* out_ptr,
                       int32_t* out_col, void* out_val, int nthreads) {
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
#endif
    {
        uint8_t* mark = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
        double* spa_f = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        uint64_t* spa_u = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int ok = mark && spa_f && spa_u && touched;
        if (!ok) err = 1;
        {
            /* every thread reaches the work-sharing loop; one without
             * scratch skips its rows and the call reports the failure */
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t r = 0; r < nsel; ++r) {
                if (!ok) continue;
                int64_t i = rows ? rows[r] : r;
                int32_t* oc = out_col ? out_col + out_ptr[r] : NULL;
                void* ov = NULL;
                if (out_col && out_val) {
                    size_t w = (sr == SR_BOOL) ? 1 : 8;
                    ov = (char*)out_val + w * (size_t)out_ptr[r];
                }
                int64_t c = product_row(sr, i, a_rp, a_col, a_val, b_rp, b_col, b_val,
                                        k_lo, k_hi, mark, spa_f, spa_u, touched, oc, ov);
                if (cnt_out) cnt_out[r] = c;
            }
        }
        free(mark); free(spa_f); free(spa_u); free(touched);
    }
    return err ? -1 : 0;
}

int oracle_spgemm_count(int sr, int64_t n, const int64_t* a_rp, const int32_t* a_col,
                        const int64_t* b_rp, const int32_t* b_col, int64_t k_lo,
                        int64_t k_hi, int64_t nsel, const int64_t* rows, int64_t* cnt_out,
                        int nthreads) {
    /* The stored set does not depend on values or on the semiring: count with
     * the boolean semiring and implicit all-true values. */
    (void)sr;
    return spgemm_rows(SR_BOOL, n, a_rp, a_col, NULL, b_rp, b_col, NULL, k_lo, k_hi, nsel, rows,
                       cnt_out, NULL, NULL, NULL, nthreads);
}

int oracle_spgemm_fill(int sr, int64_t n, const int64_t* a_rp, const int32_t* a_col,
                       const void* a_val, const int64_t* b_rp, const int32_t* b_col,
                       const void* b_val, int64_t k_lo, int64_t k_hi, int64_t nsel,
                       const int64_t* rows, const int64_t* out_ptr, int32_t* out_col,
                       void* out_val, int nthreads) {
    return spgemm_rows(sr, n, a_rp, a_col, a_val, b_rp, b_col, b_val, k_lo, k_hi, nsel, rows,
                       NULL, out_ptr, out_col, out_val, nthreads);
}

/* FP64 parity support.  For every stored entry of the product, in the
 * oracle's output order (rows as selected, columns ascending):
 *   comp   the terms A(i,k)*B(k,j) (each rounded once, as every product is)
 *          added in ascending k with Neumaier's compensated summation, so
 *          comp is within about one rounding of their exact sum;
 *   absum  the sum of |A(i,k)*B(k,j)| over the same terms;
 *   nterms the number of terms.
 * A result summed in any other order from the same rounded terms differs
 * from their exact sum by at most (nterms-1)*u*absum to first order
 * (u = 2^-53, the standard bound for recursive summation).  out_ptr as for
 * the fill pass; the selected rows' structure must be that of the fill
 * pass. */
static void check_row(int64_t i, const int64_t* a_rp, const int32_t* a_col, const double* a_val,
                      const int64_t* b_rp, const int32_t* b_col, const double* b_val, int64_t k_lo,
                      int64_t k_hi, uint8_t* mark, double* sum, double* comp, double* absum,
                      int64_t* nterms, int32_t* touched, double* comp_out, double* abs_out,
                      int64_t* nterms_out) {
    int64_t nt = 0;
    for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
        int64_t k = a_col[p];
        if (k < k_lo || k >= k_hi) continue;
        for (int64_t q = b_rp[k]; q < b_rp[k + 1]; ++q) {
            int32_t j = b_col[q];
            double t = a_val[p] * b_val[q];
            if (!mark[j]) {
                mark[j] = 1;
                sum[j] = t;
                comp[j] = 0.0;
                absum[j] = t < 0 ? -t : t;
                nterms[j] = 1;
                touched[nt++] = j;
            } else {
                /* Neumaier: the rounding error of s + t, recovered exactly
                 * from the larger operand, accumulates in comp */
                double s = sum[j];
                double r = s + t;
                double as = s < 0 ? -s : s, at = t < 0 ? -t : t;
                if (as >= at) comp[j] += (s - r) + t;
                else comp[j] += (t - r) + s;
                sum[j] = r;
                absum[j] += at;
                nterms[j] += 1;
            }
        }
    }
    qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t j = touched[t];
        comp_out[t] = sum[j] + comp[j];
        abs_out[t] = absum[j];
        nterms_out[t] = nterms[j];
        mark[j] = 0;
    }
}

int oracle_spgemm_f64_check(int64_t n, const int64_t* a_rp, const int32_t* a_col, const double* a_val,
                            const int64_t* b_rp, const int32_t* b_col, const double* b_val,
                            int64_t k_lo, int64_t k_hi, int64_t nsel, const int64_t* rows,
                            const int64_t* out_ptr, double* comp_out, double* abs_out,
                            int64_t* nterms_out, int nthreads) {
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
#endif
    {
        size_t nn = (size_t)(n > 0 ? n : 1);
        uint8_t* mark = (uint8_t*)calloc(nn, 1);
        double* sum = (double*)malloc(sizeof(double) * nn);
        double* comp = (double*)malloc(sizeof(double) * nn);
        double* absum = (double*)malloc(sizeof(double) * nn);
        int64_t* nterms = (int64_t*)malloc(sizeof(int64_t) * nn);
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * nn);
        int ok = mark && sum && comp && absum && nterms && touched;
        if (!ok) err = 1;
        {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t r = 0; r < nsel; ++r) {
                if (!ok) continue;
                int64_t i = rows ? rows[r] : r;
                int64_t o = out_ptr[r];
                check_row(i, a_rp, a_col, a_val, b_rp, b_col, b_val, k_lo, k_hi, mark, sum, comp, absum,
                          nterms, touched, comp_out + o, abs_out + o, nterms_out + o);
            }
        }
        free(mark); free(sum); free(comp); free(absum); free(nterms); free(touched);
    }
    return err ? -1 : 0;
}

/* Merge of c layers (all m x n, canonical).  Same accumulator; the layers
 * are visited in ascending order, so equal (i,j) fold in layer order. */
static int64_t merge_row(int sr, int64_t i, int c, const int64_t* const* rps,
                         const int32_t* const* cols, const void* const* vals,
                         uint8_t* mark, double* spa_f, uint64_t* spa_u, int32_t* touched,
                         int32_t* out_col, void* out_val) {
    int64_t nt = 0;
    for (int l = 0; l < c; ++l) {
        for (int64_t q = rps[l][i]; q < rps[l][i + 1]; ++q) {
            int32_t j = cols[l][q];
            if (sr == SR_F64) {
                double t = vals ? ((const double*)vals[l])[q] : 0.0;
                if (!mark[j]) { mark[j] = 1; spa_f[j] = t; touched[nt++] = j; }
                else spa_f[j] = spa_f[j] + t;
            } else if (sr == SR_I64) {
                uint64_t t = vals ? (uint64_t)((const int64_t*)vals[l])[q] : 0;
                if (!mark[j]) { mark[j] = 1; spa_u[j] = t; touched[nt++] = j; }
                else spa_u[j] = spa_u[j] + t;
            } else {
                uint64_t t = (vals && vals[l]) ? (((const uint8_t*)vals[l])[q] != 0) : 1;
                if (!mark[j]) { mark[j] = 1; spa_u[j] = t; touched[nt++] = j; }
                else spa_u[j] = spa_u[j] | t;
            }
        }
    }
    if (out_col) qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t j = touched[t];
        if (out_col) {
            out_col[t] = j;
            if (out_val) {
                if (sr == SR_F64) ((double*)out_val)[t] = spa_f[j];
                else if (sr == SR_I64) ((int64_t*)out_val)[t] = (int64_t)spa_u[j];
                else ((uint8_t*)out_val)[t] = (uint8_t)spa_u[j];
            }
        }
        mark[j] = 0;
    }
    return nt;
}

static int merge_rows(int sr, int64_t m, int64_t n, int c, const int64_t* const* rps,
                      const int32_t* const* cols, const void* const* vals, int64_t* cnt_out,
                      const int64_t* out_ptr, int32_t* out_col, void* out_val, int nthreads) {
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
#endif
    {
        uint8_t* mark = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
        double* spa_f = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        uint64_t* spa_u = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int ok = mark && spa_f && spa_u && touched;
        if (!ok) err = 1;
        {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
            for (int64_t i = 0; i < m; ++i) {
                if (!ok) continue;
                int32_t* oc = out_col ? out_col + out_ptr[i] : NULL;
                void* ov = NULL;
                if (out_col && out_val) {
                    size_t w = (sr == SR_BOOL) ? 1 : 8;
                    ov = (char*)out_val + w * (size_t)out_ptr[i];
                }
                int64_t k = merge_row(sr, i, c, rps, cols, vals, mark, spa_f, spa_u, touched,
                                      oc, ov);
                if (cnt_out) cnt_out[i] = k;
            }
        }
        free(mark); free(spa_f); free(spa_u); free(touched);
    }
    return err ? -1 : 0;
}

int oracle_merge_count(int64_t m, int64_t n, int c, const int64_t* const* rps,
                       const int32_t* const* cols, int64_t* cnt_out, int nthreads) {
    return merge_rows(SR_BOOL, m, n, c, rps, cols, NULL, cnt_out, NULL, NULL, NULL, nthreads);
}

int oracle_merge_fill(int sr, int64_t m, int64_t n, int c, const int64_t* const* rps,
                      const int32_t* const* cols, const void* const* vals,
                      const int64_t* out_ptr, int32_t* out_col, void* out_val, int nthreads) {
    return merge_rows(sr, m, n, c, rps, cols, vals, NULL, out_ptr, out_col, out_val, nthreads);
}
