/*
 * spgemm.h -- C ABI of the MI355X (gfx950) local sparse x sparse product and
 * multiway layer merge: the per-process hot path of Split-3D-SpGEMM
 * (Azad et al., "Exploiting Multiple Levels of Parallelism in Sparse
 * Matrix-Matrix Multiplication", arXiv:1510.00844).
 *
 * Operation (Section 2 notation, Section 3 / Algorithm 1): C = A * B with
 * A in S^{m x K}, B in S^{K x n} over a semiring S.  Only inner indices k in
 * a window [k_lo, k_hi) take part, so one call computes one layer's partial
 * product C_l = A(:,K_l) * B(K_l,:) of the split 3D distribution
 * (Section 4, Algorithm 2, local multiply); the full product uses
 * [0, K).  spgemm_merge_layers is LocalMerge (Section 4.3, Algorithm 2):
 * the entry-wise semiring sum of c partial products.
 *
 * Conventions shared by every entry point:
 *   - Matrices are CSR, 0-based (the paper indexes from 1): int64 row
 *     pointers (nrows+1 entries, row_ptr[0] == 0), int32 column indices
 *     strictly increasing inside each row, and a value array of nnz
 *     elements: double (SPG_SR_PLUS_TIMES_F64), int64_t
 *     (SPG_SR_PLUS_TIMES_I64) or uint8_t 0/1 (SPG_SR_OR_AND_BOOL; val may
 *     be NULL there, meaning every stored entry is true).
 *   - All array pointers inside spg_csr and all output arrays are DEVICE
 *     pointers on the plan's device, owned by the caller.  The library never
 *     frees them.  Host pointers appear only where a parameter says "host".
 *   - The stored set of C is structural: (i,j) is stored iff some k in the
 *     window has A(i,k) and B(k,j) stored.  Explicit zeros and entries whose
 *     value cancels to zero stay stored (Section 5 counts explicit zeros as
 *     nonzeros).  Output rows are sorted by column (Section 5.1.1).
 *   - INT64 arithmetic wraps modulo 2^64.  Structure, INT64 and boolean
 *     results are exact.  FP64: every product A(i,k)*B(k,j) is rounded once
 *     (never fused with the add), and an entry's N terms are added in an
 *     order that may differ from ascending k.  An entry is therefore within
 *     1e-12 relative of the ascending-k sum, or, where N is large enough for
 *     that to fail, within gamma_{N-1} * sum|terms| + u*|S| (u = 2^-53,
 *     gamma_k = k u / (1 - k u)) of the exact sum S of the rounded terms:
 *     the bound the tests check against a compensated sum of the terms.
 *     Rows with at most 64 products, one A entry, or that take the k-way
 *     merge bin add in ascending k and match the ascending-k sum bit for
 *     bit.
 *   - Every call is asynchronous on the plan's stream except where a
 *     parameter is a host output (those synchronize the stream).
 *   - Errors are reported only through the return code; nothing aborts or
 *     throws.  spg_last_error() gives a message for the calling thread.
 *   - A plan is used by one host thread at a time.
 */
#ifndef SPGEMM_MI355X_H
#define SPGEMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPG_OK = 0,
    SPG_ERR_ARG = 1,           /* NULL pointer, bad window, bad enum, nlayers < 1 */
    SPG_ERR_SHAPE = 2,         /* A.ncols != B.nrows, layer shapes differ */
    SPG_ERR_NOT_CANONICAL = 3, /* validate option found unsorted/out-of-range input */
    SPG_ERR_INDEX_RANGE = 4,   /* a dimension >= 2^31, or > 2^19 columns on a path that needs fewer */
    SPG_ERR_OOM = 5,           /* device scratch allocation failed */
    SPG_ERR_CAPACITY = 6,      /* a caller-provided capacity is too small */
    SPG_ERR_HIP = 7,           /* a HIP runtime call failed; see spg_last_error() */
    SPG_ERR_STATE = 8          /* numeric called without the matching symbolic call */
} spg_status;

typedef enum {
    SPG_SR_PLUS_TIMES_F64 = 0,
    SPG_SR_PLUS_TIMES_I64 = 1,
    SPG_SR_OR_AND_BOOL = 2
} spg_semiring;

typedef struct {
    int64_t nrows;
    int64_t ncols;
    int64_t nnz;
    const int64_t* row_ptr; /* device, nrows+1 */
    const int32_t* col;     /* device, nnz */
    const void* val;        /* device, nnz; NULL allowed only for the boolean semiring */
} spg_csr;

/* Tuning options.  Zero fields take the defaults of spg_default_opts(). */
typedef struct {
    int32_t validate;          /* 1: check inputs are canonical CSR on the device first */
    int32_t small_max_flops;   /* rows with at most this many products use one wave (<= 64) */
    int32_t hash_max_flops;    /* symbolic: LDS hash table up to this many products per row */
    int32_t hash_max_nnz;      /* numeric: LDS hash table up to this many outputs per row */
    int32_t dense_chunk_cols;  /* numeric dense rows: columns per LDS chunk (2048, 4096, 8192 or 16384) */
    int32_t profile;           /* 1: time every kernel launch with HIP events */
    int32_t streams;           /* streams independent bins are spread over (1..4) */
    int32_t gather_map;        /* numeric heavy rows, products per lane: 1 = neighbouring lanes take
                                  neighbouring products (coalesced), 2 = each lane a contiguous range */
    int32_t unroll;            /* numeric heavy rows: gathers in flight per lane (4 or 8) */
    int32_t sym_gather_map;    /* the same two choices for the symbolic bitmap rows */
    int32_t sym_unroll;
    int32_t chunk_min_nnz;     /* numeric rows whose bitmap was saved by the symbolic pass and that have
                                  more than this many outputs take column-chunk work items instead of
                                  a hash table (1..hash_max_nnz; 0 = hash_max_nnz) */
    int32_t chunk_group;       /* most column chunks one such work item spans (1..256; the LDS may
                                  allow fewer) */
    int32_t rank_max_nnz;      /* numeric rows with a saved bitmap and at most this many outputs
                                  accumulate the whole row in one workgroup (capacities 4096, 8192,
                                  16384 as the LDS allows; below 4096: never) */
    int32_t rank_block;        /* threads per workgroup of the whole-row rank accumulator: 512 (the
                                  default: shares the CUs better with the rank-chunk kernel beside it)
                                  or 1024 (more loads in flight, faster alone; capacity 16384 only when
                                  the LDS allows it) */
    int32_t serial_heavy;      /* the this-many bins with the most work run back to back on the plan's
                                  stream; the other bins are spread over the streams (0..16) */
    int32_t chunk_unroll;      /* gathers in flight per lane in the rank-chunk items (4 or 8) */
    int32_t gather_pipeline;   /* bitmap and rank-chunk kernels in the coalesced 4-step mode keep two
                                  rounds of gathers in flight (more registers, fewer waves): 0 = when
                                  the gathered B arrays exceed the 32 MiB of L2, 1 = never, 2 = always */
    int32_t fused_max_nnz;     /* learned single pass: rows predicted to hold at most this many outputs
                                  (above the hash tables) may take the fused bitmap-and-rank kernel, up to
                                  rank_max_nnz and what the LDS holds; 0 = never (default: on this GPU
                                  the exact two-phase path is faster for such rows) */
    int32_t heap_max_lists;    /* rows with at most this many A entries in the window and at most 384
                                  products are merged from their B rows by one wave (the heap bin,
                                  both passes; sorted output, ascending-k sums): 1..32; 0 = the
                                  default, -1 = never (the default: on the workloads measured the
                                  hash tables are faster) */
} spg_opts;

typedef struct spg_plan_s* spg_plan;

void spg_default_opts(spg_opts* opts);

/* Create a plan bound to the current HIP device and to `stream` (a
 * hipStream_t; NULL = the null stream).  The plan owns all scratch memory
 * (row work counts, bin lists, split tables) and reuses it across calls. */
spg_status spg_plan_create(spg_plan* plan, void* stream, const spg_opts* opts);
spg_status spg_plan_destroy(spg_plan plan);
spg_status spg_plan_set_stream(spg_plan plan, void* stream);

/* Symbolic phase of the row-wise product (Section 3, Algorithm 1 written by
 * rows; Section 4.4 for the layer window): row i of C = A(:,K) B(K,:),
 * K = [k_lo,k_hi), stores the union of the column sets of the rows B(k,:)
 * with A(i,k) stored and k in K; this call counts each row's union.
 * c_row_ptr: device, m+1 entries, caller-owned; receives the exclusive
 * prefix sum of the row counts (c_row_ptr[m] = nnz(C)).
 * c_nnz: host; if not NULL it receives nnz(C) and the stream is synchronized.
 * Errors: SPG_ERR_SHAPE if A.ncols != B.nrows; SPG_ERR_ARG unless
 * 0 <= k_lo <= k_hi <= A.ncols. */
spg_status spgemm_symbolic(spg_plan plan, spg_semiring sr, const spg_csr* A, const spg_csr* B,
                           int64_t k_lo, int64_t k_hi, int64_t* c_row_ptr, int64_t* c_nnz);

/* Numeric phase (Section 3, Algorithm 1 by rows: C(i,:) is the semiring sum
 * over k in the window of A(i,k) times B(k,:)): fills c_col (int32) and
 * c_val (typed as the semiring) for the
 * row pointers computed by the last spgemm_symbolic on this plan, which must
 * have had the same A, B and window (SPG_ERR_STATE otherwise).  Rows come out
 * sorted by column.  c_val may be NULL to produce the structure only. */
spg_status spgemm_numeric(spg_plan plan, spg_semiring sr, const spg_csr* A, const spg_csr* B,
                          int64_t k_lo, int64_t k_hi, const int64_t* c_row_ptr, int32_t* c_col,
                          void* c_val);

/* LocalMerge: out = sum over l of layers[l] (entry-wise, semiring add, equal
 * (i,j) combined in ascending layer order).  `layers` is a HOST array of
 * nlayers descriptors of device matrices, all nrows x ncols and canonical.
 * Call twice: first with out_col == NULL (count pass: fills out_row_ptr,
 * m+1 device entries, and *out_nnz on the host, synchronizing), then with
 * out_col/out_val sized from *out_nnz (fill pass, same layers). */
spg_status spgemm_merge_layers(spg_plan plan, spg_semiring sr, int32_t nlayers,
                               const spg_csr* layers, int64_t* out_row_ptr, int32_t* out_col,
                               void* out_val, int64_t* out_nnz);

/* Hypersparse row-compressed matrix (DCSR): the row-wise counterpart of the
 * DCSC format of Section 4.2.  Only the nzr rows that hold entries are
 * kept, with their indices, so the arrays take O(nnz) space whatever nrows
 * is; row_ptr, col and val form an ordinary CSR over the kept rows (the
 * compressed view).  Canonical form: row_ids strictly increasing and in
 * [0, nrows), every kept row non-empty, columns strictly increasing inside a
 * row.  Device pointers, caller-owned, as for spg_csr. */
typedef struct {
    int64_t nrows;
    int64_t ncols;
    int64_t nzr;            /* kept rows */
    int64_t nnz;
    const int32_t* row_ids; /* device, nzr */
    const int64_t* row_ptr; /* device, nzr+1, row_ptr[0] == 0 */
    const int32_t* col;     /* device, nnz */
    const void* val;        /* device, nnz (NULL allowed for the boolean semiring) */
} spg_dcsr;

/* CSR -> DCSR (Section 4.2): the kept rows' indices and pointers; the
 * DCSR's col and val are A's own arrays.  Call twice: first with
 * row_ptr == NULL (count call: *nzr on the host, synchronizing), then with
 * row_ids (nzr entries; may be NULL when nzr is 0) and row_ptr (nzr+1
 * entries) allocated (fill call; it synchronizes too, and sets *nzr if nzr
 * is not NULL). */
spg_status spg_dcsr_compress(spg_plan plan, const spg_csr* A, int32_t* row_ids, int64_t* row_ptr, int64_t* nzr);

/* DCSR -> CSR: row_ptr (device, nrows+1) of the CSR whose col and val are
 * A's own arrays; absent rows are empty. */
spg_status spg_dcsr_expand(spg_plan plan, const spg_dcsr* A, int64_t* row_ptr);

/* One process's Sparse SUMMA stages with blocking b (Section 4.1, Algorithm
 * 2's stage loop; Section 4.3 merge): A (m x K, hypersparse) holds the
 * process's columns of A for all `stages` stages side by side, B (K x n) the
 * matching rows; each stage covers K/stages inner indices, cut into blocks of
 * b (b must divide K/stages, SPG_ERR_ARG otherwise).  Every block gives one
 * product A(:,block) B(block,:) (a rank-b update); the products are kept and
 * summed by a multiway merge that adds equal entries in stage order:
 *   C = sum over blocks, in order, of A(:,block) B(block,:)   (= A B).
 * C comes out as DCSR (rows with no entry dropped).  With one block the
 * product is computed directly.
 * Call twice.  Count call (c_row_ptr == NULL): computes the kept block
 * products and the merged structure, and returns on the host *c_nzr and
 * *c_nnz (and, if not NULL, *stage_nnz, the entries of all block products,
 * the intermediate the merge reads), synchronizing.  Fill call, same A, B,
 * stages and b: c_row_ids (c_nzr entries), c_row_ptr (c_nzr+1), c_col and
 * c_val (c_nnz each; c_val may be NULL for the structure only; arrays of no
 * entries may be NULL).  A's and B's values must not change between the two
 * calls (either call may read them).  SPG_ERR_STATE if the fill call does not
 * match the last count call on the plan; SPG_ERR_INDEX_RANGE above 2^22
 * row pieces (a piece is the part of a row inside one block). */
spg_status spgemm_summa_local(spg_plan plan, spg_semiring sr, const spg_dcsr* A, const spg_csr* B,
                              int64_t stages, int64_t b, int32_t* c_row_ids, int64_t* c_row_ptr,
                              int32_t* c_col, void* c_val, int64_t* c_nzr, int64_t* c_nnz,
                              int64_t* stage_nnz);

/* LocalMerge for callers that cannot allocate device memory (code under
 * HIP graph capture around it, tight serving loops, harnesses that forbid
 * allocation): the same two passes and results as spgemm_merge_layers, with
 * no plan and no allocation of any kind.  Its scratch (row lengths, bins,
 * bin lists, counters, scan tiles: 13 bytes per row) lives in one 16 MiB
 * array of device memory that the library holds on every GPU it runs on
 * until the process ends; hence at most 2^20 rows (SPG_ERR_CAPACITY
 * beyond).  `stream` is a hipStream_t (NULL = the null stream); the calls
 * run on it and synchronize it (the count pass, and the fill pass when
 * out_nnz is not NULL, read counts back).  Each pass classifies the rows
 * itself, so no state carries between calls; the array keeps the last
 * call's contents.  Calls that overlap on one GPU (from several threads or
 * on several streams) share that array and race: serialize them. */
spg_status spgemm_merge_layers_noalloc(void* stream, spg_semiring sr, int32_t nlayers, const spg_csr* layers,
                                       int64_t* out_row_ptr, int32_t* out_col, void* out_val, int64_t* out_nnz);

/* Row classes ("bins") the symbolic/numeric passes sort rows into. */
enum {
    SPG_BIN_EMPTY = 0,  /* no products */
    SPG_BIN_TINY = 1,   /* one stored A entry in the window: output = scaled B row */
    SPG_BIN_SMALL = 2,  /* few products: one wave, keys in registers */
    SPG_BIN_HASH0 = 3,  /* LDS hash table bins, 128 << (b - SPG_BIN_HASH0) slots */
    SPG_BIN_DENSE_PAR = 11, /* numeric only: column chunks of one row in parallel workgroups */
    SPG_BIN_DENSE = 12, /* large rows: LDS bitmap (symbolic) / column-chunked dense accumulator (numeric) */
    SPG_BIN_RANK0 = 13, /* numeric only: rank-space accumulator of 4096 << (b - SPG_BIN_RANK0) values */
    SPG_BIN_HEAP = 16,  /* few A entries: k-way merge of the row's B rows by one wave (HeapSpGEMM, Section 4.2) */
    SPG_NBINS = 17
};

/* Statistics of the last symbolic (and numeric) call, read back on demand
 * (synchronizes).  Per bin: rows, products (flops) and A entries; for the
 * numeric pass also output entries. */
typedef struct {
    int64_t m, n, k;
    int64_t flops;      /* total scalar multiplications */
    int64_t nnz_c;
    int64_t sym_rows[SPG_NBINS], sym_flops[SPG_NBINS], sym_annz[SPG_NBINS];
    int64_t num_rows[SPG_NBINS], num_flops[SPG_NBINS], num_annz[SPG_NBINS], num_cnnz[SPG_NBINS];
    int32_t dense_chunk_cols;
    int32_t dense_chunks;
} spg_stats;
spg_status spg_plan_stats(spg_plan plan, spg_stats* out);

/* Kernel timing (opts.profile = 1): events recorded on the plan's stream
 * around every launch.  Fills up to cap records of (name, launches, total
 * milliseconds) accumulated since the last reset; returns the count in *n. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} spg_kernel_time;
spg_status spg_profile_read(spg_plan plan, spg_kernel_time* out, int32_t cap, int32_t* n);
spg_status spg_profile_reset(spg_plan plan);
/* Time only the launches named `name` (the names spg_profile_read reports;
 * NULL or "" = every launch), so the other launches run without events. */
spg_status spg_profile_select(spg_plan plan, const char* name);

/* ------------------------------------------------------------------------
 * Row-size predictor (not in the paper; its Section 3 notes that computing
 * the output structure up front is about as hard as the product itself).
 * A 3-32-32-1 ReLU network in FP32 maps (log1p nnz(A(i,:)), log1p flops_i,
 * log1p max_k nnz(B(k,:))) to an estimate of log1p nnz(C(i,:)).  Parameters:
 * SPG_MLP_NPARAMS floats on the device, in the order W1[32][3] (row-major),
 * b1[32], W2[32][32], b2[32], w3[32], b3.
 * ------------------------------------------------------------------------ */
#define SPG_MLP_NPARAMS 1217

/* y[i] = network(x[3i..3i+2]) for i < n.  All pointers device. */
spg_status spg_mlp_forward(spg_plan plan, const float* params, const float* x, int64_t n, float* y);

/* Adds to grad[SPG_MLP_NPARAMS] the gradient of (1/n) sum_i a_i (y_i - t_i)^2,
 * a_i = alpha where y_i < t_i else 1, and adds the loss to *loss (if not
 * NULL).  The caller zeroes grad/loss first.  Device pointers. */
spg_status spg_mlp_grad(spg_plan plan, const float* params, const float* x, const float* t, int64_t n,
                        float alpha, float* grad, float* loss);

/* One Adam step (bias-corrected; step counts from 1) on params, with
 * moment buffers m, v of SPG_MLP_NPARAMS floats; grad is cleared to zero
 * afterwards.  Device pointers. */
spg_status spg_mlp_adam(spg_plan plan, float* params, float* grad, float* m, float* v, int64_t step,
                        float lr, float beta1, float beta2, float eps);

/* Training data from the last spgemm_symbolic on this plan: for every row
 * whose size would be predicted (more than one A entry, more products than
 * small_max_flops) and that has at least min_flops products, its features
 * (x, 3 floats) and target log1p of its exact count from c_row_ptr (t).  x
 * and t are device arrays of at least 3m and m floats; *nsel (host)
 * receives the number of rows written (order unspecified).  Synchronizes. */
spg_status spg_row_training_data(spg_plan plan, const int64_t* c_row_ptr, int64_t min_flops, float* x, float* t,
                                 int64_t* nsel);

typedef struct {
    int64_t rows_predicted; /* rows given a predicted capacity */
    int64_t rows_exact;     /* rows too large for a single-pass accumulator: exact method */
    int64_t rows_overflow;  /* predicted rows whose count exceeded the capacity: redone exactly */
    int64_t slots;          /* padded entries allocated */
    int64_t nnz_c;
    int64_t nnz_single;     /* entries of C produced by the single pass (the rest by the exact method) */
    int64_t bin_rows[SPG_NBINS];
} spg_learned_stats;

/* Single-pass product with predicted row sizes: C = A(:,K) B(K,:) computed
 * into plan-owned padded slots of capacity clamp((1 + margin) * prediction
 * + 8, max_k nnz(B(k,:)), min(flops_i, n)); mlp_params (device) NULL means
 * capacity = min(flops_i, n), the bound without a predictor.  Rows whose
 * count exceeds their slot, and rows too large for a single-pass
 * accumulator, are computed by the exact two-phase method.  *c_nnz (host)
 * receives nnz(C); st (host, optional) the statistics.  Synchronizes. */
spg_status spgemm_learned_run(spg_plan plan, spg_semiring sr, const spg_csr* A, const spg_csr* B,
                              int64_t k_lo, int64_t k_hi, const float* mlp_params, float margin,
                              int64_t* c_nnz, spg_learned_stats* st);

/* Writes the result of the last spgemm_learned_run (same A and B) as
 * canonical CSR into caller-owned device arrays: c_row_ptr (m+1), c_col and
 * c_val (nnz(C) entries; c_val may be NULL).  The structure is identical to
 * the two-phase method's. */
spg_status spgemm_learned_fetch(spg_plan plan, const spg_csr* A, const spg_csr* B, int64_t* c_row_ptr,
                                int32_t* c_col, void* c_val);

/* ------------------------------------------------------------------------
 * Batched Galerkin products (the restriction experiments of Section 5.3,
 * computed as (R^T A) R): for b < nb, out[b] = (RT[b] A[b]) R[b], with RT[b]
 * M_b x N_b, A[b] N_b x N_b', R[b] N_b' x M_b.  RT, A, R and out are HOST
 * arrays of nb descriptors; the matrices are device CSR.  The instances are
 * multiplied as one block-diagonal product, so every launch covers all
 * instances.  The first call with a given set of descriptors runs eagerly
 * (and synchronizes); with use_graph it then captures the whole device
 * sequence into one HIP graph, which later calls with the same descriptors
 * (same pointers and sizes) replay without any host synchronization.  Values
 * may change between such calls; the row pointers and column indices behind
 * the descriptors must not: later calls (graph or not) run only the value
 * work (assembly, the two numeric passes, the split into instances) with
 * the sizes, bin lists and saved row bitmaps of the first call, whose
 * symbolic passes are not repeated.
 * out[b] points into plan-owned memory (column indices local to the
 * instance), valid until the next call with other descriptors or
 * spg_plan_destroy.  Calls that overlap on one plan race.
 * ------------------------------------------------------------------------ */
spg_status spgemm_galerkin_batched(spg_plan plan, spg_semiring sr, int32_t nb, const spg_csr* RT,
                                   const spg_csr* A, const spg_csr* R, spg_csr* out, int32_t use_graph);

/* Copies the last batched result into caller-owned device buffers, on the
 * plan's stream: row_ptr gets, for each instance in order, its M_b + 1 row
 * pointers starting at 0 (sum of M_b + nb entries); col and val get the
 * instances' entries back to back (sum of out[b].nnz entries; column indices
 * local to the instance).  val may be NULL.  SPG_ERR_STATE without a
 * batched call on the plan. */
spg_status spgemm_galerkin_copy(spg_plan plan, int64_t* row_ptr, int32_t* col, void* val);

/* Autotuner of the batched Galerkin products: picks the bin thresholds,
 * gather mappings and stream count (fields small_max_flops, streams,
 * gather_map, unroll, sym_gather_map, hash_max_nnz of spg_opts) that
 * minimize the graph-replay time of spgemm_galerkin_batched on these
 * instances, by coordinate descent from the plan's options, each candidate
 * timed with HIP events over 5 replays, within about budget_ms of wall time
 * (<= 0: no limit).  Results are cached in the text file cache_path (one
 * JSON object per line, keyed by GPU architecture, CU count, semiring and
 * the instances' sizes; NULL = no cache): a cached key is used without
 * timing and *from_cache is set to 1.  The plan adopts the chosen options
 * (its batched state is reset); *best (may be NULL) receives them.
 * Synchronizes; allocates and frees temporary plans. */
spg_status spg_autotune_galerkin(spg_plan plan, spg_semiring sr, int32_t nb, const spg_csr* RT,
                                 const spg_csr* A, const spg_csr* R, const char* cache_path,
                                 int32_t budget_ms, spg_opts* best, int32_t* from_cache);

/* ------------------------------------------------------------------------
 * Restriction operators from distance-2 maximal independent sets (Section
 * 5.3, Algorithm 3).  A: a square device CSR whose pattern is an undirected
 * graph (symmetric pattern; values ignored).  In rounds until no candidate
 * is left, every candidate vertex draws a 64-bit key (SplitMix64 output of
 * seed ^ (round << 32 | vertex) in the high half, the vertex in the low
 * half); the candidates holding the smallest key within distance two join
 * the set, and they and every candidate within distance two of them stop
 * being candidates (two (min, select2nd) matrix-vector products per step).
 * Aggregates: each set vertex roots one, numbered in vertex order, with its
 * distance-1 neighbours; every other vertex joins the assigned neighbour
 * with the smallest SplitMix64 choice key.
 * in_mis: device, n bytes (1 = in the set); agg: device, n int32 aggregate
 * numbers; *n_agg (host): number of aggregates; *rounds (host, may be
 * NULL): rounds taken.  Synchronizes every round.  SPG_ERR_SHAPE if A is
 * not square; SPG_ERR_STATE if the rounds do not end (asymmetric pattern).
 * ------------------------------------------------------------------------ */
spg_status spg_mis2_aggregate(spg_plan plan, const spg_csr* A, uint64_t seed, uint8_t* in_mis, int32_t* agg,
                              int64_t* n_agg, int32_t* rounds);

/* R (n x n_agg) with R(i, agg[i]) = one, and R^T (n_agg x n), as canonical
 * CSR in caller-owned device arrays: r_rp n+1, r_col n, r_val n; rt_rp
 * n_agg+1, rt_col n, rt_val n (values typed by the semiring: 1.0, 1 or
 * true; r_val/rt_val may be NULL).  Synchronizes.  SPG_ERR_CAPACITY if an
 * aggregate holds more than 4096 vertices. */
spg_status spg_restriction(spg_plan plan, spg_semiring sr, int64_t n, int64_t n_agg, const int32_t* agg,
                           int64_t* r_rp, int32_t* r_col, void* r_val, int64_t* rt_rp, int32_t* rt_col,
                           void* rt_val);

const char* spg_status_string(spg_status s);
const char* spg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
