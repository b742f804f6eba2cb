// Single-pass product with predicted row sizes.
//
// The symbolic pass of the two-phase method exists only to size each output
// row.  Here the predictor (mlp.hpp) gives every row a capacity instead; the
// numeric kernels write each row into a padded slot of that capacity and
// report the row's true count.  A row whose true count exceeds its capacity
// (or which is too large for any single-pass accumulator) is recomputed by
// the exact two-phase method; then the exact counts are scanned and the
// slots are compacted into canonical CSR.  Every prediction is checked
// against the exact count.
#pragma once
#include "mlp.hpp"
#include "numeric.hpp"
#include "rowinfo.hpp"

namespace spg {

// Rows whose size the predictor decides (not empty, not single-entry, more
// products than the one-wave bin).
__device__ inline bool row_is_predicted(int sym_bin_id) {
    return sym_bin_id != BIN_EMPTY && sym_bin_id != BIN_TINY && sym_bin_id != BIN_SMALL;
}

__device__ inline void row_features(int64_t annz, int64_t flops, int32_t maxb, float& x0, float& x1, float& x2) {
    x0 = log1pf((float)annz);
    x1 = log1pf((float)flops);
    x2 = log1pf((float)maxb);
}

// Training data from a finished symbolic pass: features and log1p of the
// exact counts of the predicted rows, compacted (order unspecified).
__global__ void __launch_bounds__(256) k_train_rows(int64_t m, const int64_t* a_beg, const int64_t* a_end,
                                                    const int64_t* flops, const int32_t* maxb, int32_t small_max,
                                                    int64_t min_flops, const int64_t* c_rp, float* x, float* t,
                                                    unsigned long long* count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    // predicted rows: not empty, more than one A entry, more than one wave of products
    if (flops[i] <= small_max || flops[i] < min_flops || a_end[i] - a_beg[i] < 2) return;
    const unsigned long long slot = atomicAdd(count, 1ull);
    float x0, x1, x2;
    row_features(a_end[i] - a_beg[i], flops[i], maxb[i], x0, x1, x2);
    x[3 * slot] = x0;
    x[3 * slot + 1] = x1;
    x[3 * slot + 2] = x2;
    t[slot] = log1pf((float)(c_rp[i + 1] - c_rp[i]));
}

struct LearnedParams {
    float margin;          // capacity = (1 + margin) * prediction + 8, then clamped
    int32_t use_mlp;       // 0: capacity = upper bound min(flops, n)
    int32_t fused_max_log2;  // largest rank-space capacity of the fused bitmap kernel (0 = none)
    int32_t hash_max_nnz;  // hash tables hold up to this many outputs
};

// Capacity and single-pass bin of every row.  Bins: EMPTY, TINY, SMALL as
// in the numeric pass; HASH by capacity; RANK0.. = fused bitmap kernel by
// capacity; DENSE = no single-pass accumulator fits, exact method.
__global__ void __launch_bounds__(256) k_learned_classify(int64_t m, int64_t n, const float* params,
                                                          LearnedParams lp, BinParams bp, const int64_t* a_beg,
                                                          const int64_t* a_end, const int64_t* flops,
                                                          const int32_t* maxb, uint8_t* bin, int64_t* cap,
                                                          int64_t* cnt, int64_t* bin_stats) {
    __shared__ float s_p[MLP_NPARAMS];
    __shared__ int s_hist[NBINS];
    __shared__ int64_t s_flops[NBINS];
    if (threadIdx.x < NBINS) {
        s_hist[threadIdx.x] = 0;
        s_flops[threadIdx.x] = 0;
    }
    if (lp.use_mlp) load_params(s_p, params);
    else __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) {
        const int sb = bin[i];  // symbolic bin from the row analysis
        const int64_t an = a_end[i] - a_beg[i];
        const int64_t f = flops[i];
        int b;
        int64_t c;
        if (!row_is_predicted(sb)) {
            b = sb;
            c = f;  // exact for TINY (and EMPTY); an upper bound for SMALL
            if (sb == BIN_EMPTY) cnt[i] = 0;
            if (sb == BIN_TINY) cnt[i] = f;
        } else {
            const int64_t hi = f < n ? f : n;
            if (lp.use_mlp) {
                float x0, x1, x2;
                row_features(an, f, maxb[i], x0, x1, x2);
                const float y = mlp_eval(s_p, x0, x1, x2);
                const double pred = expm1((double)fminf(y, 40.f));
                double cd = ceil((1.0 + (double)lp.margin) * pred) + 8.0;
                c = cd > (double)hi ? hi : (int64_t)cd;
            } else {
                c = hi;
            }
            if (c < maxb[i]) c = maxb[i];
            if (c > hi) c = hi;
            const bool bitmap_cheaper = bp.dense_ok && f * 32 >= n;
            if (c <= lp.hash_max_nnz && !bitmap_cheaper) {
                int lg = ceil_log2_i64(2 * c);
                if (lg < HASH_MIN_LOG2) lg = HASH_MIN_LOG2;
                b = BIN_HASH0 + (lg - HASH_MIN_LOG2);
            } else if (bp.dense_ok && lp.fused_max_log2 && c <= (1ll << lp.fused_max_log2)) {
                int lg = ceil_log2_i64(c);
                if (lg < RANK_MIN_LOG2) lg = RANK_MIN_LOG2;
                b = BIN_RANK0 + (lg - RANK_MIN_LOG2);
            } else {
                b = BIN_DENSE;
            }
        }
        bin[i] = (uint8_t)b;
        cap[i] = b == BIN_DENSE ? 0 : c;  // exact-method rows get no slot
        atomicAdd(&s_hist[b], 1);
        atomicAdd((unsigned long long*)&s_flops[b], (unsigned long long)f);
    }
    __syncthreads();
    if (threadIdx.x < NBINS && s_hist[threadIdx.x]) {
        atomicAdd((unsigned long long*)&bin_stats[threadIdx.x], (unsigned long long)s_hist[threadIdx.x]);
        atomicAdd((unsigned long long*)&bin_stats[NBINS + threadIdx.x], (unsigned long long)s_flops[threadIdx.x]);
    }
}

// Fused bitmap + rank kernel for rows whose count is not known: build the
// row's bitmap, count it, and if the count fits the slot, emit columns from
// the bitmap and accumulate values by rank (as the two-phase bitmap and rank
// kernels do, without the bitmap's round trip through memory).
// Dynamic LDS: nwords 64-bit words, then `acc_cap` accumulators.
template <int SR, int NT, int GM>
__global__ void __launch_bounds__(NT) k_learned_fused(Csr A, Csr B, const int32_t* rows, const int64_t* a_beg,
                                                      const int64_t* a_end, int32_t nwords, int64_t acc_cap,
                                                      const int64_t* slot, int64_t* cnt_out, int32_t* c_col,
                                                      void* c_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    extern __shared__ uint64_t dyn[];
    uint64_t* bw = dyn;
    uint32_t* bm = reinterpret_cast<uint32_t*>(dyn);  // bits first, in the low words
    V* acc = reinterpret_cast<V*>(dyn + nwords);
    __shared__ V s_av[NT];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    const int64_t i = rows[blockIdx.x];
    const int64_t off = slot[i];
    const int64_t room = slot[i + 1] - off;
    // bitmap in the first nwords 32-bit words
    for (int t = threadIdx.x; t < nwords; t += NT) bm[t] = 0u;
    __syncthreads();
    for_each_product_gm<NT, GM>(
        a_beg[i], a_end[i], L,
        [&](int64_t p, int64_t& bs, int32_t& len) {
            int64_t k = A.col[p];
            bs = B.rp[k];
            len = (int32_t)(B.rp[k + 1] - bs);
        },
        [&](int, int64_t) {},
        [&](int64_t q) { return (uint32_t)B.col[q]; },
        [&](int, uint32_t j) { atomicOr(&bm[j >> 5], 1u << (j & 31)); });
    // spread to (prefix << 32 | bits): read own words, then rewrite in place
    const int wpt = (nwords + NT - 1) / NT;
    const int w0 = threadIdx.x * wpt;
    const int w1 = w0 + wpt < nwords ? w0 + wpt : nwords;
    uint32_t mine[8];  // wpt <= 8 (nwords <= 8 * NT)
    int32_t part = 0;
    for (int w = w0, x = 0; w < w1; ++w, ++x) {
        mine[x] = bm[w];
        part += __popc(mine[x]);
    }
    int32_t total;
    int32_t run = block_exclusive_scan<NT, int32_t>(part, &total, red);  // barriers: all reads done
    if (threadIdx.x == 0) cnt_out[i] = total;
    if (total > room || total > acc_cap) return;  // overflow: the exact method redoes this row
    for (int w = w0, x = 0; w < w1; ++w, ++x) {
        uint32_t bits = mine[x];
        bw[w] = ((uint64_t)(uint32_t)run << 32) | bits;
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            c_col[off + run] = w * 32 + b;
            ++run;
        }
    }
    for (int r = threadIdx.x; r < total; r += NT) acc[r] = S::zero();
    __syncthreads();
    for_each_product_gm<NT, GM>(
        a_beg[i], a_end[i], L,
        [&](int64_t p, int64_t& bs, int32_t& len) {
            int64_t k = A.col[p];
            bs = B.rp[k];
            len = (int32_t)(B.rp[k + 1] - bs);
        },
        [&](int t, int64_t p) { s_av[t] = S::load(A.val, p); },
        [&](int64_t q) { return BEntry<V>{B.col[q], S::load(B.val, q)}; },
        [&](int t, const BEntry<V>& x) {
            const uint32_t j = (uint32_t)x.col;
            const uint64_t wd = bw[j >> 5];
            const int32_t rank = (int32_t)(wd >> 32) + __popc((uint32_t)wd & ((1u << (j & 31)) - 1u));
            S::lds_add(&acc[rank], S::mul(s_av[t], x.val));
        });
    if (c_val)
        for (int r = threadIdx.x; r < total; r += NT) S::store(c_val, off + r, acc[r]);
}

// Rows the exact method must (re)compute: DENSE rows, and predicted rows
// whose true count exceeded their capacity.  Appends to `list`.
__global__ void __launch_bounds__(256) k_fallback_rows(int64_t m, const uint8_t* bin, const int64_t* cap,
                                                       const int64_t* cnt, int32_t* list, int32_t* count,
                                                       uint8_t* redo) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int b = bin[i];
    const bool r = b == BIN_DENSE || (b != BIN_EMPTY && b != BIN_TINY && b != BIN_SMALL && cnt[i] > cap[i]);
    redo[i] = r ? 1 : 0;
    if (r) list[atomicAdd(count, 1)] = (int32_t)i;
}

// Row lengths of the listed rows of A (first pass of gathering them into a
// compact CSR).
__global__ void __launch_bounds__(256) k_gather_len(const int64_t* a_rp, const int32_t* list, int32_t nl,
                                                    int64_t* len) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < nl) len[r] = a_rp[list[r] + 1] - a_rp[list[r]];
}

// Copy the listed rows of A into the compact CSR (one wave per row).
template <int SR>
__global__ void __launch_bounds__(256) k_gather_rows(Csr A, const int32_t* list, int32_t nl, const int64_t* sub_rp,
                                                     int32_t* sub_col, void* sub_val) {
    typedef Sr<SR> S;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nl) return;
    const int64_t i = list[r];
    const int64_t s = A.rp[i], e = A.rp[i + 1], o = sub_rp[r] - s;
    for (int64_t p = s + lane_id(); p < e; p += SPG_WAVE) {
        sub_col[o + p] = A.col[p];
        if (sub_val) {
            if (SR == SR_F64) ((double*)sub_val)[o + p] = ((const double*)A.val)[p];
            else if (SR == SR_I64) ((int64_t*)sub_val)[o + p] = ((const int64_t*)A.val)[p];
            else ((uint8_t*)sub_val)[o + p] = A.val ? ((const uint8_t*)A.val)[p] : (uint8_t)1;
        }
    }
}

// Exact counts of the recomputed rows back into the per-row counts.
__global__ void __launch_bounds__(256) k_scatter_counts(const int32_t* list, int32_t nl, const int64_t* sub_rp,
                                                        int64_t* cnt) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < nl) cnt[list[r]] = sub_rp[r + 1] - sub_rp[r];
}

// Final output offset of every listed row (the recomputed rows then write
// straight into the full product).
__global__ void __launch_bounds__(256) k_gather_offsets(const int32_t* list, int32_t nl, const int64_t* c_rp,
                                                        int64_t* pos) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < nl) pos[r] = c_rp[list[r]];
}

// Compaction: one wave per row copies `len` entries from src offset to the
// final offset.  mode 0: rows 0..m-1 from their slots, skipping redo rows;
// mode 1: listed rows from the recomputed compact result.
template <int SR>
__global__ void __launch_bounds__(256) k_copy_rows(int64_t nrows, const int32_t* list, const uint8_t* redo,
                                                   const int64_t* src_off, const int64_t* dst_rp,
                                                   const int32_t* src_col, const void* src_val, int32_t* dst_col,
                                                   void* dst_val) {
    // one workgroup per row (grid-stride), four entries in flight per thread
    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t i = list ? list[r] : r;
        if (!list && redo[i]) continue;
        const int64_t s = list ? src_off[r] : src_off[i];
        const int64_t d = dst_rp[i];
        const int64_t len = dst_rp[i + 1] - d;
        for (int64_t x0 = 0; x0 < len; x0 += 4 * 256) {
            int32_t c[4];
            uint64_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t x = x0 + u * 256 + threadIdx.x;
                if (x < len) {
                    c[u] = src_col[s + x];
                    if (dst_val) v[u] = SR == SR_BOOL ? ((const uint8_t*)src_val)[s + x] : ((const uint64_t*)src_val)[s + x];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t x = x0 + u * 256 + threadIdx.x;
                if (x < len) {
                    dst_col[d + x] = c[u];
                    if (dst_val) {
                        if (SR == SR_BOOL) ((uint8_t*)dst_val)[d + x] = (uint8_t)v[u];
                        else ((uint64_t*)dst_val)[d + x] = v[u];
                    }
                }
            }
        }
    }
}

}  // namespace spg
