// Multiway merge with reduction (Section 4.3; LocalMerge of Algorithm 2):
// out = entry-wise semiring sum of c layers of equal shape.  Row i of the
// output is the sorted union of the c sorted segments layer_l(i,:), with
// values of equal columns combined in ascending layer order.  The paper
// merges triples with a size-c heap per thread; here a row is merged by a
// wave (<= 64 entries in all layers), a workgroup (<= 4096 entries: LDS
// bitonic sort of (column, position) keys, positions taken layer by layer so
// ties keep layer order), or, for longer rows, a workgroup sweeping column
// chunks with an LDS dense accumulator, each layer's chunk range found by
// binary search (the column-range split of Section 4.3).
#pragma once
#include "products.hpp"
#include "rowinfo.hpp"

namespace spg {

struct LayerDesc {
    const int64_t* rp;
    const int32_t* col;
    const void* val;
};

constexpr int MBIN_EMPTY = 0, MBIN_SMALL = 1, MBIN_LDS = 2, MBIN_DENSE = 3;
constexpr int MERGE_LDS_MAX = 4096;

__global__ void __launch_bounds__(256) k_merge_rowinfo(int64_t m, int32_t c, const LayerDesc* layers,
                                                       int64_t* total_len, uint8_t* bin,
                                                       int64_t* bin_stats) {
    __shared__ int s_hist[NBINS];
    __shared__ int64_t s_len[NBINS];
    if (threadIdx.x < NBINS) {
        s_hist[threadIdx.x] = 0;
        s_len[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) {
        int64_t L = 0;
        for (int l = 0; l < c; ++l) L += layers[l].rp[i + 1] - layers[l].rp[i];
        total_len[i] = L;
        int b = L == 0 ? MBIN_EMPTY : (L <= SPG_WAVE ? MBIN_SMALL : (L <= MERGE_LDS_MAX ? MBIN_LDS : MBIN_DENSE));
        bin[i] = (uint8_t)b;
        atomicAdd(&s_hist[b], 1);
        atomicAdd((unsigned long long*)&s_len[b], (unsigned long long)L);
    }
    __syncthreads();
    if (threadIdx.x < NBINS && s_hist[threadIdx.x]) {
        atomicAdd((unsigned long long*)&bin_stats[threadIdx.x], (unsigned long long)s_hist[threadIdx.x]);
        atomicAdd((unsigned long long*)&bin_stats[NBINS + threadIdx.x], (unsigned long long)s_len[threadIdx.x]);
    }
}

// cnt != nullptr: count pass; otherwise fill pass into out_rp/out_col/out_val.
template <int SR>
__global__ void __launch_bounds__(256) k_merge_small(int32_t c, const LayerDesc* layers,
                                                     const int32_t* rows, int32_t nrows, int64_t* cnt,
                                                     const int64_t* out_rp, int32_t* out_col,
                                                     void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nrows) return;
    const int64_t i = rows[r];
    const int lane = lane_id();
    int pos = 0, my_l = -1;
    int64_t my_q = 0;
    for (int l = 0; l < c; ++l) {
        const int64_t rs = layers[l].rp[i];
        const int len = (int)(layers[l].rp[i + 1] - rs);
        if (lane >= pos && lane < pos + len) {
            my_l = l;
            my_q = rs + (lane - pos);
        }
        pos += len;
    }
    uint64_t key = ~0ull;
    V v = S::zero();
    if (my_l >= 0) {
        key = ((uint64_t)(uint32_t)layers[my_l].col[my_q] << 6) | (uint64_t)lane;
        if (!cnt) v = S::load(layers[my_l].val, my_q);
    }
    key = wave_bitonic_sort_u64(key);
    const bool valid = key != ~0ull;
    const uint64_t col = key >> 6;
    const uint64_t prev = __shfl_up(col, 1, SPG_WAVE);
    const bool head = valid && (lane == 0 || prev != col);
    const uint64_t heads = __ballot(head);
    if (cnt) {
        if (lane == 0) cnt[i] = __popcll(heads);
        return;
    }
    v = __shfl(v, (int)(key & 63), SPG_WAVE);
    V acc = v;
    bool open = head;
    for (int s = 1; s < SPG_WAVE; ++s) {
        if (!__any(open)) break;
        uint64_t ncol = __shfl_down(col, s, SPG_WAVE);
        V nv = __shfl_down(v, s, SPG_WAVE);
        bool nvalid = __shfl_down((int)valid, s, SPG_WAVE) != 0;
        open = open && (lane + s < SPG_WAVE) && nvalid && ncol == col;
        if (open) acc = S::add(acc, nv);
    }
    if (head) {
        const int64_t o = out_rp[i] + lanes_below(heads);
        out_col[o] = (int32_t)col;
        if (out_val) S::store(out_val, o, acc);
    }
}

template <int SR, int NT>
__global__ void __launch_bounds__(NT) k_merge_lds(int32_t c, const LayerDesc* layers,
                                                  const int32_t* rows, const int64_t* total_len,
                                                  int64_t* cnt, const int64_t* out_rp,
                                                  int32_t* out_col, void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    constexpr int LMAX = MERGE_LDS_MAX;
    constexpr int PER = LMAX / NT;
    __shared__ uint64_t keys[LMAX];
    __shared__ V vals[LMAX];
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    const int64_t i = rows[blockIdx.x];
    const int L = (int)total_len[i];
    int P = 1;
    while (P < L) P <<= 1;
    int pos = 0;
    for (int l = 0; l < c; ++l) {
        const int64_t rs = layers[l].rp[i];
        const int len = (int)(layers[l].rp[i + 1] - rs);
        for (int t = threadIdx.x; t < len; t += NT) {
            const int idx = pos + t;
            keys[idx] = ((uint64_t)(uint32_t)layers[l].col[rs + t] << 12) | (uint64_t)idx;
            if (!cnt) vals[idx] = S::load(layers[l].val, rs + t);
        }
        pos += len;
    }
    for (int t = L + threadIdx.x; t < P; t += NT) keys[t] = ~0ull;
    __syncthreads();
    block_bitonic_sort_u64<NT>(keys, P);
    // heads over positions [t*PER, (t+1)*PER)
    int32_t mine = 0;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const int x = threadIdx.x * PER + s;
        if (x < L) {
            const uint64_t col = keys[x] >> 12;
            mine += (x == 0 || (keys[x - 1] >> 12) != col) ? 1 : 0;
        }
    }
    int32_t heads_total;
    int32_t rank = block_exclusive_scan<NT, int32_t>(mine, &heads_total, red);
    if (cnt) {
        if (threadIdx.x == 0) cnt[i] = heads_total;
        return;
    }
    const int64_t o = out_rp[i];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const int x = threadIdx.x * PER + s;
        if (x < L) {
            const uint64_t col = keys[x] >> 12;
            if (x == 0 || (keys[x - 1] >> 12) != col) {
                V acc = vals[keys[x] & 0xfff];
                for (int y = x + 1; y < L && (keys[y] >> 12) == col; ++y)
                    acc = S::add(acc, vals[keys[y] & 0xfff]);
                out_col[o + rank] = (int32_t)col;
                if (out_val) S::store(out_val, o + rank, acc);
                ++rank;
            }
        }
    }
}

template <int SR, int NT, int W>
__global__ void __launch_bounds__(NT) k_merge_dense(int32_t c, const LayerDesc* layers,
                                                    const int32_t* rows, int64_t ncols, int64_t* cnt,
                                                    const int64_t* out_rp, int32_t* out_col,
                                                    void* out_val) {
    typedef Sr<SR> S;
    typedef typename S::acc_t V;
    constexpr int NWD = W / 32;
    __shared__ V acc[W];
    __shared__ uint32_t bits[NWD];
    __shared__ int32_t wpre[NWD];
    __shared__ int8_t s_layer[NT];
    __shared__ ProductLds<NT> L;
    __shared__ int32_t red[NT / SPG_WAVE + 1];
    const int64_t i = rows[blockIdx.x];
    const int P = (int)((ncols + W - 1) / W);
    int64_t off = cnt ? 0 : out_rp[i];
    int64_t count = 0;
    for (int ch = 0; ch < P; ++ch) {
        for (int t = threadIdx.x; t < W; t += NT) acc[t] = S::zero();
        for (int t = threadIdx.x; t < NWD; t += NT) bits[t] = 0u;
        __syncthreads();
        const int64_t cbase = (int64_t)ch * W;
        // "A entries" of the product enumeration are the c layers
        for_each_product<NT>(
            0, c, L,
            [&](int64_t l, int64_t& bs, int32_t& len) {
                const int64_t rs = layers[l].rp[i], re = layers[l].rp[i + 1];
                const int64_t lo = lower_bound_col(layers[l].col, rs, re, cbase);
                const int64_t hi = lower_bound_col(layers[l].col, lo, re, cbase + W);
                bs = lo;
                len = (int32_t)(hi - lo);
            },
            [&](int t, int64_t l) { s_layer[t] = (int8_t)l; },
            [&](int t, int64_t, int64_t q) {
                const int l = s_layer[t];
                const int32_t j = (int32_t)(layers[l].col[q] - cbase);
                if (!cnt) S::lds_add(&acc[j], S::load(layers[l].val, q));
                atomicOr(&bits[j >> 5], 1u << (j & 31));
            });
        constexpr int WPT = (NWD + NT - 1) / NT;
        int32_t wc[WPT];
        int32_t s = 0;
#pragma unroll
        for (int x = 0; x < WPT; ++x) {
            int w = threadIdx.x * WPT + x;
            wc[x] = w < NWD ? __popc(bits[w]) : 0;
            s += wc[x];
        }
        int32_t chunk_total;
        int32_t pre = block_exclusive_scan<NT, int32_t>(s, &chunk_total, red);
#pragma unroll
        for (int x = 0; x < WPT; ++x) {
            int w = threadIdx.x * WPT + x;
            if (w < NWD) wpre[w] = pre;
            pre += wc[x];
        }
        __syncthreads();
        if (!cnt && chunk_total) {
            for (int j = threadIdx.x; j < W; j += NT) {
                const uint32_t wbits = bits[j >> 5];
                const uint32_t b = 1u << (j & 31);
                if (wbits & b) {
                    const int64_t o = off + wpre[j >> 5] + __popc(wbits & (b - 1));
                    out_col[o] = (int32_t)(cbase + j);
                    if (out_val) S::store(out_val, o, acc[j]);
                }
            }
        }
        off += chunk_total;
        count += chunk_total;
        __syncthreads();
    }
    if (cnt && threadIdx.x == 0) cnt[i] = count;
}

}  // namespace spg
