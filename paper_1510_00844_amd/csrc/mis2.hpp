// Distance-2 maximal independent sets and the aggregation that builds a
// restriction operator from them (Section 5.3, Algorithm 3).  Vectors are
// dense on the device: an absent entry of the algorithm's sparse vectors is
// the largest 64-bit key (or a zero flag).  Every row operation uses 8 lanes
// per row, so rows of any length are handled and short rows (stencils)
// still fill the waves.
#pragma once
#include "common.hpp"

namespace spg {

constexpr uint64_t MIS_ABSENT = ~0ull;
constexpr int MIS_LANES = 8;  // lanes per row

// SplitMix64 (Steele, Lea, Flood): the output for generator state x, i.e.
// the state advanced by the golden gamma and passed through the mixer.
__device__ inline uint64_t splitmix64_output(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Round-r key of vertex v: random high half, the vertex id as the low half
// (keys never tie).
__device__ inline uint64_t mis_key(uint64_t seed, int32_t round, int64_t v) {
    const uint64_t h = splitmix64_output(seed ^ (((uint64_t)(uint32_t)round << 32) | (uint64_t)v));
    return (h & 0xFFFFFFFF00000000ull) | (uint64_t)v;
}

// Key by which an unassigned vertex v ranks an assigned neighbour u.
__device__ inline uint64_t choice_key(uint64_t seed, int64_t v, int64_t u) {
    return splitmix64_output(seed ^ 0x5DEECE66D2B9A1F3ull ^ (((uint64_t)v << 32) | (uint64_t)u));
}

template <typename T, class Op>
__device__ inline T group_reduce(T v, Op op) {
#pragma unroll
    for (int d = MIS_LANES / 2; d > 0; d >>= 1) v = op(v, __shfl_xor(v, d, SPG_WAVE));
    return v;
}

__global__ void __launch_bounds__(256) k_mis_keys(int64_t n, const uint8_t* cand, uint64_t seed, int32_t round,
                                                  uint64_t* key) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n) key[v] = cand[v] ? mis_key(seed, round, v) : MIS_ABSENT;
}

// y(i) = min over stored A(i,j) of x(j)   (semiring (min, select2nd))
__global__ void __launch_bounds__(256) k_mis_row_min(Csr A, const uint64_t* x, uint64_t* y) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / MIS_LANES;
    const int gl = threadIdx.x % MIS_LANES;
    uint64_t m = MIS_ABSENT;
    if (i < A.nrows)
        for (int64_t p = A.rp[i] + gl; p < A.rp[i + 1]; p += MIS_LANES) {
            const uint64_t t = x[A.col[p]];
            m = t < m ? t : m;
        }
    m = group_reduce(m, [](uint64_t a, uint64_t b) { return a < b ? a : b; });
    if (i < A.nrows && gl == 0) y[i] = m;
}

// Second hop and selection: minadj = min(m1(i), min over A(i,j) of m1(j));
// a candidate whose key is not larger joins (newS) and stops being a
// candidate.
__global__ void __launch_bounds__(256) k_mis_select(Csr A, const uint64_t* key, const uint64_t* m1, uint8_t* cand,
                                                    uint8_t* news) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / MIS_LANES;
    const int gl = threadIdx.x % MIS_LANES;
    uint64_t m = MIS_ABSENT;
    if (i < A.nrows)
        for (int64_t p = A.rp[i] + gl; p < A.rp[i + 1]; p += MIS_LANES) {
            const uint64_t t = m1[A.col[p]];
            m = t < m ? t : m;
        }
    m = group_reduce(m, [](uint64_t a, uint64_t b) { return a < b ? a : b; });
    if (i < A.nrows && gl == 0) {
        const uint64_t mn = m1[i] < m ? m1[i] : m;
        const bool c = cand[i] != 0;
        const bool joins = c && key[i] <= mn;
        news[i] = joins ? 1 : 0;
        if (joins) cand[i] = 0;
    }
}

// y(i) = OR over stored A(i,j) of x(j)
__global__ void __launch_bounds__(256) k_mis_row_any(Csr A, const uint8_t* x, uint8_t* y) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / MIS_LANES;
    const int gl = threadIdx.x % MIS_LANES;
    int hit = 0;
    if (i < A.nrows)
        for (int64_t p = A.rp[i] + gl; p < A.rp[i + 1] && !hit; p += MIS_LANES) hit = x[A.col[p]] ? 1 : 0;
    hit = group_reduce(hit, [](int a, int b) { return a | b; });
    if (i < A.nrows && gl == 0) y[i] = (uint8_t)hit;
}

// Second hop of the new vertices' neighbourhood, pruning of the candidates,
// MIS-2 update, and the count of remaining candidates.
__global__ void __launch_bounds__(256) k_mis_prune(Csr A, const uint8_t* a1, const uint8_t* news, uint8_t* cand,
                                                   uint8_t* in_mis, int32_t* remaining) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / MIS_LANES;
    const int gl = threadIdx.x % MIS_LANES;
    int hit = 0;
    if (i < A.nrows)
        for (int64_t p = A.rp[i] + gl; p < A.rp[i + 1] && !hit; p += MIS_LANES) hit = a1[A.col[p]] ? 1 : 0;
    hit = group_reduce(hit, [](int a, int b) { return a | b; });
    bool left = false;
    if (i < A.nrows && gl == 0) {
        if (hit || a1[i]) cand[i] = 0;
        if (news[i]) in_mis[i] = 1;
        left = cand[i] != 0;
    }
    const uint64_t b = __ballot(left);
    if (lane_id() == 0 && b) atomicAdd(remaining, __popcll(b));
}

// flags[v + 1] = in_mis(v), for the exclusive scan that numbers the roots
__global__ void __launch_bounds__(256) k_mis_flags(int64_t n, const uint8_t* in_mis, int64_t* flags) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n) flags[v + 1] = in_mis[v] ? 1 : 0;
}

// Roots take their number; their neighbours join them (a vertex is adjacent
// to at most one root); others stay -1.
__global__ void __launch_bounds__(256) k_agg_roots(Csr A, const uint8_t* in_mis, const int64_t* root_id,
                                                   int32_t* agg1) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / MIS_LANES;
    const int gl = threadIdx.x % MIS_LANES;
    int64_t r = -1;
    if (i < A.nrows && !in_mis[i])
        for (int64_t p = A.rp[i] + gl; p < A.rp[i + 1]; p += MIS_LANES) {
            const int64_t j = A.col[p];
            if (in_mis[j]) r = j > r ? j : r;
        }
    r = group_reduce(r, [](int64_t a, int64_t b) { return a > b ? a : b; });
    if (i < A.nrows && gl == 0) agg1[i] = in_mis[i] ? (int32_t)root_id[i] : (r >= 0 ? (int32_t)root_id[r] : -1);
}

// Unassigned vertices join the assigned neighbour with the smallest
// (choice key, neighbour) pair; *unassigned counts any left over.
__global__ void __launch_bounds__(256) k_agg_rest(Csr A, const int32_t* agg1, uint64_t seed, int32_t* agg,
                                                  int32_t* unassigned) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / MIS_LANES;
    const int gl = threadIdx.x % MIS_LANES;
    const bool need = i < A.nrows && agg1[i] < 0;
    uint64_t bk = MIS_ABSENT;
    int64_t bj = -1;
    if (need)
        for (int64_t p = A.rp[i] + gl; p < A.rp[i + 1]; p += MIS_LANES) {
            const int64_t j = A.col[p];
            if (agg1[j] < 0) continue;
            const uint64_t k = choice_key(seed, i, j);
            if (bj < 0 || k < bk || (k == bk && j < bj)) {
                bk = k;
                bj = j;
            }
        }
#pragma unroll
    for (int d = MIS_LANES / 2; d > 0; d >>= 1) {
        const uint64_t ok = __shfl_xor(bk, d, SPG_WAVE);
        const int64_t oj = __shfl_xor(bj, d, SPG_WAVE);
        if (oj >= 0 && (bj < 0 || ok < bk || (ok == bk && oj < bj))) {
            bk = ok;
            bj = oj;
        }
    }
    if (i < A.nrows && gl == 0) {
        const int32_t a = need ? (bj >= 0 ? agg1[bj] : -1) : agg1[i];
        agg[i] = a;
        if (a < 0) atomicAdd(unassigned, 1);
    }
}

// R (n x n_agg): one entry per row at the aggregate; counts of R^T's rows.
template <int SR>
__global__ void __launch_bounds__(256) k_restrict_rows(int64_t n, const int32_t* agg, int64_t* r_rp, int32_t* r_col,
                                                       void* r_val, int64_t* rt_cnt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > n) return;
    r_rp[i] = i;
    if (i == n) return;
    r_col[i] = agg[i];
    if (r_val) {
        if (SR == SR_F64) ((double*)r_val)[i] = 1.0;
        else if (SR == SR_I64) ((int64_t*)r_val)[i] = 1;
        else ((uint8_t*)r_val)[i] = 1;
    }
    atomicAdd((unsigned long long*)&rt_cnt[agg[i] + 1], 1ull);
}

// R^T: vertex i goes to row agg(i) (any order; rows are sorted afterwards).
template <int SR>
__global__ void __launch_bounds__(256) k_restrict_cols(int64_t n, const int32_t* agg, const int64_t* rt_rp,
                                                       int64_t* cursor, int32_t* rt_col, void* rt_val) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t a = agg[i];
    const int64_t q = rt_rp[a] + (int64_t)atomicAdd((unsigned long long*)&cursor[a], 1ull);
    rt_col[q] = (int32_t)i;
    if (rt_val) {
        if (SR == SR_F64) ((double*)rt_val)[q] = 1.0;
        else if (SR == SR_I64) ((int64_t*)rt_val)[q] = 1;
        else ((uint8_t*)rt_val)[q] = 1;
    }
}

// Sort each row's column indices (values are all equal): a wave per row,
// register sort up to 64 entries, LDS sort up to 4096; *too_long counts rows
// beyond that.
__global__ void __launch_bounds__(64) k_sort_row_cols(int64_t nrows, const int64_t* rp, int32_t* col,
                                                      int32_t* too_long) {
    __shared__ uint64_t keys[4096];
    const int64_t r = blockIdx.x;
    if (r >= nrows) return;
    const int64_t s = rp[r];
    const int len = (int)(rp[r + 1] - s);
    const int lane = lane_id();
    if (len <= SPG_WAVE) {
        uint64_t k = lane < len ? (uint64_t)(uint32_t)col[s + lane] : ~0ull;
        k = wave_bitonic_sort_u64(k);
        if (lane < len) col[s + lane] = (int32_t)k;
        return;
    }
    if (len > 4096) {
        if (lane == 0) atomicAdd(too_long, 1);
        return;
    }
    int P = 1;
    while (P < len) P <<= 1;
    for (int t = lane; t < P; t += SPG_WAVE) keys[t] = t < len ? (uint64_t)(uint32_t)col[s + t] : ~0ull;
    __syncthreads();
    block_bitonic_sort_u64<SPG_WAVE>(keys, P);
    for (int t = lane; t < len; t += SPG_WAVE) col[s + t] = (int32_t)keys[t];
}

}  // namespace spg
