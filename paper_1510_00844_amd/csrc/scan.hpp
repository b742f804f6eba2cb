// Device prefix sum of int64 row counts into CSR row pointers: in place over
// rp[1..m] (inclusive), with rp[0] = 0.  Three launches: per-tile sums,
// one workgroup scanning the tile sums, per-tile rescan with the offset.
#pragma once
#include "common.hpp"

namespace spg {

constexpr int SCAN_NT = 256;
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = SCAN_NT * SCAN_PER;

__global__ void __launch_bounds__(SCAN_NT) k_scan_tiles(const int64_t* in, int64_t n, int64_t* tile_sums) {
    __shared__ int64_t red[SCAN_NT / SPG_WAVE + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    int64_t s = 0;
#pragma unroll
    for (int x = 0; x < SCAN_PER; ++x)
        if (base + x < n) s += in[base + x];
    int64_t total = block_reduce_add<SCAN_NT, int64_t>(s, red);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// Exclusive scan of ntiles sums in place by one workgroup; tile_sums[ntiles]
// receives the grand total.
__global__ void __launch_bounds__(SCAN_NT) k_scan_top(int64_t* tile_sums, int64_t ntiles) {
    __shared__ int64_t red[SCAN_NT / SPG_WAVE + 1];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < ntiles; base += SCAN_NT) {
        const int64_t idx = base + threadIdx.x;
        int64_t v = idx < ntiles ? tile_sums[idx] : 0;
        int64_t total;
        int64_t ex = block_exclusive_scan<SCAN_NT, int64_t>(v, &total, red);
        if (idx < ntiles) tile_sums[idx] = ex + carry;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sums[ntiles] = carry;
}

// out[x] = tile offset + inclusive prefix inside the tile.  in and out may
// alias (each element is read before it is written by the same thread).
__global__ void __launch_bounds__(SCAN_NT) k_scan_apply(const int64_t* in, int64_t n,
                                                        const int64_t* tile_off, int64_t* out) {
    __shared__ int64_t red[SCAN_NT / SPG_WAVE + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    int64_t v[SCAN_PER];
    int64_t s = 0;
#pragma unroll
    for (int x = 0; x < SCAN_PER; ++x) {
        v[x] = base + x < n ? in[base + x] : 0;
        s += v[x];
    }
    int64_t total;
    int64_t pre = block_exclusive_scan<SCAN_NT, int64_t>(s, &total, red) + tile_off[blockIdx.x];
#pragma unroll
    for (int x = 0; x < SCAN_PER; ++x) {
        pre += v[x];
        if (base + x < n) out[base + x] = pre;
    }
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

}  // namespace spg
