// Shared device helpers for the gfx950 SpGEMM kernels: semiring value
// types, wave and workgroup scans, LDS bitonic sort.  Wavefronts are 64
// lanes wide on CDNA; every helper here assumes that.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SPG_WAVE 64

namespace spg {

struct Csr {
    int64_t nrows, ncols, nnz;
    const int64_t* rp;
    const int32_t* col;
    const void* val;
};

// ---------------------------------------------------------------------------
// Semirings (Section 2: matrices over a semiring S).
//   acc_t : accumulator type held in LDS / registers
//   load  : stored value -> accumulator (boolean NULL array = all true)
//   mul   : semiring multiply,  add : semiring add
//   lds_add: atomic semiring add into LDS (workgroup scope)
// ---------------------------------------------------------------------------
enum { SR_F64 = 0, SR_I64 = 1, SR_BOOL = 2 };

template <int SR> struct Sr;

template <> struct Sr<SR_F64> {
    typedef double acc_t;
    __device__ static inline acc_t load(const void* v, int64_t p) { return ((const double*)v)[p]; }
    __device__ static inline acc_t mul(acc_t a, acc_t b) { return a * b; }
    __device__ static inline acc_t add(acc_t a, acc_t b) { return a + b; }
    __device__ static inline acc_t zero() { return 0.0; }
    __device__ static inline void lds_add(acc_t* p, acc_t v) {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ static inline void store(void* out, int64_t p, acc_t v) { ((double*)out)[p] = v; }
};

template <> struct Sr<SR_I64> {
    typedef unsigned long long acc_t;  // two's-complement wrap-around
    __device__ static inline acc_t load(const void* v, int64_t p) {
        return (acc_t)((const int64_t*)v)[p];
    }
    __device__ static inline acc_t mul(acc_t a, acc_t b) { return a * b; }
    __device__ static inline acc_t add(acc_t a, acc_t b) { return a + b; }
    __device__ static inline acc_t zero() { return 0ull; }
    __device__ static inline void lds_add(acc_t* p, acc_t v) {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ static inline void store(void* out, int64_t p, acc_t v) {
        ((int64_t*)out)[p] = (int64_t)v;
    }
};

template <> struct Sr<SR_BOOL> {
    typedef uint32_t acc_t;  // 0/1
    __device__ static inline acc_t load(const void* v, int64_t p) {
        return v ? (((const uint8_t*)v)[p] != 0 ? 1u : 0u) : 1u;
    }
    __device__ static inline acc_t mul(acc_t a, acc_t b) { return a & b; }
    __device__ static inline acc_t add(acc_t a, acc_t b) { return a | b; }
    __device__ static inline acc_t zero() { return 0u; }
    __device__ static inline void lds_add(acc_t* p, acc_t v) {
        if (v) __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ static inline void store(void* out, int64_t p, acc_t v) {
        ((uint8_t*)out)[p] = (uint8_t)v;
    }
};

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

template <typename T>
__device__ inline T wave_inclusive_scan_add(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < SPG_WAVE; d <<= 1) {
        T o = __shfl_up(v, d, SPG_WAVE);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ inline T wave_reduce_add(T v) {
#pragma unroll
    for (int d = SPG_WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, SPG_WAVE);
    return v;
}

template <typename T>
__device__ inline T wave_reduce_max(T v) {
#pragma unroll
    for (int d = SPG_WAVE / 2; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, SPG_WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// Number of set lanes strictly below this lane in a 64-bit mask.
__device__ inline int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// ---------------------------------------------------------------------------
// Workgroup exclusive scan of one value per thread.  `tmp` must hold
// NT/64 + 1 elements of T.  Returns the exclusive prefix; *total gets the
// sum over the workgroup.  Contains barriers: all threads must call it.
// ---------------------------------------------------------------------------
template <int NT, typename T>
__device__ inline T block_exclusive_scan(T v, T* total, T* tmp) {
    constexpr int NW = NT / SPG_WAVE;
    const int lane = lane_id();
    const int wid = threadIdx.x / SPG_WAVE;
    T inc = wave_inclusive_scan_add(v);
    if (NW == 1) {
        *total = __shfl(inc, SPG_WAVE - 1, SPG_WAVE);
        return inc - v;
    }
    if (lane == SPG_WAVE - 1) tmp[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NW; ++w) {
            T t = tmp[w];
            tmp[w] = run;
            run += t;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    T res = inc - v + tmp[wid];
    *total = tmp[NW];
    __syncthreads();
    return res;
}

// Workgroup min and max of one value per thread (tmp: 2*(NT/64) elements).
template <int NT, typename T>
__device__ inline void block_min_max(T& mn, T& mx, T* tmp) {
    constexpr int NW = NT / SPG_WAVE;
#pragma unroll
    for (int d = SPG_WAVE / 2; d > 0; d >>= 1) {
        T a = __shfl_xor(mn, d, SPG_WAVE);
        T b = __shfl_xor(mx, d, SPG_WAVE);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if (NW == 1) return;
    const int wid = threadIdx.x / SPG_WAVE;
    if (lane_id() == 0) {
        tmp[wid] = mn;
        tmp[NW + wid] = mx;
    }
    __syncthreads();
    mn = tmp[0];
    mx = tmp[NW];
    for (int w = 1; w < NW; ++w) {
        mn = tmp[w] < mn ? tmp[w] : mn;
        mx = tmp[NW + w] > mx ? tmp[NW + w] : mx;
    }
    __syncthreads();
}

template <int NT, typename T>
__device__ inline T block_reduce_add(T v, T* tmp) {
    T total;
    (void)block_exclusive_scan<NT, T>(v, &total, tmp);
    return total;
}

// ---------------------------------------------------------------------------
// Bitonic sort of n (power of two) 64-bit keys in LDS, ascending, by NT
// threads.  Contains barriers.
// ---------------------------------------------------------------------------
template <int NT>
__device__ inline void block_bitonic_sort_u64(uint64_t* keys, int n) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (n >> 1); t += NT) {
                // index of the lower element of the pair handled by t
                int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                int p = i | j;
                uint64_t a = keys[i], b = keys[p];
                bool up = (i & k) == 0;
                if ((a > b) == up) {
                    keys[i] = b;
                    keys[p] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Bitonic sort of one 64-bit key per lane across a wave (ascending by lane).
__device__ inline uint64_t wave_bitonic_sort_u64(uint64_t key) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= SPG_WAVE; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t o = __shfl_xor(key, j, SPG_WAVE);
            bool lower = (lane & j) == 0;
            bool up = (lane & k) == 0;
            // lower lane keeps min when ascending, max when descending
            bool keep_min = (lower == up);
            uint64_t mn = key < o ? key : o;
            uint64_t mx = key < o ? o : key;
            key = keep_min ? mn : mx;
        }
    }
    return key;
}

__device__ inline uint32_t hash_slot(int32_t key, int log2t) {
    return ((uint32_t)key * 2654435761u) >> (32 - log2t);
}

}  // namespace spg
