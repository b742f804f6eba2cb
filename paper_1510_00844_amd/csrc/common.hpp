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
    // every product is rounded on its own and never fused with the add that
    // takes it (no FMA contraction): the terms are those of the definition
    __device__ static inline acc_t mul(acc_t a, acc_t b) {
#pragma clang fp contract(off)
        return a * b;
    }
    __device__ static inline acc_t add(acc_t a, acc_t b) {
#pragma clang fp contract(off)
        return a + b;
    }
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

// Value of lane (lane ^ j), j a power of two known after unrolling.  Within
// 16 lanes the data moves by DPP (a VALU operand modifier, no LDS round
// trip): quad permutes for j = 1, 2; the two row shifts by 4 for j = 4;
// the row rotation by 8 for j = 8.  ds_swizzle (xor mode, within 32 lanes)
// serves j = 16 and ds_bpermute j = 32.
template <int CTRL>
__device__ inline int dpp_mov(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
__device__ inline uint32_t lane_xor_u32(uint32_t v, int j) {
    const int x = (int)v;
    switch (j) {
        case 1: return (uint32_t)dpp_mov<0xB1>(x);  // quad_perm [1,0,3,2]
        case 2: return (uint32_t)dpp_mov<0x4E>(x);  // quad_perm [2,3,0,1]
        case 4: {
            const int up = dpp_mov<0x104>(x);  // row_shl:4, lane i reads i + 4
            const int dn = dpp_mov<0x114>(x);  // row_shr:4, lane i reads i - 4
            return (uint32_t)((lane_id() & 4) ? dn : up);
        }
        case 8: return (uint32_t)dpp_mov<0x128>(x);  // row_ror:8
        case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401F);  // and 0x1f, xor 0x10
        default: return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ j) << 2, x);
    }
}
template <typename T>
__device__ inline T lane_xor(T v, int j) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u = lane_xor_u32(u, j);
        __builtin_memcpy(&v, &u, 4);
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        const uint32_t lo = lane_xor_u32((uint32_t)u, j), hi = lane_xor_u32((uint32_t)(u >> 32), j);
        u = ((uint64_t)hi << 32) | lo;
        __builtin_memcpy(&v, &u, 8);
    }
    return v;
}

// Value of lane l (per-lane l) of a 32- or 64-bit quantity (ds_bpermute).
template <typename T>
__device__ inline T lane_get(T v, int l) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 4) {
        int u;
        __builtin_memcpy(&u, &v, 4);
        u = __builtin_amdgcn_ds_bpermute(l << 2, u);
        __builtin_memcpy(&v, &u, 4);
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)u);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)(u >> 32));
        u = ((uint64_t)hi << 32) | lo;
        __builtin_memcpy(&v, &u, 8);
    }
    return v;
}

// Value of lane i + 1 (DPP wave_shl:1) and of lane i - 1 (wave_shr:1).  The
// end lanes (63, resp. 0) receive an unspecified value: callers exclude them.
template <int CTRL, typename T>
__device__ inline T lane_shift(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 4) {
        int u;
        __builtin_memcpy(&u, &v, 4);
        u = dpp_mov<CTRL>(u);
        __builtin_memcpy(&v, &u, 4);
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        const uint32_t lo = (uint32_t)dpp_mov<CTRL>((int)(uint32_t)u);
        const uint32_t hi = (uint32_t)dpp_mov<CTRL>((int)(uint32_t)(u >> 32));
        u = ((uint64_t)hi << 32) | lo;
        __builtin_memcpy(&v, &u, 8);
    }
    return v;
}
template <typename T>
__device__ inline T lane_next(T v) { return lane_shift<0x130>(v); }
template <typename T>
__device__ inline T lane_prev(T v) { return lane_shift<0x138>(v); }

// Inclusive prefix sum over the wave.  32-bit integers: Hillis-Steele
// within each row of 16 lanes by DPP row shifts (out-of-row sources read
// 0), then each row's total is broadcast to the rows above (row_bcast:15
// into rows 1 and 3, row_bcast:31 into rows 2 and 3).
template <typename T>
__device__ inline T wave_inclusive_scan_add(T v) {
    if constexpr (sizeof(T) == 4 && __is_integral(T)) {
        int x = (int)v;
        x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);  // row_shr:1
        x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);  // row_shr:2
        x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);  // row_shr:4
        x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);  // row_shr:8
        x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
        x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
        return (T)x;
    } else {
        const int lane = lane_id();
#pragma unroll
        for (int d = 1; d < SPG_WAVE; d <<= 1) {
            T o = __shfl_up(v, d, SPG_WAVE);
            if (lane >= d) v += o;
        }
        return v;
    }
}

// (The reductions keep ds_bpermute: with DPP steps the bitmap kernel's
// per-chunk count loop ran 1.7x longer on 524288-column rows, measured.)
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
        T a = lane_xor(mn, d);
        T b = lane_xor(mx, d);
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
            uint64_t o = lane_xor(key, j);
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

// The same sort for 32-bit keys: one lane exchange, a min and a max per
// step instead of two exchanges and 64-bit selects.
__device__ inline uint32_t wave_bitonic_sort_u32(uint32_t key) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= SPG_WAVE; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t o = lane_xor_u32(key, j);
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            const uint32_t mn = key < o ? key : o;
            const uint32_t mx = key < o ? o : key;
            key = keep_min ? mn : mx;
        }
    }
    return key;
}

__device__ inline uint32_t hash_slot(int32_t key, int log2t) {
    return ((uint32_t)key * 2654435761u) >> (32 - log2t);
}

// LDS writes of one lane visible to the other lanes of the wave.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sorts the n <= N keys keys[off, off + n) of the calling thread ascending,
// in registers: unused places hold the largest key, a bitonic network of
// compile-time comparators (a min and a max each) orders them, and the first
// n are written back.  Reads stay inside [0, T).
template <int N>
__device__ inline void bucket_sort_net(uint32_t* keys, int32_t off, int32_t n, int32_t T) {
    uint32_t a[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
        const int32_t x = off + u < T - 1 ? off + u : T - 1;
        const uint32_t v = keys[x];
        a[u] = u < n ? v : 0xffffffffu;
    }
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t lo = a[i] < a[l] ? a[i] : a[l];
                    const uint32_t hi = a[i] < a[l] ? a[l] : a[i];
                    const bool up = (i & k) == 0;
                    a[i] = up ? lo : hi;
                    a[l] = up ? hi : lo;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < N; ++u)
        if (u < n) keys[off + u] = a[u];
}

// Sorts keys[0, P) ascending (P a power of two) with the calling wave
// alone: a bitonic network whose compare-exchanges the lanes share, one
// stage between wave-level LDS fences.
__device__ inline void wave_lds_bitonic_u32(uint32_t* keys, int P) {
    const int lane = lane_id();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < P / 2; t += SPG_WAVE) {
                const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));  // bit j of i clear
                const int l = i | j;
                const uint32_t x = keys[i], y = keys[l];
                const bool up = (i & k) == 0;
                if ((x > y) == up) {
                    keys[i] = y;
                    keys[l] = x;
                }
            }
            wave_lds_sync();
        }
    }
}

}  // namespace spg
