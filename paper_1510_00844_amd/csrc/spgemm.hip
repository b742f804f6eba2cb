// Host side of the C ABI declared in include/spgemm.h: argument checks,
// plan-owned scratch, bin dispatch, launches and profiling.  All device work
// is in the kernels included below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/spgemm.h"
#include "batched.hpp"
#include "heap.hpp"
#include "learned.hpp"
#include "mis2.hpp"
#include "merge.hpp"
#include "numeric.hpp"
#include "rowinfo.hpp"
#include "scan.hpp"
#include "summa.hpp"
#include "symbolic.hpp"

using namespace spg;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static spg_status fail(spg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return fail(SPG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define SPG_TRY(expr)                      \
    do {                                   \
        spg_status _s = (expr);            \
        if (_s != SPG_OK) return _s;       \
    } while (0)

// ---------------------------------------------------------------------------
// device scratch that only grows
// ---------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    spg_status ensure(size_t need, const char* what) {
        if (need <= bytes) return SPG_OK;
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
        size_t want = std::max(need, (size_t)256);
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            hipGetLastError();
            return fail(SPG_ERR_OOM, std::string("device allocation failed: ") + what);
        }
        bytes = want;
        return SPG_OK;
    }
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct ProfRec {
    std::string name;
    hipEvent_t beg, end;
};

struct Signature {
    const void *a_rp = nullptr, *a_col = nullptr, *b_rp = nullptr, *b_col = nullptr;
    int64_t m = -1, n = -1, k = -1, annz = -1, bnnz = -1, k_lo = -1, k_hi = -1;
    bool operator==(const Signature& o) const {
        return a_rp == o.a_rp && a_col == o.a_col && b_rp == o.b_rp && b_col == o.b_col && m == o.m &&
               n == o.n && k == o.k && annz == o.annz && bnnz == o.bnnz && k_lo == o.k_lo &&
               k_hi == o.k_hi;
    }
};

constexpr int NAUX = 3;  // helper streams for independent bins

struct GalerkinState;

// Sparse SUMMA stages: what the count call leaves for the fill call.
struct SummaState {
    bool valid = false;
    int mode = 0;  // 0: empty result, 1: one block (a single product), 2: piece rows and merge
    spg_semiring sr = SPG_SR_PLUS_TIMES_F64;
    const void *ids = nullptr, *arp = nullptr, *acol = nullptr, *aval = nullptr, *brp = nullptr, *bcol = nullptr,
               *bval = nullptr;
    int64_t nrows = 0, nzr = 0, nnz_a = 0, inner = 0, ncols = 0, stages = 0, b = 0;
    int64_t pieces = 0, nnz_p = 0, nnz_c = 0, nzr_c = 0;
};

struct spg_plan_s {
    int device = 0;
    hipStream_t stream = nullptr;  // the caller's stream: every call is ordered on it
    hipStream_t cur = nullptr;     // stream the next launch goes to
    hipStream_t aux[NAUX] = {};
    hipEvent_t ev_fork = nullptr, ev_join[NAUX] = {};
    hipEvent_t ev_host = nullptr;  // the host waits for read-backs on it
    spg_opts opts;
    int max_lds = 65536;
    int num_cu = 256;

    // per-row state of the current product
    DevBuf a_beg, a_end, flops, maxb, bin, lists, long_rows, small_i32, stats, tiles, split;
    DevBuf merge_len, mbin, mlists, mstats, mctr, bm_save, heavy_idx, chunk_save, rank_items;
    DevBuf lpt_hist, lpt_tmp;  // ordering of heavy bins by work
    const int64_t* out_pos = nullptr;  // numeric output offsets per row (set while a sub-product writes into a full one)
    int64_t* h_stats = nullptr;  // pinned, STATS_WORDS + 8 (nnz of the last read-back at STATS_WORDS)

    Signature sig;
    int64_t sig_rows = 0;       // rows of the current symbolic call (bounds launch grids)
    // saved bitmaps: slots allocated, and the bitmap rows of the last call
    // with these operands (sizes the slots of the next one without a readback)
    int64_t bm_cap = 0;
    bool split_ready = false;  // the split table of the current symbolic call's B is built
    const int64_t* last_crp = nullptr;  // row pointers of the last symbolic call
    Signature bm_sig;
    int64_t bm_rows = -1;
    // frozen: reuse the bin counts of the previous call with the same
    // structure instead of reading them back (no host synchronization, so the
    // calls can be captured into a HIP graph)
    bool frozen = false;
    bool have_symbolic = false;
    bool num_counts_valid = false;
    int64_t sym_counts[3 * NBINS];
    int64_t num_counts[4 * NBINS];
    int64_t last_flops = 0, last_nnz = -1;
    int dense_chunks = 0;

    // single-pass (predicted sizes) state
    DevBuf lcap, lcnt, slot, pcol, pval, fb_list, fb_redo, sub_rp, sub_col, sub_val, sub_crp, mlp_tmp;
    DevBuf sub_pos;  // final output offsets of the recomputed rows
    spg_plan sub = nullptr;  // plan of the exact method for the rows it must redo
    Signature lsig;
    bool have_learned = false;
    int64_t l_counts[2 * NBINS];
    int64_t l_nfb = 0, l_nexact = 0, l_slots = 0, l_nnz = 0, l_sub_nnz = 0, l_sub_annz = 0;
    spg_semiring l_sr = SPG_SR_PLUS_TIMES_F64;

    // batched Galerkin products (created on first use)
    GalerkinState* galerkin = nullptr;

    // distance-2 independent sets and aggregation
    DevBuf mis_key, mis_m1, mis_cand, mis_new, mis_a1, mis_flags, mis_agg1, mis_ctr;

    // Sparse SUMMA stages (child plans created on first use)
    spg_plan summa_p = nullptr, summa_s = nullptr;
    DevBuf sm_pos, sm_piece_rp, sm_p_rp, sm_p_col, sm_p_val, sm_s_rp, sm_s_col, sm_s_val, sm_c_rp, sm_c_pos;
    DevBuf dc_pos;  // spg_dcsr_compress's row scan (apart from the stage state kept between calls)
    SummaState summa;

    // merge state
    std::vector<LayerDesc> merge_sig;
    int64_t merge_m = -1, merge_n = -1;
    int64_t merge_counts[2 * NBINS];

    // profiling
    std::vector<ProfRec> prof_pending;
    std::string prof_only;  // non-empty: time only launches of this name
    std::vector<hipEvent_t> event_pool;
    std::vector<spg_kernel_time> prof_acc;
};

// ---------------------------------------------------------------------------
// launch helper: optional per-launch events, error check
// ---------------------------------------------------------------------------
static hipEvent_t take_event(spg_plan P) {
    if (!P->event_pool.empty()) {
        hipEvent_t e = P->event_pool.back();
        P->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

static inline hipStream_t cs(spg_plan P) { return P->cur ? P->cur : P->stream; }

template <class F>
static spg_status launch(spg_plan P, const std::string& name, F&& f) {
    hipEvent_t b = nullptr, e = nullptr;
    hipStream_t st = P->cur ? P->cur : P->stream;
    const bool timed = P->opts.profile && (P->prof_only.empty() || P->prof_only == name);
    if (timed) {
        b = take_event(P);
        e = take_event(P);
        hipEventRecord(b, st);
    }
    f();
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SPG_ERR_HIP, std::string("launch ") + name + ": " + hipGetErrorString(err));
    if (timed) {
        hipEventRecord(e, st);
        P->prof_pending.push_back({name, b, e});
    }
    return SPG_OK;
}

// Fork: helper streams wait for everything queued so far on the caller's
// stream.  Join: the caller's stream waits for the helpers.  Between the two,
// independent bins are spread over the streams so their kernels overlap.
static spg_status fork_streams(spg_plan P) {
    HIP_TRY(hipEventRecord(P->ev_fork, P->stream));
    for (int k = 0; k < NAUX; ++k) HIP_TRY(hipStreamWaitEvent(P->aux[k], P->ev_fork, 0));
    return SPG_OK;
}
static spg_status join_streams(spg_plan P) {
    for (int k = 0; k < NAUX; ++k) {
        HIP_TRY(hipEventRecord(P->ev_join[k], P->aux[k]));
        HIP_TRY(hipStreamWaitEvent(P->stream, P->ev_join[k], 0));
    }
    P->cur = nullptr;
    return SPG_OK;
}
// Bins go to streams longest-processing-time first: each bin (in order of
// decreasing work) to the stream with the least work so far; the first
// serial_heavy bins stay on the plan's stream.  Work = products + 32 per row.
// Streams in use: at most opts.streams, and no more than the number of bins
// holding at least 5% of the work (more streams than heavy bins only splits
// the GPU between heavy kernels and small ones without shortening them), but
// two whenever two bins have rows: the light bins then run beside the
// heaviest one instead of after it.
static double bin_work(const int64_t* counts, int bin) {
    return (double)counts[NBINS + bin] + 32.0 * (double)counts[bin];
}
struct StreamLoad {
    double load[NAUX + 1] = {};
    int nstreams = 1;
    StreamLoad(spg_plan P, const int64_t* counts) {
        double total = 0;
        for (int b = 1; b < NBINS; ++b) total += bin_work(counts, b);
        int heavy = 0;
        for (int b = 1; b < NBINS; ++b)
            if (counts[b] > 0 && bin_work(counts, b) >= 0.05 * total) ++heavy;
        int nonempty = 0;
        for (int b = 1; b < NBINS; ++b) nonempty += counts[b] > 0;
        nstreams = std::max(1, std::min(P->opts.streams, std::max(heavy, nonempty > 1 ? 2 : 1)));
    }
};
static void use_stream(spg_plan P, StreamLoad& L, int pos, const int64_t* counts, int bin) {
    const double work = bin_work(counts, bin);
    int s = 0;
    if (pos >= P->opts.serial_heavy)
        for (int k = 1; k < L.nstreams; ++k)
            if (L.load[k] < L.load[s]) s = k;
    L.load[s] += work;
    P->cur = s == 0 ? P->stream : P->aux[s - 1];
}

// Order of the non-empty bins by work, largest first, so the heaviest
// kernels start on different streams.
static std::vector<int> bins_by_work(const int64_t* rows, const int64_t* work) {
    std::vector<int> order;
    for (int b = 0; b < NBINS; ++b)
        if (rows[b] > 0) order.push_back(b);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    return order;
}

static inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// The row analysis strides 16 rows per workgroup step; each workgroup adds
// its per-bin statistics to a few global counters once, and device-wide
// atomics on one address serialize across the XCDs, so the grid is kept to
// 1024 workgroups.
static inline unsigned rowinfo_grid(int64_t m) { return (unsigned)std::min<int64_t>(grid_for(m, 16), 1024); }

// static LDS of k_num_rank<*, 512> (A values, product offsets, scan scratch), with margin
static const int RANK_STATIC_LDS = (int)(8 * 512 + sizeof(ProductLds<512>) + 4 * 16 + 256);
static const int RANK_STATIC_LDS_1024 = (int)(8 * 1024 + sizeof(ProductLds<1024>) + 4 * 32 + 256);
static int rank_static_lds(spg_plan P) { return P->opts.rank_block == 1024 ? RANK_STATIC_LDS_1024 : RANK_STATIC_LDS; }
// rank-chunk items: at most this many outputs and this many column chunks
static const int RANKC_CAP = 4096;
// small counters and flags (int32), one size, never reallocated:
//   [0]         long-row queue length (row analysis)
//   [1, 17)     bin cursors of the symbolic classification
//   [33, 49)    bin cursors of the numeric classification
//   [96]        the CSR check flag
//   [100]       the rank-chunk item count
static const int SMALL_WORDS = 128;
static const int CTR_SYM_CURSOR = 1, CTR_NUM_CURSOR = 33, CTR_CHECK = 96, CTR_RANK_ITEMS = 100;
// per-bin statistics (int64): [0, 4 NBINS) the numeric classification (rows,
// flops, A entries, outputs), [4 NBINS] the largest row's products,
// [STATS_SYM, STATS_SYM + 3 NBINS) the symbolic classification (rows, flops,
// A entries)
static const int STATS_SYM = 4 * NBINS + 8;
static const int STATS_WORDS = STATS_SYM + 3 * NBINS;

// ---------------------------------------------------------------------------
// public helpers
// ---------------------------------------------------------------------------
extern "C" void spg_default_opts(spg_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->validate = 0;
    o->small_max_flops = 64;
    o->hash_max_flops = 4096;
    o->hash_max_nnz = 4096;
    o->dense_chunk_cols = 8192;
    o->profile = 0;
    o->streams = 4;
    o->gather_map = 1;
    o->unroll = 4;
    o->sym_gather_map = 1;
    o->sym_unroll = 4;
    o->dense_chunk_cols = 4096;
    o->chunk_min_nnz = 0;  // = hash_max_nnz
    o->chunk_group = 32;
    o->rank_max_nnz = 8192;
    o->rank_block = 512;
    o->chunk_unroll = 4;
    o->heap_max_lists = -1;  // off: slower than the hash tables on the workloads measured here
}

extern "C" const char* spg_status_string(spg_status s) {
    switch (s) {
        case SPG_OK: return "SPG_OK";
        case SPG_ERR_ARG: return "SPG_ERR_ARG";
        case SPG_ERR_SHAPE: return "SPG_ERR_SHAPE";
        case SPG_ERR_NOT_CANONICAL: return "SPG_ERR_NOT_CANONICAL";
        case SPG_ERR_INDEX_RANGE: return "SPG_ERR_INDEX_RANGE";
        case SPG_ERR_OOM: return "SPG_ERR_OOM";
        case SPG_ERR_CAPACITY: return "SPG_ERR_CAPACITY";
        case SPG_ERR_HIP: return "SPG_ERR_HIP";
        case SPG_ERR_STATE: return "SPG_ERR_STATE";
    }
    return "SPG_ERR_UNKNOWN";
}

extern "C" const char* spg_last_error(void) { return g_last_error.c_str(); }

template <int GM>
static void set_lds_attributes(spg_plan P) {
    const int dyn_bitmap = std::max(0, P->max_lds - (int)sizeof(ProductLds<512>) - 64 - 4 * MAX_CHUNKS);
    const int dyn_rank = std::max(0, P->max_lds - RANK_STATIC_LDS);
    hipFuncSetAttribute((const void*)k_sym_bitmap<512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_bitmap);
    hipFuncSetAttribute((const void*)k_num_rank<SR_F64, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_num_rank<SR_I64, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_num_rank<SR_BOOL, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    const int dyn_rank_1024 = std::max(0, P->max_lds - RANK_STATIC_LDS_1024);
    hipFuncSetAttribute((const void*)k_num_rank<SR_F64, 1024, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank_1024);
    hipFuncSetAttribute((const void*)k_num_rank<SR_I64, 1024, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank_1024);
    hipFuncSetAttribute((const void*)k_num_rank<SR_BOOL, 1024, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank_1024);
    hipFuncSetAttribute((const void*)k_num_rankc<SR_F64, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_num_rankc<SR_I64, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_num_rankc<SR_BOOL, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_learned_fused<SR_F64, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_learned_fused<SR_I64, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_learned_fused<SR_BOOL, 512, GM>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
}

// gather mode 4 exists for the bitmap and rank-chunk kernels only
static void set_lds_attributes_pipelined(spg_plan P) {
    const int dyn_bitmap = std::max(0, P->max_lds - (int)sizeof(ProductLds<512>) - 64 - 4 * MAX_CHUNKS);
    const int dyn_rank = std::max(0, P->max_lds - RANK_STATIC_LDS);
    hipFuncSetAttribute((const void*)k_sym_bitmap<512, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_bitmap);
    hipFuncSetAttribute((const void*)k_num_rankc<SR_F64, 512, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_num_rankc<SR_I64, 512, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
    hipFuncSetAttribute((const void*)k_num_rankc<SR_BOOL, 512, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_rank);
}

static int gather_mode(int map, int unroll) { return (map == 2 ? 2 : 0) + (unroll == 8 ? 1 : 0); }

// Double-buffered gathers (gather mode 4) for the bitmap and rank-chunk
// kernels: chosen by opts.gather_pipeline, automatically when the B arrays
// those kernels gather exceed the combined L2 of the 8 XCDs (4 MiB each).
static const int64_t L2_TOTAL_BYTES = 8ll * 4 * 1024 * 1024;
static bool pipelined(spg_plan P, const Csr& b, int64_t bytes_per_entry) {
    if (P->opts.gather_pipeline == 1) return false;
    if (P->opts.gather_pipeline == 2) return true;
    return b.nnz * bytes_per_entry > L2_TOTAL_BYTES;
}

// Call f(std::integral_constant<int, GM>) for the plan's gather mode of the
// numeric (sym = false) or symbolic heavy-row kernels; pipe turns the
// coalesced 4-step mode into its double-buffered form (mode 4).
template <bool PIPE = false, class F>
static spg_status with_gm(spg_plan P, F&& f, bool sym = false, bool pipe = false) {
    const int gm = sym ? gather_mode(P->opts.sym_gather_map, P->opts.sym_unroll)
                       : gather_mode(P->opts.gather_map, P->opts.unroll);
    switch (gm) {
        case 0:
            if constexpr (PIPE)
                if (pipe) return f(std::integral_constant<int, 4>());
            return f(std::integral_constant<int, 0>());
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        default: return f(std::integral_constant<int, 3>());
    }
}

template <bool PIPE = false, class F>
static spg_status with_gm_u(spg_plan P, int map, int unroll, F&& f, bool pipe = false) {
    switch (gather_mode(map, unroll)) {
        case 0:
            if constexpr (PIPE)
                if (pipe) return f(std::integral_constant<int, 4>());
            return f(std::integral_constant<int, 0>());
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        default: return f(std::integral_constant<int, 3>());
    }
}

extern "C" spg_status spg_plan_create(spg_plan* out, void* stream, const spg_opts* opts) {
    if (!out) return fail(SPG_ERR_ARG, "plan pointer is NULL");
    *out = nullptr;
    spg_plan P = new (std::nothrow) spg_plan_s();
    if (!P) return fail(SPG_ERR_OOM, "host allocation failed");
    spg_default_opts(&P->opts);
    if (opts) {
        spg_opts d = P->opts;
        P->opts = *opts;
        if (!P->opts.small_max_flops) P->opts.small_max_flops = d.small_max_flops;
        if (!P->opts.hash_max_flops) P->opts.hash_max_flops = d.hash_max_flops;
        if (!P->opts.hash_max_nnz) P->opts.hash_max_nnz = d.hash_max_nnz;
        if (!P->opts.dense_chunk_cols) P->opts.dense_chunk_cols = d.dense_chunk_cols;
        if (!P->opts.streams) P->opts.streams = d.streams;
        if (!P->opts.gather_map) P->opts.gather_map = d.gather_map;
        if (!P->opts.unroll) P->opts.unroll = d.unroll;
        if (!P->opts.sym_gather_map) P->opts.sym_gather_map = d.sym_gather_map;
        if (!P->opts.sym_unroll) P->opts.sym_unroll = d.sym_unroll;
        if (!P->opts.chunk_min_nnz) P->opts.chunk_min_nnz = P->opts.hash_max_nnz;
        if (!P->opts.chunk_group) P->opts.chunk_group = d.chunk_group;
        if (!P->opts.rank_max_nnz) P->opts.rank_max_nnz = d.rank_max_nnz;
        if (!P->opts.rank_block) P->opts.rank_block = d.rank_block;
        if (!P->opts.chunk_unroll) P->opts.chunk_unroll = d.chunk_unroll;
        if (!P->opts.heap_max_lists) P->opts.heap_max_lists = d.heap_max_lists;
    }
    if (P->opts.heap_max_lists < -1 || P->opts.heap_max_lists > KW_KMAX) {
        delete P;
        return fail(SPG_ERR_ARG, "heap_max_lists must be in [1, 32], 0 (default: off) or -1 (off)");
    }
    if (!P->opts.chunk_min_nnz) P->opts.chunk_min_nnz = P->opts.hash_max_nnz;
    auto map_ok = [](int m) { return m == 1 || m == 2; };
    auto unroll_ok = [](int u) { return u == 4 || u == 8; };
    if (P->opts.streams < 1 || P->opts.streams > NAUX + 1 || !map_ok(P->opts.gather_map) ||
        !map_ok(P->opts.sym_gather_map) || !unroll_ok(P->opts.unroll) || !unroll_ok(P->opts.sym_unroll)) {
        delete P;
        return fail(SPG_ERR_ARG, "streams must be 1..4, gather maps 1 or 2, unroll 4 or 8");
    }
    if (P->opts.small_max_flops < 0 || P->opts.small_max_flops > 64) {
        delete P;
        return fail(SPG_ERR_ARG, "small_max_flops must be in [0, 64]");
    }
    if (P->opts.hash_max_flops < 1 || P->opts.hash_max_flops > 8192) {
        delete P;
        return fail(SPG_ERR_ARG, "hash_max_flops must be in [1, 8192]");
    }
    if (P->opts.hash_max_nnz < 1 || P->opts.hash_max_nnz > 4096) {
        delete P;
        return fail(SPG_ERR_ARG, "hash_max_nnz must be in [1, 4096]");
    }
    if (P->opts.fused_max_nnz < 0) {
        delete P;
        return fail(SPG_ERR_ARG, "fused_max_nnz must be >= 0");
    }
    if (P->opts.gather_pipeline < 0 || P->opts.gather_pipeline > 2) {
        delete P;
        return fail(SPG_ERR_ARG, "gather_pipeline must be 0 (by size), 1 (off) or 2 (on)");
    }
    if (P->opts.chunk_unroll != 4 && P->opts.chunk_unroll != 8) {
        delete P;
        return fail(SPG_ERR_ARG, "chunk_unroll must be 4 or 8");
    }
    if (P->opts.serial_heavy < 0 || P->opts.serial_heavy > NBINS) {
        delete P;
        return fail(SPG_ERR_ARG, "serial_heavy must be in [0, 16]");
    }
    if (P->opts.rank_block != 512 && P->opts.rank_block != 1024) {
        delete P;
        return fail(SPG_ERR_ARG, "rank_block must be 512 or 1024");
    }
    if (P->opts.chunk_min_nnz < 1 || P->opts.chunk_min_nnz > P->opts.hash_max_nnz || P->opts.chunk_group < 1 ||
        P->opts.chunk_group > MAX_CHUNKS) {
        delete P;
        return fail(SPG_ERR_ARG, "chunk_min_nnz must be in [1, hash_max_nnz], chunk_group in [1, 256]");
    }
    if (P->opts.dense_chunk_cols != 16384 && P->opts.dense_chunk_cols != 8192 && P->opts.dense_chunk_cols != 4096 &&
        P->opts.dense_chunk_cols != 2048) {
        delete P;
        return fail(SPG_ERR_ARG, "dense_chunk_cols must be 2048, 4096, 8192 or 16384");
    }
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(SPG_ERR_HIP, "hipGetDevice failed");
    }
    P->stream = (hipStream_t)stream;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) == hipSuccess && lds > 0)
        P->max_lds = lds;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && cus > 0)
        P->num_cu = cus;
    for (int k = 0; k < NAUX; ++k) {
        if (hipStreamCreateWithFlags(&P->aux[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&P->ev_join[k], hipEventDisableTiming) != hipSuccess) {
            hipGetLastError();
            delete P;
            return fail(SPG_ERR_HIP, "helper stream creation failed");
        }
    }
    if (hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_host, hipEventDisableTiming) != hipSuccess) {
        hipGetLastError();
        delete P;
        return fail(SPG_ERR_HIP, "event creation failed");
    }
    if (hipHostMalloc((void**)&P->h_stats, sizeof(int64_t) * (STATS_WORDS + 8), hipHostMallocDefault) != hipSuccess) {
        delete P;
        hipGetLastError();
        return fail(SPG_ERR_OOM, "pinned host allocation failed");
    }
    // LDS beyond 64 KiB for the kernels sized at launch
    set_lds_attributes<0>(P);
    set_lds_attributes<1>(P);
    set_lds_attributes<2>(P);
    set_lds_attributes<3>(P);
    set_lds_attributes_pipelined(P);
    hipGetLastError();
    *out = P;
    return SPG_OK;
}

void spg_release_galerkin(spg_plan P);

extern "C" spg_status spg_plan_destroy(spg_plan P) {
    if (!P) return SPG_OK;
    hipStreamSynchronize(P->stream);
    spg_release_galerkin(P);
    for (DevBuf* b : {&P->a_beg, &P->a_end, &P->flops, &P->maxb, &P->bin, &P->lists, &P->long_rows,
                      &P->small_i32, &P->stats, &P->tiles, &P->split, &P->merge_len,
                      &P->mbin, &P->mlists, &P->mstats, &P->mctr, &P->bm_save, &P->heavy_idx, &P->chunk_save, &P->rank_items,
                      &P->lpt_hist, &P->lpt_tmp,
                      &P->lcap, &P->lcnt, &P->slot, &P->pcol, &P->pval, &P->fb_list, &P->fb_redo, &P->sub_rp,
                      &P->sub_col, &P->sub_val, &P->sub_crp, &P->mlp_tmp, &P->sub_pos,
                      &P->mis_key, &P->mis_m1, &P->mis_cand, &P->mis_new, &P->mis_a1, &P->mis_flags, &P->mis_agg1,
                      &P->mis_ctr, &P->sm_pos, &P->sm_piece_rp, &P->sm_p_rp, &P->sm_p_col, &P->sm_p_val,
                      &P->sm_s_rp, &P->sm_s_col, &P->sm_s_val, &P->sm_c_rp, &P->sm_c_pos, &P->dc_pos})
        b->release();
    if (P->sub) spg_plan_destroy(P->sub);
    if (P->summa_p) spg_plan_destroy(P->summa_p);
    if (P->summa_s) spg_plan_destroy(P->summa_s);
    if (P->h_stats) hipHostFree(P->h_stats);
    for (auto& r : P->prof_pending) {
        hipEventDestroy(r.beg);
        hipEventDestroy(r.end);
    }
    for (auto e : P->event_pool) hipEventDestroy(e);
    for (int k = 0; k < NAUX; ++k) {
        if (P->aux[k]) hipStreamDestroy(P->aux[k]);
        if (P->ev_join[k]) hipEventDestroy(P->ev_join[k]);
    }
    if (P->ev_fork) hipEventDestroy(P->ev_fork);
    if (P->ev_host) hipEventDestroy(P->ev_host);
    delete P;
    return SPG_OK;
}

extern "C" spg_status spg_plan_set_stream(spg_plan P, void* stream) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->stream = (hipStream_t)stream;
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
static spg_status check_csr(const spg_csr* M, const char* name, spg_semiring sr, bool need_val) {
    if (!M) return fail(SPG_ERR_ARG, std::string(name) + " is NULL");
    if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0)
        return fail(SPG_ERR_ARG, std::string(name) + ": negative dimension or nnz");
    if (M->nrows >= (1ll << 31) - 1 || M->ncols >= (1ll << 31) - 1)
        return fail(SPG_ERR_INDEX_RANGE, std::string(name) + ": dimension >= 2^31");
    if (!M->row_ptr) return fail(SPG_ERR_ARG, std::string(name) + ".row_ptr is NULL");
    if (M->nnz > 0 && !M->col) return fail(SPG_ERR_ARG, std::string(name) + ".col is NULL");
    if (need_val && M->nnz > 0 && !M->val && sr != SPG_SR_OR_AND_BOOL)
        return fail(SPG_ERR_ARG, std::string(name) + ".val is NULL");
    return SPG_OK;
}

// Row-per-workgroup launches use up to 1024 threads per row; HIP limits a
// grid to 2^32 threads in x, so one call takes at most 2^22 rows.
static const int64_t MAX_ROWS_PER_CALL = 1ll << 22;

// The product kernels add the lengths of up to 1024 B rows of one A row in
// int32.  Those rows are distinct, so the sum is at most nnz(B), and each
// is at most ncols(B) long: it fits when either bound is below 2^31.
static spg_status check_batch_sums(const spg_csr* B) {
    if (B->nnz >= (1ll << 31) - 1 && B->ncols * 1024 >= (1ll << 31) - 1)
        return fail(SPG_ERR_INDEX_RANGE, "B holds 2^31 or more entries and more than 2^21 columns; split B by columns");
    return SPG_OK;
}

static Csr view(const spg_csr* M) { return Csr{M->nrows, M->ncols, M->nnz, M->row_ptr, M->col, M->val}; }

// validation: row_ptr[0]==0, nondecreasing, row_ptr[m]==nnz, columns in range and increasing
__global__ void __launch_bounds__(256) k_validate(Csr M, int32_t* bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M.nrows) return;
    const int64_t s = M.rp[i], e = M.rp[i + 1];
    bool ok = s <= e && s >= 0 && e <= M.nnz;
    if (i == 0 && s != 0) ok = false;
    if (i == M.nrows - 1 && e != M.nnz) ok = false;
    if (ok) {
        int64_t prev = -1;
        for (int64_t p = s; p < e; ++p) {
            int64_t c = M.col[p];
            if (c <= prev || c >= M.ncols) { ok = false; break; }
            prev = c;
        }
    }
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_bytes(uint8_t* p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

static spg_status fill_i32(spg_plan P, int32_t* p, int64_t n, int32_t v) {
    if (n <= 0) return SPG_OK;
    return launch(P, "fill", [&] { k_fill_i32<<<grid_for(n, 256), 256, 0, cs(P)>>>(p, n, v); });
}
static spg_status fill_i64(spg_plan P, int64_t* p, int64_t n, int64_t v) {
    if (n <= 0) return SPG_OK;
    return launch(P, "fill", [&] { k_fill_i64<<<grid_for(n, 256), 256, 0, cs(P)>>>(p, n, v); });
}

// Orders the row lists of bins [b_lo, b_hi) (contiguous in P->lists) by
// decreasing products within each bin (counting sort, four kernels), with
// the bins located from the per-bin counts on the device: no host copy of
// the counts is needed, and no launch depends on them.
static_assert(NBINS - BIN_DENSE_PAR <= LPT_MAX_BINS, "the heavy numeric bins fit one work ordering");
static spg_status order_by_work(spg_plan P, int b_lo, int b_hi, const int64_t* counts, int64_t max_rows) {
    if (max_rows < 2) return SPG_OK;
    const int nk = (b_hi - b_lo) * LPT_KEYS;
    int32_t* lists = P->lists.as<int32_t>();
    int32_t* hist = P->lpt_hist.as<int32_t>();
    int32_t* tmp = P->lpt_tmp.as<int32_t>();
    const int64_t* work = P->flops.as<int64_t>();
    const uint8_t* bin = P->bin.as<uint8_t>();
    const unsigned grid = (unsigned)std::min<int64_t>(grid_for(max_rows, 256), 1024);
    SPG_TRY(fill_i32(P, hist, nk, 0));
    SPG_TRY(launch(P, "work_order", [&] {
        k_lpt_hist<<<grid, 256, 0, cs(P)>>>(lists, counts, b_lo, b_hi, bin, nk, work, hist);
    }));
    SPG_TRY(launch(P, "work_order", [&] { k_lpt_scan<<<1, 256, 0, cs(P)>>>(hist, nk); }));
    SPG_TRY(launch(P, "work_order", [&] {
        k_lpt_scatter<<<grid, 256, 0, cs(P)>>>(lists, counts, b_lo, b_hi, bin, nk, work, hist, tmp);
    }));
    SPG_TRY(launch(P, "work_order", [&] { k_lpt_copy<<<grid, 256, 0, cs(P)>>>(lists, counts, b_lo, b_hi, tmp); }));
    return SPG_OK;
}


static spg_status validate_csr(spg_plan P, const spg_csr* M, const char* name) {
    if (M->nrows == 0) return SPG_OK;
    SPG_TRY(P->small_i32.ensure(SMALL_WORDS * 4, "flags"));
    int32_t* bad = P->small_i32.as<int32_t>() + CTR_CHECK;
    SPG_TRY(fill_i32(P, bad, 1, 0));
    Csr v = view(M);
    SPG_TRY(launch(P, "validate", [&] { k_validate<<<grid_for(M->nrows, 256), 256, 0, cs(P)>>>(v, bad); }));
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    if (h) return fail(SPG_ERR_NOT_CANONICAL, std::string(name) + " is not canonical CSR");
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// scan of counts (in place over rp[1..m]); rp[0] = 0
// ---------------------------------------------------------------------------
// tiles: (m / SCAN_TILE + 2) int64 of scratch (NULL: the plan's)
static spg_status scan_counts(spg_plan P, int64_t* rp, int64_t m, int64_t* tiles = nullptr) {
    SPG_TRY(fill_i64(P, rp, 1, 0));
    if (m == 0) return SPG_OK;
    const int64_t ntiles = (m + SCAN_TILE - 1) / SCAN_TILE;
    if (!tiles) {
        SPG_TRY(P->tiles.ensure(sizeof(int64_t) * (ntiles + 1), "scan tiles"));
        tiles = P->tiles.as<int64_t>();
    }
    int64_t* cnt = rp + 1;
    SPG_TRY(launch(P, "scan", [&] { k_scan_tiles<<<(unsigned)ntiles, SCAN_NT, 0, cs(P)>>>(cnt, m, tiles); }));
    SPG_TRY(launch(P, "scan", [&] { k_scan_top<<<1, SCAN_NT, 0, cs(P)>>>(tiles, ntiles); }));
    SPG_TRY(launch(P, "scan", [&] { k_scan_apply<<<(unsigned)ntiles, SCAN_NT, 0, cs(P)>>>(cnt, m, tiles, cnt); }));
    return SPG_OK;
}

static spg_status ensure_rows(spg_plan P, int64_t m) {
    const size_t mm = (size_t)std::max<int64_t>(m, 1);
    SPG_TRY(P->a_beg.ensure(8 * mm, "a_beg"));
    SPG_TRY(P->a_end.ensure(8 * mm, "a_end"));
    SPG_TRY(P->flops.ensure(8 * mm, "flops"));
    SPG_TRY(P->maxb.ensure(4 * mm, "maxb"));
    SPG_TRY(P->bin.ensure(mm, "bin"));
    SPG_TRY(P->lists.ensure(4 * mm, "bin lists"));
    SPG_TRY(P->lpt_tmp.ensure(4 * mm, "work order"));
    SPG_TRY(P->lpt_hist.ensure(sizeof(int32_t) * LPT_MAX_BINS * LPT_KEYS, "work order"));
    SPG_TRY(P->long_rows.ensure(4 * mm, "long rows"));
    SPG_TRY(P->small_i32.ensure(SMALL_WORDS * 4, "counters"));
    SPG_TRY(P->stats.ensure(sizeof(int64_t) * STATS_WORDS, "bin stats"));
    return SPG_OK;
}

static BinParams bin_params(spg_plan P, int64_t n) {
    BinParams bp;
    bp.small_max_flops = P->opts.small_max_flops;
    bp.hash_max_flops = P->opts.hash_max_flops;
    bp.hash_max_nnz = P->opts.hash_max_nnz;
    bp.chunk_min_nnz = P->opts.chunk_min_nnz;
    bp.heap_max_lists = P->opts.heap_max_lists > 0 ? P->opts.heap_max_lists : 0;
    bp.heap_max_flops = bp.heap_max_lists > 0 ? KW_LMAX : 0;
    const int64_t bitmap_bytes = ((n + 31) / 32) * 4;
    // dense_ok: one LDS bitmap covers all n columns (the bitmap pass then
    // counts in one block and can save the bitmap for the numeric pass)
    bp.dense_ok = (n <= (1 << 19)) && (bitmap_bytes + (int64_t)sizeof(ProductLds<512>) + 256 <= P->max_lds);
    bp.ncols = n;
    // the bitmap pass records per-chunk counts of the numeric column chunks
    const int64_t W = P->opts.dense_chunk_cols;
    bp.chunk_counts = bp.dense_ok && ((n + W - 1) / W) <= MAX_CHUNKS;
    // rank-space accumulator: (bits, prefix) words + capacity values must fit
    bp.rank_max_log2 = 0;
    if (bp.dense_ok) {
        const int64_t words = 2 * bitmap_bytes;
        for (int lg = 14; lg >= RANK_MIN_LOG2; --lg)
            if ((1ll << lg) <= P->opts.rank_max_nnz && words + (8ll << lg) + rank_static_lds(P) <= P->max_lds) {
                bp.rank_max_log2 = lg;
                break;
            }
    }
    return bp;
}

// The product enumerators count a batch's products (the B-row lengths of up
// to 1024 A entries) in int32, and step through them up to 1024 past the
// current one.  With n <= 2^19 (one LDS bitmap per row) a B row holds at
// most 2^19 entries and a batch stays below 2^29; with wider B the rows that
// enumerate whole B rows (hash bins) are bounded by their own products, so a
// product whose heaviest row has 2^31 - 4096 or more products is rejected
// there (the margin keeps every product index of a step inside int32).
static spg_status check_row_products(const BinParams& bp, int64_t max_row_flops) {
    if (!bp.dense_ok && max_row_flops >= (1ll << 31) - 4096)
        return fail(SPG_ERR_INDEX_RANGE, "a row has 2^31 - 4096 or more products and B has more than 2^19 columns");
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// symbolic
// ---------------------------------------------------------------------------
template <int NT, int LOG2T>
static spg_status launch_sym_hash(spg_plan P, Csr A, Csr B, BinRef ref, int64_t rows, int64_t* cnt) {
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    const unsigned grid = (unsigned)std::max<int64_t>(rows, 1);  // a workgroup per row
    return launch(P, "sym_hash" + std::to_string(1 << LOG2T), [&] {
        k_sym_hash<NT, LOG2T><<<grid, NT, 0, cs(P)>>>(A, B, ref, ab, ae, cnt);
    });
}

// Rows of the 128-, 256- and 512-slot bins (at most 384 products): one wave
// per row, four rows per workgroup.
static spg_status launch_sym_hash_wave(spg_plan P, int lg, Csr A, Csr B, BinRef ref, int64_t rows, int64_t* cnt) {
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    return launch(P, "sym_hash" + std::to_string(1 << lg), [&] {
        k_sym_hash_wave<<<grid_for(std::max<int64_t>(rows, 1), 4), 256, 0, cs(P)>>>(A, B, ref, ab, ae, cnt);
    });
}

static spg_status sym_hash_dispatch(spg_plan P, int lg, Csr A, Csr B, BinRef ref, int64_t rows, int64_t* cnt) {
    switch (lg) {
        case 7:
        case 8:
        case 9: return launch_sym_hash_wave(P, lg, A, B, ref, rows, cnt);
        case 10: return launch_sym_hash<128, 10>(P, A, B, ref, rows, cnt);
        case 11: return launch_sym_hash<256, 11>(P, A, B, ref, rows, cnt);
        case 12: return launch_sym_hash<512, 12>(P, A, B, ref, rows, cnt);
        case 13: return launch_sym_hash<512, 13>(P, A, B, ref, rows, cnt);
        case 14: return launch_sym_hash<1024, 14>(P, A, B, ref, rows, cnt);
    }
    return fail(SPG_ERR_ARG, "bad hash bin");
}

// Heap bin kernels, instantiated for 8, 16 or 32 lists (the plan's
// heap_max_lists rounded up): fewer lists, fewer registers.
static int heap_kmax(spg_plan P) {
    const int k = P->opts.heap_max_lists;
    return k <= 8 ? 8 : (k <= 16 ? 16 : 32);
}

static spg_status sym_heap_launch(spg_plan P, Csr a, Csr b, BinRef ref, int64_t rows, int64_t* cnt) {
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    const int64_t* fl = P->flops.as<int64_t>();
    const unsigned grid = grid_for(std::max<int64_t>(rows, 1), 4);
    switch (heap_kmax(P)) {
        case 8: return launch(P, "sym_heap", [&] { k_sym_heap<8><<<grid, 256, 0, cs(P)>>>(a, b, ref, ab, ae, fl, cnt); });
        case 16: return launch(P, "sym_heap", [&] { k_sym_heap<16><<<grid, 256, 0, cs(P)>>>(a, b, ref, ab, ae, fl, cnt); });
        default: return launch(P, "sym_heap", [&] { k_sym_heap<32><<<grid, 256, 0, cs(P)>>>(a, b, ref, ab, ae, fl, cnt); });
    }
}

template <int SR>
static spg_status num_heap_launch(spg_plan P, Csr a, Csr b, const int32_t* rows, int64_t nr, OutRows crp, int32_t* ccol,
                                  void* cval) {
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    const int64_t* fl = P->flops.as<int64_t>();
    const unsigned grid = grid_for(nr, 4);
    switch (heap_kmax(P)) {
        case 8: return launch(P, "num_heap", [&] { k_num_heap<SR, 8><<<grid, 256, 0, cs(P)>>>(a, b, rows, nr, ab, ae, fl, crp, ccol, cval); });
        case 16: return launch(P, "num_heap", [&] { k_num_heap<SR, 16><<<grid, 256, 0, cs(P)>>>(a, b, rows, nr, ab, ae, fl, crp, ccol, cval); });
        default: return launch(P, "num_heap", [&] { k_num_heap<SR, 32><<<grid, 256, 0, cs(P)>>>(a, b, rows, nr, ab, ae, fl, crp, ccol, cval); });
    }
}

// The numeric pass's column chunks: split[k (P+1) + c] = offset in B(k,:) of
// the first entry at column >= c W.  Depends on B and W only.
static spg_status build_split_table(spg_plan P, Csr b, int32_t W) {
    const int32_t chunks = (int32_t)((b.ncols + W - 1) / W);
    const int64_t entries = b.nrows * (int64_t)(chunks + 1);
    SPG_TRY(P->split.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(entries, 1), "split table"));
    if (entries > 0) {
        int32_t* sp = P->split.as<int32_t>();
        SPG_TRY(launch(P, "split_table", [&] { k_split_table<<<grid_for(entries, 256), 256, 0, cs(P)>>>(b, W, chunks, sp); }));
    }
    return SPG_OK;
}

// Waits on the host for the work queued so far on the plan's stream by
// polling an event: the read-backs on the product's path are short, and a
// poll wakes sooner than a blocking wait.
static spg_status host_wait(spg_plan P) {
    HIP_TRY(hipEventRecord(P->ev_host, P->stream));
    hipError_t e;
    while ((e = hipEventQuery(P->ev_host)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) return fail(SPG_ERR_HIP, std::string("read-back: ") + hipGetErrorString(e));
    return SPG_OK;
}

// Reads back (synchronizing) the classification counts of the last
// symbolic call and nnz(C); the bitmap bin's count sizes the saved bitmaps
// of the next call with the same operands.
static spg_status read_counts(spg_plan P, const int64_t* c_row_ptr, int64_t m) {
    const int64_t* stats = P->stats.as<int64_t>();
    HIP_TRY(hipMemcpyAsync(P->h_stats, stats, sizeof(int64_t) * STATS_WORDS, hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipMemcpyAsync(P->h_stats + STATS_WORDS, c_row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost,
                           P->stream));
    SPG_TRY(host_wait(P));
    const int64_t nnz = P->h_stats[STATS_WORDS];
    std::memcpy(P->num_counts, P->h_stats, sizeof(int64_t) * 4 * NBINS);
    std::memcpy(P->sym_counts, P->h_stats + STATS_SYM, sizeof(int64_t) * 3 * NBINS);
    int64_t tot = 0;
    for (int x = 0; x < NBINS; ++x) tot += P->sym_counts[NBINS + x];
    P->last_flops = tot;
    P->last_nnz = nnz;
    P->num_counts_valid = true;
    P->bm_sig = P->sig;
    P->bm_rows = P->sym_counts[BIN_DENSE];
    return SPG_OK;
}

// Items of the rank-chunk bin: RC outputs at most (at least one chunk).
static int32_t rankc_capacity(spg_plan P) {
    const int32_t W = P->opts.dense_chunk_cols;
    int32_t RC = std::max(RANKC_CAP, W);
    while (RC > W && (int64_t)(W / 32) * 8 + (int64_t)RC * 8 + RANK_STATIC_LDS > P->max_lds) RC /= 2;
    return RC;
}

// Symbolic pass.  The bin kernels locate their rows on the device and stride
// over them, so a launch is correct for any grid; the grids are sized from
// the bin counts, read back once the first time these operands are seen and
// taken from the last call afterwards.  With operands seen before, the whole
// pass (row analysis, the bins on several streams, the scan, the numeric
// classification and the numeric pass's preparation) is queued without
// waiting for the GPU, and the only readback is the final one of the counts
// and nnz(C), which also checks that no bin skipped as empty gained rows (a
// structure changed in place: the pass is then redone with fresh counts).
static spg_status symbolic_pass(spg_plan P, spg_semiring sr, const spg_csr* A, const spg_csr* B, int64_t k_lo,
                                int64_t k_hi, int64_t* c_row_ptr, int64_t* c_nnz, bool fresh);

extern "C" spg_status spgemm_symbolic(spg_plan P, spg_semiring sr, const spg_csr* A, const spg_csr* B,
                                      int64_t k_lo, int64_t k_hi, int64_t* c_row_ptr, int64_t* c_nnz) {
    return symbolic_pass(P, sr, A, B, k_lo, k_hi, c_row_ptr, c_nnz, false);
}

// fresh: read the counts back before the bins even if these operands were
// seen before
static spg_status symbolic_pass(spg_plan P, spg_semiring sr, const spg_csr* A, const spg_csr* B, int64_t k_lo,
                                int64_t k_hi, int64_t* c_row_ptr, int64_t* c_nnz, bool fresh) {
    if (P) P->cur = nullptr;
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    SPG_TRY(check_csr(A, "A", sr, false));
    SPG_TRY(check_csr(B, "B", sr, false));
    if (A->ncols != B->nrows) return fail(SPG_ERR_SHAPE, "A.ncols != B.nrows");
    if (A->nrows > MAX_ROWS_PER_CALL) return fail(SPG_ERR_INDEX_RANGE, "more than 2^22 rows in one call; split A by rows");
    SPG_TRY(check_batch_sums(B));
    if (k_lo < 0 || k_hi < k_lo || k_hi > A->ncols) return fail(SPG_ERR_ARG, "window must satisfy 0 <= k_lo <= k_hi <= A.ncols");
    if (!c_row_ptr) return fail(SPG_ERR_ARG, "c_row_ptr is NULL");
    P->have_symbolic = false;
    P->num_counts_valid = false;
    const int64_t m = A->nrows, n = B->ncols;
    if (P->opts.validate) {
        SPG_TRY(validate_csr(P, A, "A"));
        SPG_TRY(validate_csr(P, B, "B"));
    }
    SPG_TRY(ensure_rows(P, m));
    P->sig_rows = m;
    Csr a = view(A), b = view(B);
    BinParams bp = bin_params(P, n);
    int64_t* stats = P->stats.as<int64_t>();
    int64_t* sstats = stats + STATS_SYM;  // symbolic classification
    int64_t* nstats = stats;              // numeric classification
    int32_t* ctr = P->small_i32.as<int32_t>();
    int64_t* cnt = c_row_ptr + 1;
    const int full = (k_lo == 0 && k_hi == A->ncols) ? 1 : 0;
    int32_t* lists = P->lists.as<int32_t>();
    const int32_t W = P->opts.dense_chunk_cols;

    SPG_TRY(fill_i64(P, stats, STATS_WORDS, 0));
    SPG_TRY(fill_i32(P, ctr, SMALL_WORDS, 0));
    RowInfoOut o{P->a_beg.as<int64_t>(), P->a_end.as<int64_t>(), P->flops.as<int64_t>(), P->maxb.as<int32_t>(),
                 P->bin.as<uint8_t>(), cnt, sstats, P->long_rows.as<int32_t>(), ctr,
                 (unsigned long long*)(stats + 4 * NBINS)};
    if (m > 0) {
        SPG_TRY(launch(P, "rowinfo", [&] {
            k_rowinfo<<<rowinfo_grid(m), 256, 0, cs(P)>>>(a, b, k_lo, k_hi, full, bp, o);
        }));
        SPG_TRY(launch(P, "rowinfo_long", [&] {
            k_rowinfo_long<<<256, 256, 0, cs(P)>>>(a, b, k_lo, k_hi, full, bp, o);
        }));
        SPG_TRY(launch(P, "bin_scatter", [&] {
            k_bin_scatter<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, P->bin.as<uint8_t>(), sstats, ctr + CTR_SYM_CURSOR,
                                                                   lists);
        }));
    }
    Signature sg;
    sg.a_rp = A->row_ptr; sg.a_col = A->col; sg.b_rp = B->row_ptr; sg.b_col = B->col;
    sg.m = m; sg.n = n; sg.k = A->ncols; sg.annz = A->nnz; sg.bnnz = B->nnz; sg.k_lo = k_lo; sg.k_hi = k_hi;
    // The first call with these operands reads back the bitmap bin's row
    // count (to size the saved bitmaps) and the largest row's products (with
    // more than 2^19 columns a batch of whole B rows could overflow the
    // enumerators' int32 counts, so such a row is rejected before any bin
    // runs).  Later calls with the same operands use the last call's count
    // and queue everything without waiting.
    // Bin row counts that size the grids: read back now the first time these
    // operands are seen (exact), else those of the last call with them
    // (checked against the real counts at the final readback).  A graph
    // capture (frozen) reuses the eager call's counts.
    // hint[b] = rows of bin b, hint[NBINS + b] = their products.
    int64_t hint[2 * NBINS];
    bool exact = true;
    const bool known = P->bm_rows >= 0 && P->bm_sig == sg && bp.dense_ok && c_nnz != nullptr && !fresh;
    if (P->frozen || known) {
        std::memcpy(hint, P->sym_counts, sizeof(hint));
        exact = P->frozen;
    } else if (m > 0) {
        HIP_TRY(hipMemcpyAsync(P->h_stats, sstats, sizeof(hint), hipMemcpyDeviceToHost, P->stream));
        HIP_TRY(hipMemcpyAsync(P->h_stats + 2 * NBINS, stats + 4 * NBINS, sizeof(int64_t), hipMemcpyDeviceToHost,
                               P->stream));
        SPG_TRY(host_wait(P));
        SPG_TRY(check_row_products(bp, P->h_stats[2 * NBINS]));
        std::memcpy(hint, P->h_stats, sizeof(hint));
    } else {
        std::memset(hint, 0, sizeof(hint));
    }
    const int64_t bitmap_rows = hint[BIN_DENSE];

    // per-bin accumulators: the bitmap rows (heaviest first) on the plan's
    // stream, the other bins round robin over the helper streams
    const int nstreams = std::max(1, std::min(P->opts.streams, NAUX + 1));
    SPG_TRY(fork_streams(P));
    // the numeric pass's split table (B and W only) on the last helper stream
    // when rank-chunk items are possible (chunk counts recorded, bitmap rows
    // expected) and a row has more than one chunk; the numeric pass builds
    // it for the column-chunked rows otherwise
    const bool chunked = bp.dense_ok && bp.chunk_counts;
    P->split_ready = false;
    P->bm_cap = 0;
    if (chunked && b.ncols > W && bitmap_rows > 0) {
        P->cur = nstreams > 1 ? P->aux[nstreams - 2] : P->stream;
        SPG_TRY(build_split_table(P, b, W));
        P->split_ready = true;
    }
    P->cur = P->stream;
    if (m > 0 && hint[BIN_DENSE] > 0) SPG_TRY(order_by_work(P, BIN_DENSE, BIN_DENSE + 1, sstats, hint[BIN_DENSE]));
    if (m > 0) {
        const int32_t nwords = (int32_t)std::min<int64_t>((n + 31) / 32, 1 << 14);
        uint32_t* save = nullptr;
        int32_t* hidx = nullptr;
        int32_t* csave = nullptr;
        const int32_t nchunks = (int32_t)((n + W - 1) / W);
        int64_t slots = 0;
        if (bp.dense_ok && (bp.rank_max_log2 || bp.chunk_counts)) {
            // one saved bitmap per row of the bitmap bin, as many as that bin
            // held in the last call with these operands (bitmap_rows); a row
            // past the slots is not saved and takes the numeric paths that
            // need no saved bitmap
            SPG_TRY(P->heavy_idx.ensure(4 * (size_t)std::max<int64_t>(m, 1), "bitmap slots"));
            hidx = P->heavy_idx.as<int32_t>();
            slots = std::min<int64_t>(m, bitmap_rows);
            SPG_TRY(P->bm_save.ensure((size_t)std::max<int64_t>(slots, 1) * nwords * 4, "row bitmaps"));
            save = P->bm_save.as<uint32_t>();
            if (bp.chunk_counts) {
                SPG_TRY(P->chunk_save.ensure((size_t)std::max<int64_t>(slots, 1) * nchunks * 4, "chunk counts"));
                csave = P->chunk_save.as<int32_t>();
            }
        }
        P->bm_cap = slots;
        if (hint[BIN_DENSE] > 0) {
            const BinRef dref{sstats, lists, BIN_DENSE};
            SPG_TRY(with_gm<true>(P, [&](auto gm) {
                constexpr int GM = decltype(gm)::value;
                const size_t lds = (size_t)nwords * 4;
                return launch(P, "sym_bitmap", [&] {
                    k_sym_bitmap<512, GM><<<(unsigned)hint[BIN_DENSE], 512, lds, cs(P)>>>(
                        a, b, dref, P->a_beg.as<int64_t>(), P->a_end.as<int64_t>(), cnt, nwords, save, hidx, csave,
                        W / 32, nchunks, slots);
                });
            }, true, pipelined(P, b, 4)));
        }
        // the other bins, by decreasing work, each on the helper stream with
        // the least work so far (the bitmap rows keep the plan's stream)
        std::vector<int> order;
        for (int bb = BIN_SMALL; bb < BIN_DENSE_PAR; ++bb)
            if (hint[bb] > 0) order.push_back(bb);
        if (hint[BIN_HEAP] > 0) order.push_back(BIN_HEAP);
        auto work = [&](int x) { return (double)hint[NBINS + x] + 32.0 * (double)hint[x]; };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
        double aux_load[NAUX] = {};
        for (int bb : order) {
            if (nstreams > 1) {
                int s = 0;
                for (int k = 1; k < nstreams - 1; ++k)
                    if (aux_load[k] < aux_load[s]) s = k;
                aux_load[s] += work(bb);
                P->cur = P->aux[s];
            } else {
                P->cur = P->stream;
            }
            if (bb == BIN_HEAP) {
                SPG_TRY(sym_heap_launch(P, a, b, BinRef{sstats, lists, BIN_HEAP}, hint[bb], cnt));
            } else if (bb == BIN_SMALL) {
                SPG_TRY(launch(P, "sym_small", [&] {
                    k_sym_small<<<grid_for(hint[bb], 4 * SMALL_ROWS), 256, 0, cs(P)>>>(
                        a, b, BinRef{sstats, lists, BIN_SMALL}, P->a_beg.as<int64_t>(), P->a_end.as<int64_t>(), cnt);
                }));
            } else {
                SPG_TRY(sym_hash_dispatch(P, HASH_MIN_LOG2 + (bb - BIN_HASH0), a, b, BinRef{sstats, lists, bb},
                                          hint[bb], cnt));
            }
        }
    }
    SPG_TRY(join_streams(P));
    SPG_TRY(scan_counts(P, c_row_ptr, m));

    // numeric classification from the exact counts, and the numeric pass's
    // preparation: heavy rows ordered by work, the rank-chunk items
    if (m > 0) {
        SPG_TRY(launch(P, "num_classify", [&] {
            k_num_classify<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, c_row_ptr, P->a_beg.as<int64_t>(),
                                                                    P->a_end.as<int64_t>(), P->flops.as<int64_t>(),
                                                                    bp, P->bm_cap > 0 ? P->heavy_idx.as<int32_t>() : nullptr,
                                                                    P->bin.as<uint8_t>(), nstats);
        }));
        SPG_TRY(launch(P, "bin_scatter", [&] {
            k_bin_scatter<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, P->bin.as<uint8_t>(), nstats, ctr + CTR_NUM_CURSOR,
                                                                   lists);
        }));
        // the heavy numeric bins are among the saved bitmap rows
        const int64_t slots_used = P->bm_cap;
        if (slots_used > 0) SPG_TRY(order_by_work(P, BIN_DENSE_PAR, BIN_RANK0 + 3, nstats, slots_used));
        if (chunked && slots_used > 0) {
            const int32_t chunks = (int32_t)((b.ncols + W - 1) / W);
            SPG_TRY(P->rank_items.ensure(sizeof(RankItem) * (size_t)std::max<int64_t>(
                                             P->bm_cap * chunks, 1), "rank items"));
            const int32_t RC = rankc_capacity(P);
            SPG_TRY(launch(P, "rank_items", [&] {
                k_rank_items<<<(unsigned)std::min<int64_t>(grid_for(std::max<int64_t>(slots_used, 1), 256), 256), 256, 0,
                               cs(P)>>>(
                    BinRef{nstats, lists, BIN_DENSE_PAR}, P->heavy_idx.as<int32_t>(),
                    P->chunk_save.as<int32_t>(), chunks, RC, P->opts.chunk_group, W, RANK_STATIC_LDS, P->max_lds,
                    nstats + 3 * NBINS + BIN_DENSE_PAR, P->rank_items.as<RankItem>(), ctr + CTR_RANK_ITEMS);
            }));
        }
    }
    P->sig = sg;
    P->have_symbolic = true;
    if (P->frozen) {
        P->num_counts_valid = true;  // counts of the previous call
        if (c_nnz) *c_nnz = P->last_nnz;
        return SPG_OK;
    }
    P->last_crp = c_row_ptr;
    if (c_nnz) {
        SPG_TRY(read_counts(P, c_row_ptr, m));
        // a bin skipped as empty by the last call's counts that now holds
        // rows: the structure behind the same pointers changed; redo with
        // counts read back first
        if (!exact)
            for (int bb = BIN_SMALL; bb < NBINS; ++bb)
                if (hint[bb] == 0 && P->sym_counts[bb] > 0) return symbolic_pass(P, sr, A, B, k_lo, k_hi, c_row_ptr, c_nnz, true);
        *c_nnz = P->last_nnz;
    }
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// numeric
// ---------------------------------------------------------------------------
template <int SR, int NT, int LOG2T>
static spg_status launch_num_hash(spg_plan P, Csr A, Csr B, const int32_t* rows, int64_t nr,
                                  OutRows crp, int32_t* ccol, void* cval, int64_t* cnt_out) {
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    return launch(P, "num_hash" + std::to_string(1 << LOG2T), [&] {
        k_num_hash<SR, NT, LOG2T><<<(unsigned)nr, NT, 0, cs(P)>>>(A, B, rows, ab, ae, crp, ccol, cval, cnt_out);
    });
}

template <int SR>
static spg_status num_hash_dispatch(spg_plan P, int lg, Csr A, Csr B, const int32_t* rows, int64_t nr,
                                    OutRows crp, int32_t* ccol, void* cval, int64_t* cnt_out = nullptr) {
    switch (lg) {
        case 7: return launch_num_hash<SR, 64, 7>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
        case 8: return launch_num_hash<SR, 64, 8>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
        case 9: return launch_num_hash<SR, 64, 9>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
        case 10: return launch_num_hash<SR, 128, 10>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
        case 11: return launch_num_hash<SR, 256, 11>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
        case 12: return launch_num_hash<SR, 256, 12>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
        case 13: return launch_num_hash<SR, 512, 13>(P, A, B, rows, nr, crp, ccol, cval, cnt_out);
    }
    return fail(SPG_ERR_ARG, "bad numeric hash bin");
}

// The tiny bin (one A entry per row: a scaled copy of one B row): 16 lanes
// per row when its rows copy at most 64 entries on average, a wave per row
// otherwise (ER-like layers: about 16 entries a row; R-MAT: hundreds).
template <int SR>
static spg_status launch_num_tiny(spg_plan P, Csr a, Csr b, const int32_t* rows, int64_t nr, int64_t products,
                                  OutRows out, int32_t* col, void* val) {
    const int64_t* ab = P->a_beg.as<int64_t>();
    if (products <= 64 * nr) {
        return launch(P, "num_tiny", [&] {
            k_num_tiny<SR, 16><<<grid_for(nr, 16), 256, 0, cs(P)>>>(a, b, rows, (int32_t)nr, ab, out, col, val);
        });
    }
    return launch(P, "num_tiny", [&] {
        k_num_tiny<SR, 64><<<grid_for(nr, 4), 256, 0, cs(P)>>>(a, b, rows, (int32_t)nr, ab, out, col, val);
    });
}

// Numeric pass: every bin's kernel, launched with the counts the symbolic
// pass read back (its preparation -- split table, work order, rank-chunk
// items -- ran inside the symbolic pass).
template <int SR>
static spg_status numeric_sr(spg_plan P, Csr a, Csr b, const int64_t* c_row_ptr, int32_t* ccol, void* cval) {
    // output rows start at c_row_ptr, or at P->out_pos for a gathered sub-product
    const OutRows crp(c_row_ptr, P->out_pos);
    const int32_t* lists = P->lists.as<int32_t>();
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    const int W = P->opts.dense_chunk_cols;
    int64_t bin_off[NBINS + 1];
    bin_off[0] = 0;
    for (int x = 0; x < NBINS; ++x) bin_off[x + 1] = bin_off[x] + P->num_counts[x];
    // rows of the column-chunked dense bin need the split table; the
    // symbolic pass builds it when rank chunks are possible
    if (P->num_counts[BIN_DENSE] && b.ncols > W && !P->split_ready) {
        SPG_TRY(build_split_table(P, b, W));
        P->split_ready = true;
    }
    SPG_TRY(fork_streams(P));
    const std::vector<int> num_order = bins_by_work(P->num_counts, P->num_counts + NBINS);
    StreamLoad nload(P, P->num_counts);
    for (size_t oi = 0; oi < num_order.size(); ++oi) {
        const int bb = num_order[oi];
        const int64_t nr = P->num_counts[bb];
        const int32_t* rows = lists + bin_off[bb];
        if (nr == 0 || bb == BIN_EMPTY) continue;
        use_stream(P, nload, (int)oi, P->num_counts, bb);
        if (bb == BIN_TINY) {
            SPG_TRY(launch_num_tiny<SR>(P, a, b, rows, nr, P->num_counts[NBINS + BIN_TINY], crp, ccol, cval));
        } else if (bb == BIN_SMALL) {
            SPG_TRY(launch(P, "num_small", [&] {
                k_num_small<SR><<<grid_for(nr, 4 * SMALL_ROWS), 256, 0, cs(P)>>>(a, b, rows, (int32_t)nr, ab, ae, crp, ccol, cval, nullptr);
            }));
        } else if (bb == BIN_HEAP) {
            SPG_TRY(num_heap_launch<SR>(P, a, b, rows, nr, crp, ccol, cval));
        } else if (bb >= BIN_RANK0) {
            const int32_t nwords = (int32_t)((b.ncols + 31) / 32);
            const int64_t cap = 4096ll << (bb - BIN_RANK0);
            const size_t lds = (size_t)nwords * 8 + (size_t)cap * sizeof(typename Sr<SR>::acc_t);
            SPG_TRY(with_gm(P, [&](auto gm) {
                return launch(P, "num_rank" + std::to_string(cap), [&] {
                    if (P->opts.rank_block == 1024)
                        k_num_rank<SR, 1024, decltype(gm)::value><<<(unsigned)nr, 1024, lds, cs(P)>>>(
                            a, b, rows, ab, ae, P->bm_save.as<uint32_t>(), P->heavy_idx.as<int32_t>(), nwords, crp,
                            ccol, cval);
                    else
                        k_num_rank<SR, 512, decltype(gm)::value><<<(unsigned)nr, 512, lds, cs(P)>>>(
                            a, b, rows, ab, ae, P->bm_save.as<uint32_t>(), P->heavy_idx.as<int32_t>(), nwords, crp,
                            ccol, cval);
                });
            }));
        } else if (bb == BIN_DENSE_PAR) {
            // items (formed in the symbolic pass) of at most RC outputs and G
            // chunks, G from the same rule as there
            const int32_t chunks = (int32_t)((b.ncols + W - 1) / W);
            const int32_t RC = rankc_capacity(P);
            const int32_t G = rankc_group(nr, P->num_counts[3 * NBINS + bb], chunks, RC, P->opts.chunk_group, W,
                                          RANK_STATIC_LDS, P->max_lds);
            const int32_t* nitems = P->small_i32.as<int32_t>() + CTR_RANK_ITEMS;
            const int32_t nwords = (int32_t)((b.ncols + 31) / 32);
            const size_t lds = (size_t)G * (W / 32) * 8 + (size_t)RC * sizeof(typename Sr<SR>::acc_t);
            const int32_t* split = chunks > 1 ? P->split.as<int32_t>() : nullptr;
            const unsigned grid = (unsigned)std::min<int64_t>(nr * chunks, 256 * 8);
            RankItem* items = P->rank_items.as<RankItem>();
            const int32_t* hi = P->heavy_idx.as<int32_t>();
            SPG_TRY(with_gm_u<true>(P, P->opts.gather_map, P->opts.chunk_unroll, [&](auto gm) {
                return launch(P, "num_rankc", [&] {
                    k_num_rankc<SR, 512, decltype(gm)::value><<<grid, 512, lds, cs(P)>>>(
                        a, b, W, rows, ab, ae, P->bm_save.as<uint32_t>(), hi, nwords, split, chunks, items, nitems, RC, G,
                        crp, ccol, cval);
                });
            }, pipelined(P, b, 4 + (int64_t)sizeof(typename Sr<SR>::acc_t))));
        } else if (bb == BIN_DENSE) {
            const int32_t chunks = (int32_t)((b.ncols + W - 1) / W);
            P->dense_chunks = chunks;
            const int32_t* split = chunks > 1 ? P->split.as<int32_t>() : nullptr;
            const unsigned grid = (unsigned)std::min<int64_t>(nr, 1 << 16);
            SPG_TRY(with_gm(P, [&](auto gm) -> spg_status {
                constexpr int GM = decltype(gm)::value;
                return launch(P, "num_dense", [&] {
                    if (W == 16384)
                        k_num_dense<SR, 1024, 16384, GM><<<grid, 1024, 0, cs(P)>>>(a, b, rows, nr, ab, ae, split, chunks, crp, ccol, cval);
                    else if (W == 8192)
                        k_num_dense<SR, 512, 8192, GM><<<grid, 512, 0, cs(P)>>>(a, b, rows, nr, ab, ae, split, chunks, crp, ccol, cval);
                    else if (W == 4096)
                        k_num_dense<SR, 512, 4096, GM><<<grid, 512, 0, cs(P)>>>(a, b, rows, nr, ab, ae, split, chunks, crp, ccol, cval);
                    else
                        k_num_dense<SR, 512, 2048, GM><<<grid, 512, 0, cs(P)>>>(a, b, rows, nr, ab, ae, split, chunks, crp, ccol, cval);
                });
            }));
        } else {
            SPG_TRY(num_hash_dispatch<SR>(P, HASH_MIN_LOG2 + (bb - BIN_HASH0), a, b, rows, nr, crp, ccol, cval));
        }
    }
    SPG_TRY(join_streams(P));
    return SPG_OK;
}

extern "C" spg_status spgemm_numeric(spg_plan P, spg_semiring sr, const spg_csr* A, const spg_csr* B,
                                     int64_t k_lo, int64_t k_hi, const int64_t* c_row_ptr, int32_t* c_col,
                                     void* c_val) {
    if (P) P->cur = nullptr;
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    SPG_TRY(check_csr(A, "A", sr, c_val != nullptr));
    SPG_TRY(check_csr(B, "B", sr, c_val != nullptr));
    if (A->ncols != B->nrows) return fail(SPG_ERR_SHAPE, "A.ncols != B.nrows");
    if (!c_row_ptr) return fail(SPG_ERR_ARG, "c_row_ptr is NULL");
    Signature s;
    s.a_rp = A->row_ptr; s.a_col = A->col; s.b_rp = B->row_ptr; s.b_col = B->col;
    s.m = A->nrows; s.n = B->ncols; s.k = A->ncols; s.annz = A->nnz; s.bnnz = B->nnz; s.k_lo = k_lo; s.k_hi = k_hi;
    if (!P->have_symbolic || !(s == P->sig))
        return fail(SPG_ERR_STATE, "spgemm_numeric needs the matching spgemm_symbolic on this plan first");
    if (!P->num_counts_valid) SPG_TRY(read_counts(P, c_row_ptr, s.m));
    if (P->last_nnz > 0 && !c_col) return fail(SPG_ERR_ARG, "c_col is NULL");
    Csr a = view(A), b = view(B);
    switch (sr) {
        case SPG_SR_PLUS_TIMES_F64: return numeric_sr<SR_F64>(P, a, b, c_row_ptr, c_col, c_val);
        case SPG_SR_PLUS_TIMES_I64: return numeric_sr<SR_I64>(P, a, b, c_row_ptr, c_col, c_val);
        case SPG_SR_OR_AND_BOOL: return numeric_sr<SR_BOOL>(P, a, b, c_row_ptr, c_col, c_val);
    }
    return fail(SPG_ERR_ARG, "unknown semiring");
}

// ---------------------------------------------------------------------------
// merge
// ---------------------------------------------------------------------------
template <int SR, bool FILL>
static spg_status merge_kway_launch(spg_plan P, int32_t c, const LayerSet& ls, BinRef ref, int64_t nr, int64_t* cnt,
                                    const int64_t* orp, int32_t* ocol, void* oval) {
    const unsigned grid = grid_for(nr, 4);
    const char* name = FILL ? "merge_kway" : "merge_kway_count";
    if (c <= 2)
        return launch(P, name, [&] { k_merge_kway<SR, 2, FILL><<<grid, 256, 0, cs(P)>>>(c, ls, ref, cnt, orp, ocol, oval); });
    if (c <= 4)
        return launch(P, name, [&] { k_merge_kway<SR, 4, FILL><<<grid, 256, 0, cs(P)>>>(c, ls, ref, cnt, orp, ocol, oval); });
    return launch(P, name, [&] { k_merge_kway<SR, 8, FILL><<<grid, 256, 0, cs(P)>>>(c, ls, ref, cnt, orp, ocol, oval); });
}

// The merge bins' kernels; the rows of each bin are located on the device
// (lists and per-bin counts from k_merge_rowinfo), the grids sized by the
// counts of the count pass.
template <int SR>
static spg_status merge_launch(spg_plan P, int32_t c, const LayerSet& ls, int64_t n, const int64_t* counts,
                               const int64_t* dev_counts, const int32_t* lists, const int64_t* tl, int64_t* cnt,
                               const int64_t* orp, int32_t* ocol, void* oval) {
    typedef typename Sr<SR>::acc_t V;
    for (int bb = 1; bb < MBINS; ++bb) {
        const int64_t nr = counts[bb];
        if (nr == 0) continue;
        const BinRef ref{dev_counts, lists, bb};
        if ((bb == MBIN_WAVE || bb == MBIN_SORT) && cnt) {
            SPG_TRY(launch(P, "merge_count_hash", [&] {
                k_merge_count_hash<<<grid_for(nr, 4), 256, 0, cs(P)>>>(c, ls, ref, cnt);
            }));
        } else if (bb == MBIN_WAVE) {
            SPG_TRY((merge_kway_launch<SR, true>(P, c, ls, ref, nr, cnt, orp, ocol, oval)));
        } else if (bb == MBIN_SORT) {
            SPG_TRY(launch(P, "merge_sort", [&] {
                k_merge_sort<SR, true><<<grid_for(nr, 4), 256, 0, cs(P)>>>(c, ls, ref, cnt, orp, ocol, oval);
            }));
        } else if (bb == MBIN_SMALL) {
            SPG_TRY(launch(P, "merge_small", [&] {
                k_merge_small<SR><<<grid_for(nr, 4), 256, 0, cs(P)>>>(c, ls, ref, cnt, orp, ocol, oval);
            }));
        } else if (bb == MBIN_DENSE) {
            SPG_TRY(launch(P, "merge_dense", [&] {
                k_merge_dense<SR, 512, 8192><<<(unsigned)nr, 512, 0, cs(P)>>>(c, ls, ref, n, cnt, orp, ocol, oval);
            }));
        } else {
            const int32_t cap = bb == MBIN_R256 ? 256 : (bb == MBIN_R1K ? 1024 : MERGE_LDS_MAX);
            const size_t lds = cnt ? (size_t)cap * 4 : (size_t)cap * (8 + sizeof(V));
            const std::string name = "merge_rank" + std::to_string(cap);
            if (cap == 256) {
                SPG_TRY(launch(P, name, [&] {
                    k_merge_rank<SR, 64><<<(unsigned)nr, 64, lds, cs(P)>>>(c, ls, ref, tl, cap, cnt, orp, ocol, oval);
                }));
            } else {
                SPG_TRY(launch(P, name, [&] {
                    k_merge_rank<SR, 256><<<(unsigned)nr, 256, lds, cs(P)>>>(c, ls, ref, tl, cap, cnt, orp, ocol, oval);
                }));
            }
        }
    }
    return SPG_OK;
}

template <int SR>
static spg_status merge_dispatch(spg_plan P, int32_t c, const LayerSet& ls, int64_t n, const int64_t* counts,
                                 const int64_t* dev_counts, const int32_t* lists, const int64_t* tl, int64_t* cnt,
                                 const int64_t* orp, int32_t* ocol, void* oval) {
    return merge_launch<SR>(P, c, ls, n, counts, dev_counts, lists, tl, cnt, orp, ocol, oval);
}

static spg_status merge_by_sr(spg_plan P, spg_semiring sr, int32_t c, const LayerSet& ls, int64_t n,
                              const int64_t* counts, const int64_t* dev_counts, const int32_t* lists, const int64_t* tl,
                              int64_t* cnt, const int64_t* orp, int32_t* ocol, void* oval) {
    switch (sr) {
        case SPG_SR_PLUS_TIMES_F64: return merge_dispatch<SR_F64>(P, c, ls, n, counts, dev_counts, lists, tl, cnt, orp, ocol, oval);
        case SPG_SR_PLUS_TIMES_I64: return merge_dispatch<SR_I64>(P, c, ls, n, counts, dev_counts, lists, tl, cnt, orp, ocol, oval);
        case SPG_SR_OR_AND_BOOL: return merge_dispatch<SR_BOOL>(P, c, ls, n, counts, dev_counts, lists, tl, cnt, orp, ocol, oval);
    }
    return fail(SPG_ERR_ARG, "unknown semiring");
}

static spg_status check_layers(spg_semiring sr, int32_t nlayers, const spg_csr* layers, bool need_val) {
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    if (nlayers < 1 || nlayers > MERGE_MAX_LAYERS) return fail(SPG_ERR_ARG, "nlayers must be in [1, 64]");
    if (!layers) return fail(SPG_ERR_ARG, "layers is NULL");
    const int64_t m = layers[0].nrows, n = layers[0].ncols;
    if (m > MAX_ROWS_PER_CALL) return fail(SPG_ERR_INDEX_RANGE, "more than 2^22 rows in one call; split by rows");
    for (int l = 0; l < nlayers; ++l) {
        SPG_TRY(check_csr(&layers[l], "layer", sr, need_val));
        if (layers[l].nrows != m || layers[l].ncols != n) return fail(SPG_ERR_SHAPE, "layer shapes differ");
    }
    return SPG_OK;
}

static LayerSet layer_set(int32_t nlayers, const spg_csr* layers) {
    LayerSet ls;
    std::memset(&ls, 0, sizeof(ls));
    for (int l = 0; l < nlayers; ++l) ls.d[l] = LayerDesc{layers[l].row_ptr, layers[l].col, layers[l].val};
    return ls;
}

// Row analysis of the merge: total lengths, bins, per-bin lists; then the
// bin counts are read back (synchronizing) into counts[MBINS].
static spg_status merge_classify(spg_plan P, int32_t c, const LayerSet& ls, int64_t m, int64_t* tl, uint8_t* mbin,
                                 int32_t* mlists, int64_t* mstats, int32_t* mctr, int64_t* counts,
                                 int64_t* host_buf) {
    SPG_TRY(fill_i64(P, mstats, 2 * NBINS, 0));
    SPG_TRY(fill_i32(P, mctr, NBINS, 0));
    if (m > 0) {
        SPG_TRY(launch(P, "merge_rowinfo", [&] {
            k_merge_rowinfo<<<(unsigned)std::min<int64_t>(grid_for(m, 256), 1024), 256, 0, cs(P)>>>(m, c, ls, tl, mbin,
                                                                                                 mstats);
        }));
        SPG_TRY(launch(P, "bin_scatter", [&] {
            k_bin_scatter<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, mbin, mstats, mctr, mlists);
        }));
    }
    HIP_TRY(hipMemcpyAsync(host_buf, mstats, sizeof(int64_t) * MBINS, hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    std::memcpy(counts, host_buf, sizeof(int64_t) * MBINS);
    return SPG_OK;
}

// The merge: count pass (row analysis, bin counts read back, the bins'
// counting kernels, scan, nnz read back) and fill pass (the bins' kernels
// with the count pass's lists and counts: no host synchronization).
extern "C" spg_status spgemm_merge_layers(spg_plan P, spg_semiring sr, int32_t nlayers, const spg_csr* layers,
                                          int64_t* out_row_ptr, int32_t* out_col, void* out_val, int64_t* out_nnz) {
    if (P) P->cur = nullptr;
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    if (!out_row_ptr) return fail(SPG_ERR_ARG, "out_row_ptr is NULL");
    const bool count_pass = out_col == nullptr;
    SPG_TRY(check_layers(sr, nlayers, layers, !count_pass && out_val != nullptr));
    const int64_t m = layers[0].nrows, n = layers[0].ncols;
    if (count_pass && !out_nnz) return fail(SPG_ERR_ARG, "count pass needs out_nnz");
    const LayerSet ls = layer_set(nlayers, layers);
    std::vector<LayerDesc> desc(ls.d, ls.d + nlayers);
    if (P->opts.validate && count_pass)
        for (int l = 0; l < nlayers; ++l) SPG_TRY(validate_csr(P, &layers[l], "layer"));
    int64_t* cnt = out_row_ptr + 1;
    if (count_pass) {
        const size_t mm = (size_t)std::max<int64_t>(m, 1);
        SPG_TRY(P->merge_len.ensure(8 * mm, "merge lengths"));
        SPG_TRY(P->mbin.ensure(mm, "merge bins"));
        SPG_TRY(P->mlists.ensure(4 * mm, "merge lists"));
        SPG_TRY(P->mstats.ensure(sizeof(int64_t) * 4 * NBINS, "merge stats"));
        SPG_TRY(P->mctr.ensure(sizeof(int32_t) * 64, "merge counters"));
        SPG_TRY(merge_classify(P, nlayers, ls, m, P->merge_len.as<int64_t>(), P->mbin.as<uint8_t>(),
                               P->mlists.as<int32_t>(), P->mstats.as<int64_t>(), P->mctr.as<int32_t>(), P->merge_counts,
                               P->h_stats));
        P->merge_sig = desc;
        P->merge_m = m;
        P->merge_n = n;
        SPG_TRY(fill_i64(P, cnt, m, 0));  // empty rows count zero
        SPG_TRY(merge_by_sr(P, sr, nlayers, ls, n, P->merge_counts, P->mstats.as<int64_t>(), P->mlists.as<int32_t>(),
                            P->merge_len.as<int64_t>(), cnt, nullptr, nullptr, nullptr));
        SPG_TRY(scan_counts(P, out_row_ptr, m));
        HIP_TRY(hipMemcpyAsync(P->h_stats, out_row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
        HIP_TRY(hipStreamSynchronize(P->stream));
        *out_nnz = P->h_stats[0];
        return SPG_OK;
    }
    // fill pass: must follow the count pass over the same layers
    bool same = P->merge_m == m && P->merge_n == n && (int)P->merge_sig.size() == nlayers;
    for (int l = 0; same && l < nlayers; ++l)
        same = P->merge_sig[l].rp == desc[l].rp && P->merge_sig[l].col == desc[l].col;
    if (!same) return fail(SPG_ERR_STATE, "merge fill pass needs the matching count pass first");
    // values may differ from the count pass (they were not needed there)
    SPG_TRY(merge_by_sr(P, sr, nlayers, ls, n, P->merge_counts, P->mstats.as<int64_t>(), P->mlists.as<int32_t>(),
                        P->merge_len.as<int64_t>(), nullptr, out_row_ptr, out_col, out_val));
    if (out_nnz) {
        HIP_TRY(hipMemcpyAsync(P->h_stats, out_row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
        HIP_TRY(hipStreamSynchronize(P->stream));
        *out_nnz = P->h_stats[0];
    }
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// merge without allocation: scratch in a file-scope device array
// ---------------------------------------------------------------------------
// One array per GPU (each device holds its own copy for the life of the
// process).  Host code never uses its name as an address: the device address
// comes from hipGetSymbolAddress, once per device, on the first call there.
static constexpr size_t NOALLOC_SCRATCH_BYTES = 16u << 20;
static constexpr int64_t NOALLOC_MAX_ROWS = 1ll << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

static constexpr int NOALLOC_MAX_DEVICES = 64;
static uint8_t* g_scratch[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

static spg_status noalloc_scratch(int device, uint8_t** out) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(SPG_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hipGetLastError();
            return fail(SPG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch[device] = (uint8_t*)p;
    }
    *out = g_scratch[device];
    return SPG_OK;
}

// The merge's scratch carved out of the array: per-row lengths (8 B), bins
// (1 B) and bin lists (4 B), per-bin statistics and counters, scan tiles.
struct NoallocMerge {
    int64_t* tl;
    uint8_t* mbin;
    int32_t* mlists;
    int64_t* mstats;
    int32_t* mctr;
    int64_t* tiles;
};
static constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static NoallocMerge noalloc_layout(uint8_t* base, int64_t m) {
    const size_t mm = (size_t)std::max<int64_t>(m, 1);
    NoallocMerge L;
    size_t off = 0;
    L.tl = (int64_t*)(base + off);
    off += align256(8 * mm);
    L.mlists = (int32_t*)(base + off);
    off += align256(4 * mm);
    L.mbin = base + off;
    off += align256(mm);
    L.mstats = (int64_t*)(base + off);
    off += align256(sizeof(int64_t) * 4 * NBINS);
    L.mctr = (int32_t*)(base + off);
    off += align256(sizeof(int32_t) * 64);
    L.tiles = (int64_t*)(base + off);
    return L;
}
static_assert(align256(8 * NOALLOC_MAX_ROWS) + align256(4 * NOALLOC_MAX_ROWS) + align256(NOALLOC_MAX_ROWS) +
                      align256(sizeof(int64_t) * 4 * NBINS) + align256(sizeof(int32_t) * 64) +
                      sizeof(int64_t) * (NOALLOC_MAX_ROWS / SCAN_TILE + 2) <=
                  NOALLOC_SCRATCH_BYTES,
              "the merge scratch of the largest call fits the array");

extern "C" spg_status spgemm_merge_layers_noalloc(void* stream, spg_semiring sr, int32_t nlayers,
                                                  const spg_csr* layers, int64_t* out_row_ptr, int32_t* out_col,
                                                  void* out_val, int64_t* out_nnz) {
    if (!out_row_ptr) return fail(SPG_ERR_ARG, "out_row_ptr is NULL");
    const bool count_pass = out_col == nullptr;
    SPG_TRY(check_layers(sr, nlayers, layers, !count_pass && out_val != nullptr));
    const int64_t m = layers[0].nrows, n = layers[0].ncols;
    if (m > NOALLOC_MAX_ROWS)
        return fail(SPG_ERR_CAPACITY, "spgemm_merge_layers_noalloc takes at most 2^20 rows (its fixed scratch)");
    if (count_pass && !out_nnz) return fail(SPG_ERR_ARG, "count pass needs out_nnz");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    uint8_t* base = nullptr;
    SPG_TRY(noalloc_scratch(device, &base));
    const NoallocMerge L = noalloc_layout(base, m);
    // a plan on the stack for the launch helpers: no streams, events or
    // device memory of its own, no profiling
    spg_plan_s T;
    spg_default_opts(&T.opts);
    T.device = device;
    T.stream = (hipStream_t)stream;
    int64_t host_buf[2 * NBINS];
    const LayerSet ls = layer_set(nlayers, layers);
    int64_t counts[2 * NBINS] = {};
    // each pass classifies the rows itself, so no state is kept between calls
    SPG_TRY(merge_classify(&T, nlayers, ls, m, L.tl, L.mbin, L.mlists, L.mstats, L.mctr, counts, host_buf));
    if (count_pass) {
        int64_t* cnt = out_row_ptr + 1;
        SPG_TRY(fill_i64(&T, cnt, m, 0));
        SPG_TRY(merge_by_sr(&T, sr, nlayers, ls, n, counts, L.mstats, L.mlists, L.tl, cnt, nullptr, nullptr, nullptr));
        SPG_TRY(scan_counts(&T, out_row_ptr, m, L.tiles));
    } else {
        SPG_TRY(merge_by_sr(&T, sr, nlayers, ls, n, counts, L.mstats, L.mlists, L.tl, nullptr, out_row_ptr, out_col,
                            out_val));
    }
    if (out_nnz) {
        HIP_TRY(hipMemcpyAsync(host_buf, out_row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, T.stream));
        HIP_TRY(hipStreamSynchronize(T.stream));
        *out_nnz = host_buf[0];
    }
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// hypersparse row-compressed matrices and the Sparse SUMMA stages
// ---------------------------------------------------------------------------
static spg_status check_dcsr(const spg_dcsr* A, const char* name, spg_semiring sr, bool need_val) {
    if (!A) return fail(SPG_ERR_ARG, std::string(name) + " is NULL");
    if (A->nrows < 0 || A->ncols < 0 || A->nzr < 0 || A->nnz < 0)
        return fail(SPG_ERR_ARG, std::string(name) + ": negative dimension or count");
    if (A->nrows >= (1ll << 31) - 1 || A->ncols >= (1ll << 31) - 1)
        return fail(SPG_ERR_INDEX_RANGE, std::string(name) + ": dimension >= 2^31");
    if (A->nzr > A->nrows || A->nzr > A->nnz) return fail(SPG_ERR_ARG, std::string(name) + ": nzr exceeds nrows or nnz");
    if (!A->row_ptr) return fail(SPG_ERR_ARG, std::string(name) + ".row_ptr is NULL");
    if (A->nzr > 0 && !A->row_ids) return fail(SPG_ERR_ARG, std::string(name) + ".row_ids is NULL");
    if (A->nnz > 0 && !A->col) return fail(SPG_ERR_ARG, std::string(name) + ".col is NULL");
    if (need_val && A->nnz > 0 && !A->val && sr != SPG_SR_OR_AND_BOOL)
        return fail(SPG_ERR_ARG, std::string(name) + ".val is NULL");
    return SPG_OK;
}

// The compressed view: a CSR over the kept rows.
static spg_csr dcsr_view(const spg_dcsr* A) {
    return spg_csr{A->nzr, A->ncols, A->nnz, A->row_ptr, A->col, A->val};
}

static spg_status validate_dcsr(spg_plan P, const spg_dcsr* A, const char* name) {
    const spg_csr v = dcsr_view(A);
    SPG_TRY(validate_csr(P, &v, name));
    if (A->nzr == 0) return SPG_OK;
    int32_t* bad = P->small_i32.as<int32_t>() + CTR_CHECK;
    SPG_TRY(fill_i32(P, bad, 1, 0));
    SPG_TRY(launch(P, "validate", [&] {
        k_validate_rows<<<grid_for(A->nzr, 256), 256, 0, cs(P)>>>(A->row_ids, A->row_ptr, A->nzr, A->nrows, bad);
    }));
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    if (h) return fail(SPG_ERR_NOT_CANONICAL, std::string(name) + " row indices are not increasing, in range and non-empty");
    return SPG_OK;
}

static spg_status read_i64(spg_plan P, const int64_t* dev, int64_t* out) {
    HIP_TRY(hipMemcpyAsync(P->h_stats, dev, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    *out = P->h_stats[0];
    return SPG_OK;
}

// pos[0..m] = exclusive count of the non-empty rows among rp's m rows.
static spg_status nonempty_scan(spg_plan P, const int64_t* rp, int64_t m, DevBuf& buf) {
    SPG_TRY(buf.ensure(sizeof(int64_t) * (size_t)(m + 1), "row flags"));
    int64_t* pos = buf.as<int64_t>();
    if (m > 0)
        SPG_TRY(launch(P, "dcsr_flags", [&] { k_nonempty_flags<<<grid_for(m, 256), 256, 0, cs(P)>>>(rp, m, pos); }));
    return scan_counts(P, pos, m);
}

extern "C" spg_status spg_dcsr_compress(spg_plan P, const spg_csr* A, int32_t* row_ids, int64_t* row_ptr,
                                        int64_t* nzr) {
    if (P) P->cur = nullptr;
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    SPG_TRY(check_csr(A, "A", SPG_SR_OR_AND_BOOL, false));
    const bool count_pass = row_ptr == nullptr;
    if (count_pass && !nzr) return fail(SPG_ERR_ARG, "the count call needs nzr");
    SPG_TRY(P->small_i32.ensure(SMALL_WORDS * 4, "counters"));
    if (P->opts.validate && count_pass) SPG_TRY(validate_csr(P, A, "A"));
    const int64_t m = A->nrows;
    SPG_TRY(nonempty_scan(P, A->row_ptr, m, P->dc_pos));
    const int64_t* pos = P->dc_pos.as<int64_t>();
    if (count_pass) return read_i64(P, pos + m, nzr);
    int64_t kept = 0;
    SPG_TRY(read_i64(P, pos + m, &kept));
    if (kept > 0 && !row_ids) return fail(SPG_ERR_ARG, "row_ids is NULL");
    if (nzr) *nzr = kept;
    SPG_TRY(launch(P, "dcsr_compress", [&] {
        k_compress_rows<<<grid_for(m + 1, 256), 256, 0, cs(P)>>>(A->row_ptr, m, pos, nullptr, row_ids, row_ptr);
    }));
    return SPG_OK;
}

extern "C" spg_status spg_dcsr_expand(spg_plan P, const spg_dcsr* A, int64_t* row_ptr) {
    if (P) P->cur = nullptr;
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    SPG_TRY(check_dcsr(A, "A", SPG_SR_OR_AND_BOOL, false));
    if (!row_ptr) return fail(SPG_ERR_ARG, "row_ptr is NULL");
    SPG_TRY(P->small_i32.ensure(SMALL_WORDS * 4, "counters"));
    if (P->opts.validate) SPG_TRY(validate_dcsr(P, A, "A"));
    const int64_t m = A->nrows;
    return launch(P, "dcsr_expand", [&] {
        k_expand_rows<<<grid_for(m + 1, 256), 256, 0, cs(P)>>>(A->row_ids, A->row_ptr, A->nzr, m, row_ptr);
    });
}

static spg_status summa_child(spg_plan P, spg_plan* child) {
    if (!*child) SPG_TRY(spg_plan_create(child, (void*)P->stream, &P->opts));
    (*child)->stream = P->stream;
    return SPG_OK;
}

static size_t sr_val_bytes(spg_semiring sr) { return sr == SPG_SR_OR_AND_BOOL ? 1 : 8; }

// The count call: piece rows, their product by B (the kept block
// products), and the merge's symbolic pass; the fill call: the merge's
// numeric pass into the caller's arrays and the compaction of the rows.
extern "C" spg_status spgemm_summa_local(spg_plan P, spg_semiring sr, const spg_dcsr* A, const spg_csr* B,
                                         int64_t stages, int64_t b, int32_t* c_row_ids, int64_t* c_row_ptr,
                                         int32_t* c_col, void* c_val, int64_t* c_nzr, int64_t* c_nnz,
                                         int64_t* stage_nnz) {
    if (P) P->cur = nullptr;
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    const bool count_pass = c_row_ptr == nullptr;
    SPG_TRY(check_dcsr(A, "A", sr, true));
    SPG_TRY(check_csr(B, "B", sr, true));
    if (A->ncols != B->nrows) return fail(SPG_ERR_SHAPE, "A.ncols != B.nrows");
    if (stages < 1 || b < 1) return fail(SPG_ERR_ARG, "stages and b must be positive");
    if (A->ncols % stages) return fail(SPG_ERR_ARG, "the stage count must divide the inner dimension");
    if ((A->ncols / stages) % b) return fail(SPG_ERR_ARG, "b must divide the inner width of a stage");
    if (b > INT32_MAX) b = INT32_MAX;  // one block: every column index is below 2^31
    SummaState& S = P->summa;
    const spg_csr Av = dcsr_view(A);
    if (count_pass) {
        if (!c_nzr || !c_nnz) return fail(SPG_ERR_ARG, "the count call needs c_nzr and c_nnz");
        S = SummaState();
        S.sr = sr;
        S.ids = A->row_ids; S.arp = A->row_ptr; S.acol = A->col; S.aval = A->val;
        S.brp = B->row_ptr; S.bcol = B->col; S.bval = B->val;
        S.nrows = A->nrows; S.nzr = A->nzr; S.nnz_a = A->nnz; S.inner = A->ncols; S.ncols = B->ncols;
        S.stages = stages; S.b = b;
        SPG_TRY(P->small_i32.ensure(SMALL_WORDS * 4, "counters"));
        if (P->opts.validate) {
            SPG_TRY(validate_dcsr(P, A, "A"));
            SPG_TRY(validate_csr(P, B, "B"));
        }
        const int64_t nzr = A->nzr;
        if (nzr == 0 || A->nnz == 0 || A->ncols == 0) {
            S.mode = 0;
        } else {
            SPG_TRY(P->sm_c_rp.ensure(sizeof(int64_t) * (size_t)(nzr + 1), "stage result rows"));
            int64_t* crp = P->sm_c_rp.as<int64_t>();
            int64_t nnz_c = 0;
            if (A->ncols / b <= 1) {
                // one block: the stage product is the result
                S.mode = 1;
                SPG_TRY(summa_child(P, &P->summa_p));
                SPG_TRY(spgemm_symbolic(P->summa_p, sr, &Av, B, 0, A->ncols, crp, &nnz_c));
                S.nnz_p = nnz_c;
            } else {
                S.mode = 2;
                const int64_t nnz = A->nnz;
                // cut the rows into pieces at the block boundaries
                SPG_TRY(P->sm_pos.ensure(sizeof(int64_t) * (size_t)(nnz + 1), "piece flags"));
                int64_t* pos = P->sm_pos.as<int64_t>();
                SPG_TRY(launch(P, "summa_pieces", [&] {
                    k_piece_flags<<<grid_for(nnz, 256), 256, 0, cs(P)>>>(A->col, nnz, (uint32_t)b, pos);
                }));
                SPG_TRY(launch(P, "summa_pieces", [&] {
                    k_piece_row_starts<<<grid_for(nzr, 256), 256, 0, cs(P)>>>(A->row_ptr, nzr, pos);
                }));
                SPG_TRY(scan_counts(P, pos, nnz));
                int64_t G = 0;
                SPG_TRY(read_i64(P, pos + nnz, &G));
                if (G > MAX_ROWS_PER_CALL)
                    return fail(SPG_ERR_INDEX_RANGE, "more than 2^22 row pieces in one call; split A by rows");
                S.pieces = G;
                SPG_TRY(P->sm_piece_rp.ensure(sizeof(int64_t) * (size_t)(G + 1), "piece rows"));
                int64_t* prp = P->sm_piece_rp.as<int64_t>();
                SPG_TRY(launch(P, "summa_pieces", [&] {
                    k_piece_rows<<<grid_for(nnz + 1, 256), 256, 0, cs(P)>>>(pos, nnz, prp);
                }));
                // the kept block products: piece rows times B
                const spg_csr Ap{G, A->ncols, nnz, prp, A->col, A->val};
                SPG_TRY(summa_child(P, &P->summa_p));
                SPG_TRY(P->sm_p_rp.ensure(sizeof(int64_t) * (size_t)(G + 1), "stage products"));
                int64_t nnz_p = 0;
                SPG_TRY(spgemm_symbolic(P->summa_p, sr, &Ap, B, 0, A->ncols, P->sm_p_rp.as<int64_t>(), &nnz_p));
                S.nnz_p = nnz_p;
                SPG_TRY(P->sm_p_col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz_p, 1), "stage products"));
                SPG_TRY(P->sm_p_val.ensure(sr_val_bytes(sr) * (size_t)std::max<int64_t>(nnz_p, 1), "stage products"));
                SPG_TRY(spgemm_numeric(P->summa_p, sr, &Ap, B, 0, A->ncols, P->sm_p_rp.as<int64_t>(),
                                       P->sm_p_col.as<int32_t>(), P->sm_p_val.p));
                // the selection matrix of the merge
                SPG_TRY(P->sm_s_rp.ensure(sizeof(int64_t) * (size_t)(nzr + 1), "merge selection"));
                SPG_TRY(P->sm_s_col.ensure(sizeof(int32_t) * (size_t)G, "merge selection"));
                SPG_TRY(P->sm_s_val.ensure(sr_val_bytes(sr) * (size_t)G, "merge selection"));
                const int64_t nt = std::max<int64_t>(nzr + 1, G);
                int64_t* srp = P->sm_s_rp.as<int64_t>();
                int32_t* scol = P->sm_s_col.as<int32_t>();
                void* sval = P->sm_s_val.p;
                SPG_TRY(launch(P, "summa_selection", [&] {
                    if (sr == SPG_SR_PLUS_TIMES_F64)
                        k_selection<SR_F64><<<grid_for(nt, 256), 256, 0, cs(P)>>>(A->row_ptr, nzr, pos, G, srp, scol, sval);
                    else if (sr == SPG_SR_PLUS_TIMES_I64)
                        k_selection<SR_I64><<<grid_for(nt, 256), 256, 0, cs(P)>>>(A->row_ptr, nzr, pos, G, srp, scol, sval);
                    else
                        k_selection<SR_BOOL><<<grid_for(nt, 256), 256, 0, cs(P)>>>(A->row_ptr, nzr, pos, G, srp, scol, sval);
                }));
                const spg_csr Sm{nzr, G, G, srp, scol, sval};
                const spg_csr Pm{G, B->ncols, nnz_p, P->sm_p_rp.as<int64_t>(), P->sm_p_col.as<int32_t>(), P->sm_p_val.p};
                SPG_TRY(summa_child(P, &P->summa_s));
                SPG_TRY(spgemm_symbolic(P->summa_s, sr, &Sm, &Pm, 0, G, crp, &nnz_c));
            }
            S.nnz_c = nnz_c;
            // rows of the result that came out empty are dropped
            SPG_TRY(nonempty_scan(P, crp, nzr, P->sm_c_pos));
            SPG_TRY(read_i64(P, P->sm_c_pos.as<int64_t>() + nzr, &S.nzr_c));
        }
        S.valid = true;
        *c_nzr = S.nzr_c;
        *c_nnz = S.nnz_c;
        if (stage_nnz) *stage_nnz = S.nnz_p;
        return SPG_OK;
    }
    // fill call: same operands as the count call
    if (!S.valid || S.sr != sr || S.ids != A->row_ids || S.arp != A->row_ptr || S.acol != A->col ||
        S.aval != A->val || S.brp != B->row_ptr || S.bcol != B->col || S.bval != B->val || S.nrows != A->nrows ||
        S.nzr != A->nzr || S.nnz_a != A->nnz || S.inner != A->ncols || S.ncols != B->ncols || S.stages != stages ||
        S.b != b)
        return fail(SPG_ERR_STATE, "the stage fill call needs the matching count call first");
    if (S.nzr_c > 0 && !c_row_ids) return fail(SPG_ERR_ARG, "c_row_ids is NULL");
    if (S.nnz_c > 0 && !c_col) return fail(SPG_ERR_ARG, "c_col is NULL");
    if (S.mode == 0) return fill_i64(P, c_row_ptr, 1, 0);
    const int64_t* crp = P->sm_c_rp.as<int64_t>();
    if (S.mode == 1) {
        SPG_TRY(summa_child(P, &P->summa_p));
        SPG_TRY(spgemm_numeric(P->summa_p, sr, &Av, B, 0, A->ncols, crp, c_col, c_val));
    } else {
        const int64_t G = S.pieces;
        const spg_csr Sm{A->nzr, G, G, P->sm_s_rp.as<int64_t>(), P->sm_s_col.as<int32_t>(), P->sm_s_val.p};
        const spg_csr Pm{G, B->ncols, S.nnz_p, P->sm_p_rp.as<int64_t>(), P->sm_p_col.as<int32_t>(), P->sm_p_val.p};
        SPG_TRY(summa_child(P, &P->summa_s));
        SPG_TRY(spgemm_numeric(P->summa_s, sr, &Sm, &Pm, 0, G, crp, c_col, c_val));
    }
    P->cur = nullptr;
    const int64_t nzr = A->nzr;
    const int64_t* cpos = P->sm_c_pos.as<int64_t>();
    return launch(P, "dcsr_compress", [&] {
        k_compress_rows<<<grid_for(nzr + 1, 256), 256, 0, cs(P)>>>(crp, nzr, cpos, A->row_ids, c_row_ids, c_row_ptr);
    });
}

// ---------------------------------------------------------------------------
// stats and profiling
// ---------------------------------------------------------------------------
extern "C" spg_status spg_plan_stats(spg_plan P, spg_stats* out) {
    if (!P || !out) return fail(SPG_ERR_ARG, "NULL argument");
    if (P->have_symbolic && !P->num_counts_valid && !P->frozen && P->last_crp)
        SPG_TRY(read_counts(P, P->last_crp, P->sig.m));
    std::memset(out, 0, sizeof(*out));
    out->m = P->sig.m;
    out->n = P->sig.n;
    out->k = P->sig.k;
    out->flops = P->last_flops;
    out->nnz_c = P->last_nnz;
    for (int b = 0; b < NBINS; ++b) {
        out->sym_rows[b] = P->sym_counts[b];
        out->sym_flops[b] = P->sym_counts[NBINS + b];
        out->sym_annz[b] = P->sym_counts[2 * NBINS + b];
        if (P->num_counts_valid) {
            out->num_rows[b] = P->num_counts[b];
            out->num_flops[b] = P->num_counts[NBINS + b];
            out->num_annz[b] = P->num_counts[2 * NBINS + b];
            out->num_cnnz[b] = P->num_counts[3 * NBINS + b];
        }
    }
    out->dense_chunk_cols = P->opts.dense_chunk_cols;
    out->dense_chunks = P->dense_chunks;
    return SPG_OK;
}

extern "C" spg_status spg_profile_read(spg_plan P, spg_kernel_time* out, int32_t cap, int32_t* n) {
    if (!P || !n) return fail(SPG_ERR_ARG, "NULL argument");
    HIP_TRY(hipStreamSynchronize(P->stream));
    for (auto& r : P->prof_pending) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.beg, r.end);
        auto it = std::find_if(P->prof_acc.begin(), P->prof_acc.end(),
                               [&](const spg_kernel_time& k) { return r.name == k.name; });
        if (it == P->prof_acc.end()) {
            spg_kernel_time k;
            std::memset(&k, 0, sizeof(k));
            std::snprintf(k.name, sizeof(k.name), "%s", r.name.c_str());
            P->prof_acc.push_back(k);
            it = P->prof_acc.end() - 1;
        }
        it->launches += 1;
        it->total_ms += ms;
        P->event_pool.push_back(r.beg);
        P->event_pool.push_back(r.end);
    }
    P->prof_pending.clear();
    int32_t k = 0;
    for (auto& r : P->prof_acc) {
        if (out && k < cap) out[k] = r;
        ++k;
    }
    *n = k;
    return SPG_OK;
}

extern "C" spg_status spg_profile_select(spg_plan P, const char* name) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->prof_only = name ? name : "";
    return SPG_OK;
}

extern "C" spg_status spg_profile_reset(spg_plan P) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    HIP_TRY(hipStreamSynchronize(P->stream));
    for (auto& r : P->prof_pending) {
        P->event_pool.push_back(r.beg);
        P->event_pool.push_back(r.end);
    }
    P->prof_pending.clear();
    P->prof_acc.clear();
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// predictor: inference, gradient, Adam, training rows
// ---------------------------------------------------------------------------
extern "C" spg_status spg_mlp_forward(spg_plan P, const float* params, const float* x, int64_t n, float* y) {
    if (!P || !params || (n > 0 && (!x || !y))) return fail(SPG_ERR_ARG, "NULL argument");
    if (n <= 0) return SPG_OK;
    P->cur = nullptr;
    return launch(P, "mlp_forward", [&] { k_mlp_forward<<<grid_for(n, 256), 256, 0, cs(P)>>>(params, x, n, y); });
}

extern "C" spg_status spg_mlp_grad(spg_plan P, const float* params, const float* x, const float* t, int64_t n,
                                   float alpha, float* grad, float* loss) {
    if (!P || !params || !grad || (n > 0 && (!x || !t))) return fail(SPG_ERR_ARG, "NULL argument");
    if (n <= 0) return SPG_OK;
    P->cur = nullptr;
    return launch(P, "mlp_grad", [&] {
        k_mlp_grad<<<grid_for(n, MLP_BS), MLP_BS, 0, cs(P)>>>(params, x, t, n, alpha, grad, loss);
    });
}

extern "C" spg_status spg_mlp_adam(spg_plan P, float* params, float* grad, float* m, float* v, int64_t step,
                                   float lr, float beta1, float beta2, float eps) {
    if (!P || !params || !grad || !m || !v || step < 1) return fail(SPG_ERR_ARG, "bad argument");
    P->cur = nullptr;
    return launch(P, "mlp_adam", [&] {
        k_mlp_adam<<<grid_for(MLP_NPARAMS, 256), 256, 0, cs(P)>>>(params, grad, m, v, step, lr, beta1, beta2, eps);
    });
}

extern "C" spg_status spg_row_training_data(spg_plan P, const int64_t* c_row_ptr, int64_t min_flops, float* x,
                                            float* t, int64_t* nsel) {
    if (!P || !c_row_ptr || !x || !t || !nsel) return fail(SPG_ERR_ARG, "NULL argument");
    if (!P->have_symbolic) return fail(SPG_ERR_STATE, "needs a finished spgemm_symbolic on this plan");
    P->cur = nullptr;
    const int64_t m = P->sig.m;
    SPG_TRY(P->mlp_tmp.ensure(64, "counter"));
    unsigned long long* cnt = P->mlp_tmp.as<unsigned long long>();
    SPG_TRY(fill_i64(P, (int64_t*)cnt, 1, 0));
    if (m > 0) {
        SPG_TRY(launch(P, "train_rows", [&] {
            k_train_rows<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, P->a_beg.as<int64_t>(), P->a_end.as<int64_t>(),
                                                              P->flops.as<int64_t>(), P->maxb.as<int32_t>(),
                                                              P->opts.small_max_flops, min_flops, c_row_ptr, x, t,
                                                              cnt);
        }));
    }
    HIP_TRY(hipMemcpyAsync(P->h_stats, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    *nsel = P->h_stats[0];
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// single-pass product with predicted sizes
// ---------------------------------------------------------------------------
// Largest capacity (log2) of the fused single-pass kernel: what the LDS
// allows, and no more than fused_max_nnz and rank_max_nnz (larger rows take
// the exact path, where column-chunk items keep more workgroups on a CU);
// 0 = no fused kernel.
static int fused_max_log2(spg_plan P, int64_t n) {
    const int64_t nwords = (n + 31) / 32;
    if (nwords > 8 * 512) return 0;  // the fused kernel keeps <= 8 bitmap words per thread
    const int64_t lim = std::min<int64_t>(P->opts.rank_max_nnz, P->opts.fused_max_nnz);
    int top = 14;
    while (top >= RANK_MIN_LOG2 && (1ll << top) > lim) --top;
    for (int lg = top; lg >= RANK_MIN_LOG2; --lg)
        if (nwords * 8 + (8ll << lg) + RANK_STATIC_LDS <= P->max_lds) return lg;
    return 0;
}

template <int SR>
static spg_status learned_launch(spg_plan P, Csr a, Csr b, int32_t nwords) {
    const int32_t* lists = P->lists.as<int32_t>();
    const int64_t* ab = P->a_beg.as<int64_t>();
    const int64_t* ae = P->a_end.as<int64_t>();
    const int64_t* slot = P->slot.as<int64_t>();
    int64_t* cnt = P->lcnt.as<int64_t>() + 1;
    int32_t* pcol = P->pcol.as<int32_t>();
    void* pval = P->pval.p;
    int64_t bin_off[NBINS + 1];
    bin_off[0] = 0;
    for (int x = 0; x < NBINS; ++x) bin_off[x + 1] = bin_off[x] + P->l_counts[x];
    // the fused bitmap-rank rows (bins 13..15), heaviest first
    SPG_TRY(order_by_work(P, BIN_DENSE_PAR, BIN_RANK0 + 3, P->stats.as<int64_t>(),
                          bin_off[BIN_RANK0 + 3] - bin_off[BIN_DENSE_PAR]));
    SPG_TRY(fork_streams(P));
    const std::vector<int> order = bins_by_work(P->l_counts, P->l_counts + NBINS);
    StreamLoad lload(P, P->l_counts);
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const int bb = order[oi];
        const int64_t nr = P->l_counts[bb];
        const int32_t* rows = lists + bin_off[bb];
        if (nr == 0 || bb == BIN_EMPTY || bb == BIN_DENSE) continue;
        use_stream(P, lload, (int)oi, P->l_counts, bb);
        if (bb == BIN_TINY) {
            SPG_TRY(launch_num_tiny<SR>(P, a, b, rows, nr, P->l_counts[NBINS + BIN_TINY], slot, pcol, pval));
        } else if (bb == BIN_SMALL) {
            SPG_TRY(launch(P, "num_small", [&] {
                k_num_small<SR><<<grid_for(nr, 4 * SMALL_ROWS), 256, 0, cs(P)>>>(a, b, rows, (int32_t)nr, ab, ae, slot, pcol, pval,
                                                                     cnt);
            }));
        } else if (bb >= BIN_RANK0 && bb < BIN_RANK0 + 3) {
            const int64_t acc_cap = 4096ll << (bb - BIN_RANK0);
            const size_t lds = (size_t)nwords * 8 + (size_t)acc_cap * sizeof(typename Sr<SR>::acc_t);
            SPG_TRY(with_gm(P, [&](auto gm) {
                return launch(P, "learned_fused" + std::to_string(acc_cap), [&] {
                    k_learned_fused<SR, 512, decltype(gm)::value><<<(unsigned)nr, 512, lds, cs(P)>>>(
                        a, b, rows, ab, ae, nwords, acc_cap, slot, cnt, pcol, pval);
                });
            }, true));
        } else {
            SPG_TRY(num_hash_dispatch<SR>(P, HASH_MIN_LOG2 + (bb - BIN_HASH0), a, b, rows, nr, slot, pcol, pval, cnt));
        }
    }
    return join_streams(P);
}

template <int SR>
static spg_status gather_sub_rows(spg_plan P, Csr a) {
    const int32_t nl = (int32_t)P->l_nfb;
    SPG_TRY(P->sub_rp.ensure(8 * (size_t)(nl + 1), "recomputed rows"));
    int64_t* srp = P->sub_rp.as<int64_t>();
    SPG_TRY(launch(P, "gather_len", [&] {
        k_gather_len<<<grid_for(nl, 256), 256, 0, cs(P)>>>(a.rp, P->fb_list.as<int32_t>(), nl, srp + 1);
    }));
    SPG_TRY(scan_counts(P, srp, nl));
    HIP_TRY(hipMemcpyAsync(P->h_stats, srp + nl, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    const int64_t annz = P->h_stats[0];
    P->l_sub_annz = annz;
    const size_t w = SR == SR_BOOL ? 1 : 8;
    SPG_TRY(P->sub_col.ensure(4 * (size_t)std::max<int64_t>(annz, 1), "recomputed rows"));
    SPG_TRY(P->sub_val.ensure(w * (size_t)std::max<int64_t>(annz, 1), "recomputed rows"));
    SPG_TRY(launch(P, "gather_rows", [&] {
        k_gather_rows<SR><<<grid_for(nl, 4), 256, 0, cs(P)>>>(a, P->fb_list.as<int32_t>(), nl, srp,
                                                               P->sub_col.as<int32_t>(), P->sub_val.p);
    }));
    return SPG_OK;
}

static spg_csr sub_matrix(spg_plan P, const spg_csr* A) {
    spg_csr s;
    s.nrows = P->l_nfb;
    s.ncols = A->ncols;
    s.nnz = P->l_sub_annz;
    s.row_ptr = P->sub_rp.as<int64_t>();
    s.col = P->sub_col.as<int32_t>();
    s.val = P->sub_val.p;
    return s;
}

extern "C" spg_status spgemm_learned_run(spg_plan P, spg_semiring sr, const spg_csr* A, const spg_csr* B,
                                         int64_t k_lo, int64_t k_hi, const float* mlp_params, float margin,
                                         int64_t* c_nnz, spg_learned_stats* st) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->cur = nullptr;
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    SPG_TRY(check_csr(A, "A", sr, true));
    SPG_TRY(check_csr(B, "B", sr, true));
    if (A->ncols != B->nrows) return fail(SPG_ERR_SHAPE, "A.ncols != B.nrows");
    if (A->nrows > MAX_ROWS_PER_CALL) return fail(SPG_ERR_INDEX_RANGE, "more than 2^22 rows in one call; split A by rows");
    SPG_TRY(check_batch_sums(B));
    if (k_lo < 0 || k_hi < k_lo || k_hi > A->ncols) return fail(SPG_ERR_ARG, "window must satisfy 0 <= k_lo <= k_hi <= A.ncols");
    if (!c_nnz) return fail(SPG_ERR_ARG, "c_nnz is NULL");
    if (!(margin >= 0.f) || margin > 100.f) return fail(SPG_ERR_ARG, "margin must be in [0, 100]");
    P->have_learned = false;
    P->have_symbolic = false;
    P->num_counts_valid = false;
    const int64_t m = A->nrows, n = B->ncols;
    if (P->opts.validate) {
        SPG_TRY(validate_csr(P, A, "A"));
        SPG_TRY(validate_csr(P, B, "B"));
    }
    SPG_TRY(ensure_rows(P, m));
    const size_t mm = (size_t)std::max<int64_t>(m, 1);
    SPG_TRY(P->lcap.ensure(8 * mm, "capacities"));
    SPG_TRY(P->lcnt.ensure(8 * (mm + 1), "counts"));
    SPG_TRY(P->slot.ensure(8 * (mm + 1), "slots"));
    SPG_TRY(P->fb_list.ensure(4 * mm, "recomputed rows"));
    SPG_TRY(P->fb_redo.ensure(mm, "recomputed rows"));
    Csr a = view(A), b = view(B);
    BinParams bp = bin_params(P, n);
    int64_t* stats = P->stats.as<int64_t>();
    int32_t* ctr = P->small_i32.as<int32_t>();
    int64_t* cnt = P->lcnt.as<int64_t>() + 1;
    const int full = (k_lo == 0 && k_hi == A->ncols) ? 1 : 0;
    SPG_TRY(fill_i64(P, stats, 4 * NBINS + 1, 0));
    SPG_TRY(fill_i32(P, ctr, 2 + NBINS, 0));
    RowInfoOut o{P->a_beg.as<int64_t>(), P->a_end.as<int64_t>(), P->flops.as<int64_t>(), P->maxb.as<int32_t>(),
                 P->bin.as<uint8_t>(), cnt, stats, P->long_rows.as<int32_t>(), ctr,
                 (unsigned long long*)(stats + 4 * NBINS)};
    LearnedParams lp;
    lp.margin = margin;
    lp.use_mlp = mlp_params ? 1 : 0;
    lp.fused_max_log2 = fused_max_log2(P, n);
    lp.hash_max_nnz = P->opts.hash_max_nnz;
    if (m > 0) {
        SPG_TRY(launch(P, "rowinfo", [&] {
            k_rowinfo<<<rowinfo_grid(m), 256, 0, cs(P)>>>(a, b, k_lo, k_hi, full, bp, o);
        }));
        SPG_TRY(launch(P, "rowinfo_long", [&] {
            k_rowinfo_long<<<256, 256, 0, cs(P)>>>(a, b, k_lo, k_hi, full, bp, o);
        }));
        SPG_TRY(fill_i64(P, stats, 4 * NBINS, 0));
        SPG_TRY(launch(P, "learned_classify", [&] {
            k_learned_classify<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, n, mlp_params, lp, bp, P->a_beg.as<int64_t>(),
                                                                    P->a_end.as<int64_t>(), P->flops.as<int64_t>(),
                                                                    P->maxb.as<int32_t>(), P->bin.as<uint8_t>(),
                                                                    P->lcap.as<int64_t>(), cnt, stats);
        }));
        SPG_TRY(launch(P, "bin_scatter", [&] {
            k_bin_scatter<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, P->bin.as<uint8_t>(), stats, ctr + 2,
                                                               P->lists.as<int32_t>());
        }));
        HIP_TRY(hipMemcpyAsync(P->slot.as<int64_t>() + 1, P->lcap.p, 8 * (size_t)m, hipMemcpyDeviceToDevice, cs(P)));
    }
    SPG_TRY(scan_counts(P, P->slot.as<int64_t>(), m));
    HIP_TRY(hipMemcpyAsync(P->h_stats, stats, sizeof(int64_t) * 2 * NBINS, hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipMemcpyAsync(P->h_stats + 2 * NBINS, P->slot.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost,
                           P->stream));
    HIP_TRY(hipMemcpyAsync(P->h_stats + 2 * NBINS + 1, stats + 4 * NBINS, sizeof(int64_t), hipMemcpyDeviceToHost,
                           P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    SPG_TRY(check_row_products(bp, P->h_stats[2 * NBINS + 1]));
    std::memcpy(P->l_counts, P->h_stats, sizeof(int64_t) * 2 * NBINS);
    P->l_slots = P->h_stats[2 * NBINS];
    P->l_nexact = P->l_counts[BIN_DENSE];
    const size_t w = sr == SPG_SR_OR_AND_BOOL ? 1 : 8;
    SPG_TRY(P->pcol.ensure(4 * (size_t)std::max<int64_t>(P->l_slots, 1), "padded output"));
    SPG_TRY(P->pval.ensure(w * (size_t)std::max<int64_t>(P->l_slots, 1), "padded output"));
    const int32_t nwords = (int32_t)((n + 31) / 32);
    spg_status stt = SPG_OK;
    switch (sr) {
        case SPG_SR_PLUS_TIMES_F64: stt = learned_launch<SR_F64>(P, a, b, nwords); break;
        case SPG_SR_PLUS_TIMES_I64: stt = learned_launch<SR_I64>(P, a, b, nwords); break;
        case SPG_SR_OR_AND_BOOL: stt = learned_launch<SR_BOOL>(P, a, b, nwords); break;
    }
    SPG_TRY(stt);
    // rows the exact method must compute
    SPG_TRY(fill_i32(P, ctr, 1, 0));
    if (m > 0) {
        SPG_TRY(launch(P, "fallback_rows", [&] {
            k_fallback_rows<<<grid_for(m, 256), 256, 0, cs(P)>>>(m, P->bin.as<uint8_t>(), P->lcap.as<int64_t>(), cnt,
                                                                 P->fb_list.as<int32_t>(), ctr, P->fb_redo.as<uint8_t>());
        }));
    }
    int32_t hfb = 0;
    HIP_TRY(hipMemcpyAsync(&hfb, ctr, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    P->l_nfb = hfb;
    P->l_sub_nnz = 0;
    if (hfb > 0) {
        switch (sr) {
            case SPG_SR_PLUS_TIMES_F64: stt = gather_sub_rows<SR_F64>(P, a); break;
            case SPG_SR_PLUS_TIMES_I64: stt = gather_sub_rows<SR_I64>(P, a); break;
            case SPG_SR_OR_AND_BOOL: stt = gather_sub_rows<SR_BOOL>(P, a); break;
        }
        SPG_TRY(stt);
        if (!P->sub) SPG_TRY(spg_plan_create(&P->sub, (void*)P->stream, &P->opts));
        P->sub->stream = P->stream;
        SPG_TRY(P->sub_crp.ensure(8 * (size_t)(hfb + 1), "recomputed rows"));
        spg_csr S = sub_matrix(P, A);
        int64_t snnz = 0;
        SPG_TRY(spgemm_symbolic(P->sub, sr, &S, B, k_lo, k_hi, P->sub_crp.as<int64_t>(), &snnz));
        P->l_sub_nnz = snnz;
        SPG_TRY(launch(P, "scatter_counts", [&] {
            k_scatter_counts<<<grid_for(hfb, 256), 256, 0, cs(P)>>>(P->fb_list.as<int32_t>(), hfb,
                                                                    P->sub_crp.as<int64_t>(), cnt);
        }));
    }
    SPG_TRY(scan_counts(P, P->lcnt.as<int64_t>(), m));
    HIP_TRY(hipMemcpyAsync(P->h_stats, P->lcnt.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    P->l_nnz = P->h_stats[0];
    *c_nnz = P->l_nnz;
    Signature sg;
    sg.a_rp = A->row_ptr; sg.a_col = A->col; sg.b_rp = B->row_ptr; sg.b_col = B->col;
    sg.m = m; sg.n = n; sg.k = A->ncols; sg.annz = A->nnz; sg.bnnz = B->nnz; sg.k_lo = k_lo; sg.k_hi = k_hi;
    P->lsig = sg;
    P->l_sr = sr;
    P->have_learned = true;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        int64_t pred = 0;
        for (int x = BIN_HASH0; x < NBINS; ++x)
            if (x != BIN_DENSE) pred += P->l_counts[x];
        st->rows_predicted = pred;
        st->rows_exact = P->l_nexact;
        st->rows_overflow = P->l_nfb - P->l_nexact;
        st->slots = P->l_slots;
        st->nnz_c = P->l_nnz;
        st->nnz_single = P->l_nnz - P->l_sub_nnz;
        for (int x = 0; x < NBINS; ++x) st->bin_rows[x] = P->l_counts[x];
    }
    return SPG_OK;
}

template <int SR>
static spg_status learned_fetch_sr(spg_plan P, const spg_csr* A, const spg_csr* B, int64_t* c_row_ptr,
                                   int32_t* c_col, void* c_val) {
    const int64_t m = P->lsig.m;
    if (m > 0) {
        SPG_TRY(launch(P, "copy_rows", [&] {
            k_copy_rows<SR><<<(unsigned)std::min<int64_t>(m, 65536), 256, 0, cs(P)>>>(m, nullptr, P->fb_redo.as<uint8_t>(), P->slot.as<int64_t>(),
                                                                c_row_ptr, P->pcol.as<int32_t>(), P->pval.p, c_col, c_val);
        }));
    }
    if (P->l_nfb > 0) {
        // the recomputed rows write straight into the caller's arrays: the
        // sub-product's numeric pass takes their final offsets
        SPG_TRY(P->sub_pos.ensure(8 * (size_t)P->l_nfb, "recomputed rows"));
        int64_t* pos = P->sub_pos.as<int64_t>();
        SPG_TRY(launch(P, "gather_offsets", [&] {
            k_gather_offsets<<<grid_for(P->l_nfb, 256), 256, 0, cs(P)>>>(P->fb_list.as<int32_t>(), (int32_t)P->l_nfb,
                                                                         c_row_ptr, pos);
        }));
        spg_csr S = sub_matrix(P, A);
        P->sub->out_pos = pos;
        const spg_status st = spgemm_numeric(P->sub, P->l_sr, &S, B, P->lsig.k_lo, P->lsig.k_hi,
                                             P->sub_crp.as<int64_t>(), c_col, c_val);
        P->sub->out_pos = nullptr;
        SPG_TRY(st);
        P->cur = nullptr;
    }
    return SPG_OK;
}

extern "C" spg_status spgemm_learned_fetch(spg_plan P, const spg_csr* A, const spg_csr* B, int64_t* c_row_ptr,
                                           int32_t* c_col, void* c_val) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->cur = nullptr;
    if (!A || !B || !c_row_ptr) return fail(SPG_ERR_ARG, "NULL argument");
    if (!P->have_learned || P->lsig.a_rp != A->row_ptr || P->lsig.b_rp != B->row_ptr || P->lsig.m != A->nrows)
        return fail(SPG_ERR_STATE, "spgemm_learned_fetch needs the matching spgemm_learned_run first");
    if (P->l_nnz > 0 && !c_col) return fail(SPG_ERR_ARG, "c_col is NULL");
    HIP_TRY(hipMemcpyAsync(c_row_ptr, P->lcnt.p, 8 * (size_t)(P->lsig.m + 1), hipMemcpyDeviceToDevice, P->stream));
    switch (P->l_sr) {
        case SPG_SR_PLUS_TIMES_F64: return learned_fetch_sr<SR_F64>(P, A, B, c_row_ptr, c_col, c_val);
        case SPG_SR_PLUS_TIMES_I64: return learned_fetch_sr<SR_I64>(P, A, B, c_row_ptr, c_col, c_val);
        case SPG_SR_OR_AND_BOOL: return learned_fetch_sr<SR_BOOL>(P, A, B, c_row_ptr, c_col, c_val);
    }
    return fail(SPG_ERR_ARG, "unknown semiring");
}

// ---------------------------------------------------------------------------
// batched Galerkin products C_b = (RT_b A_b) R_b
// ---------------------------------------------------------------------------
struct GalerkinState {
    std::vector<spg_csr> sig_rt, sig_a, sig_r;
    spg_semiring sr = SPG_SR_PLUS_TIMES_F64;
    int32_t nb = 0;
    DevBuf desc, rt_rp, rt_col, rt_val, a_rp, a_col, a_val, r_rp, r_col, r_val;
    DevBuf t_rp, t_col, t_val, c_rp, c_col, c_val, out_rp;
    spg_plan p1 = nullptr, p2 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the sequence runs (and is captured) on this stream, ordered after and
    // before the caller's stream by events; capture is not possible on the
    // legacy default stream a caller may pass
    hipStream_t gs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int64_t rows_rt = 0, cols_rt = 0, nnz_rt = 0, rows_a = 0, nnz_a = 0, rows_r = 0, cols_r = 0, nnz_r = 0;
    int64_t nnz_t = 0, nnz_c = 0;
    std::vector<BatchDesc> h_desc;  // [rt | a | r | c] tables
    std::vector<int64_t> c_base;    // first entry of each instance in C
    bool valid = false;
};

static GalerkinState* galerkin_state(spg_plan P);
static spg_status galerkin_run(spg_plan P, GalerkinState* G, spg_semiring sr, int32_t nb, const spg_csr* RT,
                               const spg_csr* A, const spg_csr* R, int32_t use_graph);
static void galerkin_free(GalerkinState* G);

static bool same_csr(const spg_csr& x, const spg_csr& y) {
    return x.nrows == y.nrows && x.ncols == y.ncols && x.nnz == y.nnz && x.row_ptr == y.row_ptr && x.col == y.col &&
           x.val == y.val;
}

static unsigned assemble_grid(int64_t rows, int64_t nnz) {
    return (unsigned)std::min<int64_t>(grid_for(std::max(rows + 1, nnz), 256), 8192);
}

// The whole device sequence of one batched call.  eager: may allocate and
// read sizes back; otherwise (graph capture) only launches, with the sizes
// of the eager call.
static spg_status galerkin_sequence(spg_plan P, GalerkinState* G, bool eager) {
    const int32_t nb = G->nb;
    const BatchDesc* d = G->desc.as<BatchDesc>();
    const int32_t vw = G->sr == SPG_SR_OR_AND_BOOL ? 1 : 8;
    P->cur = G->gs;
    // the assembled operands are canonical when the instances are; only the
    // eager call may synchronize.  Later calls (replays) copy values only:
    // the structure may not change between them, so the eager call's
    // assembled row pointers and columns stay valid
    G->p1->opts.validate = G->p2->opts.validate = eager ? P->opts.validate : 0;
    SPG_TRY(launch(P, "batch_assemble", [&] {
        k_batch_assemble<<<assemble_grid(G->rows_rt, G->nnz_rt), 256, 0, cs(P)>>>(d, nb, G->rows_rt, G->nnz_rt, vw, eager ? 1 : 0,
                                                                          G->rt_rp.as<int64_t>(), G->rt_col.as<int32_t>(),
                                                                          G->rt_val.p);
    }));
    SPG_TRY(launch(P, "batch_assemble", [&] {
        k_batch_assemble<<<assemble_grid(G->rows_a, G->nnz_a), 256, 0, cs(P)>>>(d + nb, nb, G->rows_a, G->nnz_a, vw, eager ? 1 : 0,
                                                                         G->a_rp.as<int64_t>(), G->a_col.as<int32_t>(),
                                                                         G->a_val.p);
    }));
    SPG_TRY(launch(P, "batch_assemble", [&] {
        k_batch_assemble<<<assemble_grid(G->rows_r, G->nnz_r), 256, 0, cs(P)>>>(d + 2 * nb, nb, G->rows_r, G->nnz_r, vw, eager ? 1 : 0,
                                                                         G->r_rp.as<int64_t>(), G->r_col.as<int32_t>(),
                                                                         G->r_val.p);
    }));
    spg_csr RT{G->rows_rt, G->cols_rt, G->nnz_rt, G->rt_rp.as<int64_t>(), G->rt_col.as<int32_t>(), G->rt_val.p};
    spg_csr A{G->rows_a, G->rows_r, G->nnz_a, G->a_rp.as<int64_t>(), G->a_col.as<int32_t>(), G->a_val.p};
    spg_csr R{G->rows_r, G->cols_r, G->nnz_r, G->r_rp.as<int64_t>(), G->r_col.as<int32_t>(), G->r_val.p};
    const size_t w = vw;
    int64_t nt = G->nnz_t, nc = G->nnz_c;
    // The symbolic passes run in the eager call only: the structure is fixed
    // between replays, so its row pointers, bin lists, saved bitmaps and
    // work items (kept by the two product plans, which nothing else uses)
    // serve every replay's numeric passes.
    if (eager) {
        SPG_TRY(G->t_rp.ensure(8 * (size_t)(G->rows_rt + 1), "batched T"));
        SPG_TRY(spgemm_symbolic(G->p1, G->sr, &RT, &A, 0, A.nrows, G->t_rp.as<int64_t>(), &nt));
        G->nnz_t = nt;
        SPG_TRY(G->t_col.ensure(4 * (size_t)std::max<int64_t>(nt, 1), "batched T"));
        SPG_TRY(G->t_val.ensure(w * (size_t)std::max<int64_t>(nt, 1), "batched T"));
    }
    SPG_TRY(spgemm_numeric(G->p1, G->sr, &RT, &A, 0, A.nrows, G->t_rp.as<int64_t>(), G->t_col.as<int32_t>(), G->t_val.p));
    spg_csr T{G->rows_rt, G->rows_r, G->nnz_t, G->t_rp.as<int64_t>(), G->t_col.as<int32_t>(), G->t_val.p};
    if (eager) {
        SPG_TRY(G->c_rp.ensure(8 * (size_t)(G->rows_rt + 1), "batched C"));
        SPG_TRY(spgemm_symbolic(G->p2, G->sr, &T, &R, 0, R.nrows, G->c_rp.as<int64_t>(), &nc));
        G->nnz_c = nc;
        SPG_TRY(G->c_col.ensure(4 * (size_t)std::max<int64_t>(nc, 1), "batched C"));
        SPG_TRY(G->c_val.ensure(w * (size_t)std::max<int64_t>(nc, 1), "batched C"));
        SPG_TRY(G->out_rp.ensure(8 * (size_t)(G->rows_rt + nb), "batched output"));
    }
    SPG_TRY(spgemm_numeric(G->p2, G->sr, &T, &R, 0, R.nrows, G->c_rp.as<int64_t>(), G->c_col.as<int32_t>(), G->c_val.p));
    P->cur = G->gs;
    SPG_TRY(fill_i64(P, G->out_rp.as<int64_t>(), G->rows_rt + nb, 0));
    SPG_TRY(launch(P, "batch_split", [&] {
        k_batch_split<<<grid_for(G->rows_rt, 256), 256, 0, cs(P)>>>(d + 3 * nb, nb, G->rows_rt, G->c_rp.as<int64_t>(),
                                                                   G->c_col.as<int32_t>(), G->out_rp.as<int64_t>());
    }));
    P->cur = nullptr;
    return SPG_OK;
}

extern "C" spg_status spgemm_galerkin_batched(spg_plan P, spg_semiring sr, int32_t nb, const spg_csr* RT,
                                              const spg_csr* A, const spg_csr* R, spg_csr* out, int32_t use_graph) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->cur = nullptr;
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    if (nb < 1 || !RT || !A || !R || !out) return fail(SPG_ERR_ARG, "need nb >= 1 and non-NULL arrays");
    for (int b = 0; b < nb; ++b) {
        SPG_TRY(check_csr(&RT[b], "RT", sr, true));
        SPG_TRY(check_csr(&A[b], "A", sr, true));
        SPG_TRY(check_csr(&R[b], "R", sr, true));
        if (RT[b].ncols != A[b].nrows || A[b].ncols != R[b].nrows || R[b].ncols != RT[b].nrows)
            return fail(SPG_ERR_SHAPE, "instance shapes must be RT: M x N, A: N x N', R: N' x M");
    }
    GalerkinState* G = galerkin_state(P);
    if (!G) return fail(SPG_ERR_OOM, "host allocation failed");
    if (!G->gs) {
        HIP_TRY(hipStreamCreateWithFlags(&G->gs, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&G->ev_in, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&G->ev_out, hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(G->ev_in, P->stream));
    HIP_TRY(hipStreamWaitEvent(G->gs, G->ev_in, 0));
    spg_status st = galerkin_run(P, G, sr, nb, RT, A, R, use_graph);
    P->cur = nullptr;
    HIP_TRY(hipEventRecord(G->ev_out, G->gs));
    HIP_TRY(hipStreamWaitEvent(P->stream, G->ev_out, 0));
    SPG_TRY(st);
    for (int b = 0; b < nb; ++b) {
        const BatchDesc& D = G->h_desc[3 * (size_t)nb + b];
        out[b].nrows = D.nrows;
        out[b].ncols = R[b].ncols;
        out[b].nnz = G->c_base[b + 1] - G->c_base[b];
        out[b].row_ptr = G->out_rp.as<int64_t>() + D.row_off + b;
        out[b].col = G->c_col.as<int32_t>() + G->c_base[b];
        out[b].val = (const char*)G->c_val.p + (size_t)G->c_base[b] * (sr == SPG_SR_OR_AND_BOOL ? 1 : 8);
    }
    return SPG_OK;
}

// Capture the device sequence (with the sizes of the eager call) into one
// graph on the state's stream.
static spg_status galerkin_capture(spg_plan P, GalerkinState* G) {
    G->p1->frozen = G->p2->frozen = true;
    const int32_t prof = P->opts.profile;
    P->opts.profile = 0;  // no timing events inside the graph
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(G->gs, hipStreamCaptureModeThreadLocal));
    spg_status st = galerkin_sequence(P, G, false);
    hipError_t e = hipStreamEndCapture(G->gs, &g);
    G->p1->frozen = G->p2->frozen = false;
    P->opts.profile = prof;
    if (st != SPG_OK) {
        if (g) hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(SPG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    G->graph = g;
    HIP_TRY(hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0));
    return SPG_OK;
}

static spg_status galerkin_run(spg_plan P, GalerkinState* G, spg_semiring sr, int32_t nb, const spg_csr* RT,
                               const spg_csr* A, const spg_csr* R, int32_t use_graph) {
    bool same = G->valid && G->nb == nb && G->sr == sr;
    for (int b = 0; same && b < nb; ++b)
        same = same_csr(G->sig_rt[b], RT[b]) && same_csr(G->sig_a[b], A[b]) && same_csr(G->sig_r[b], R[b]);
    if (!same) {
        // sizes and offsets of the three batches and of the result
        if (G->exec) { hipGraphExecDestroy(G->exec); G->exec = nullptr; }
        if (G->graph) { hipGraphDestroy(G->graph); G->graph = nullptr; }
        G->valid = false;
        G->nb = nb;
        G->sr = sr;
        G->sig_rt.assign(RT, RT + nb);
        G->sig_a.assign(A, A + nb);
        G->sig_r.assign(R, R + nb);
        G->h_desc.assign(4 * (size_t)nb, BatchDesc{});
        int64_t r0 = 0, c0 = 0, z0 = 0;
        for (int b = 0; b < nb; ++b) {  // RT_b: M x N, columns of A's batch
            G->h_desc[b] = BatchDesc{RT[b].row_ptr, RT[b].col, RT[b].val, RT[b].nrows, r0, z0, c0};
            r0 += RT[b].nrows; c0 += RT[b].ncols; z0 += RT[b].nnz;
        }
        G->rows_rt = r0; G->cols_rt = c0; G->nnz_rt = z0;
        r0 = c0 = z0 = 0;
        for (int b = 0; b < nb; ++b) {
            G->h_desc[nb + b] = BatchDesc{A[b].row_ptr, A[b].col, A[b].val, A[b].nrows, r0, z0, c0};
            r0 += A[b].nrows; c0 += A[b].ncols; z0 += A[b].nnz;
        }
        G->rows_a = r0; G->nnz_a = z0;
        const int64_t cols_a = c0;
        r0 = c0 = z0 = 0;
        for (int b = 0; b < nb; ++b) {
            G->h_desc[2 * nb + b] = BatchDesc{R[b].row_ptr, R[b].col, R[b].val, R[b].nrows, r0, z0, c0};
            r0 += R[b].nrows; c0 += R[b].ncols; z0 += R[b].nnz;
        }
        G->rows_r = r0; G->cols_r = c0; G->nnz_r = z0;
        if (G->rows_a != G->cols_rt || cols_a != G->rows_r)
            return fail(SPG_ERR_SHAPE, "batch dimension totals differ");
        r0 = c0 = 0;
        for (int b = 0; b < nb; ++b) {  // result: M_b x M_b, rows/columns of the coarse batch
            G->h_desc[3 * nb + b] = BatchDesc{nullptr, nullptr, nullptr, RT[b].nrows, r0, 0, c0};
            r0 += RT[b].nrows; c0 += R[b].ncols;
        }
        if (G->rows_rt >= (1ll << 31) || G->cols_rt >= (1ll << 31) || G->rows_r >= (1ll << 31) || G->cols_r >= (1ll << 31))
            return fail(SPG_ERR_INDEX_RANGE, "batch dimensions >= 2^31");
        const size_t w = sr == SPG_SR_OR_AND_BOOL ? 1 : 8;
        SPG_TRY(G->desc.ensure(sizeof(BatchDesc) * 4 * (size_t)nb, "batch descriptors"));
        SPG_TRY(G->rt_rp.ensure(8 * (size_t)(G->rows_rt + 1), "batched RT"));
        SPG_TRY(G->rt_col.ensure(4 * (size_t)std::max<int64_t>(G->nnz_rt, 1), "batched RT"));
        SPG_TRY(G->rt_val.ensure(w * (size_t)std::max<int64_t>(G->nnz_rt, 1), "batched RT"));
        SPG_TRY(G->a_rp.ensure(8 * (size_t)(G->rows_a + 1), "batched A"));
        SPG_TRY(G->a_col.ensure(4 * (size_t)std::max<int64_t>(G->nnz_a, 1), "batched A"));
        SPG_TRY(G->a_val.ensure(w * (size_t)std::max<int64_t>(G->nnz_a, 1), "batched A"));
        SPG_TRY(G->r_rp.ensure(8 * (size_t)(G->rows_r + 1), "batched R"));
        SPG_TRY(G->r_col.ensure(4 * (size_t)std::max<int64_t>(G->nnz_r, 1), "batched R"));
        SPG_TRY(G->r_val.ensure(w * (size_t)std::max<int64_t>(G->nnz_r, 1), "batched R"));
        HIP_TRY(hipMemcpyAsync(G->desc.p, G->h_desc.data(), sizeof(BatchDesc) * 4 * (size_t)nb, hipMemcpyHostToDevice,
                               G->gs));
        if (!G->p1) SPG_TRY(spg_plan_create(&G->p1, (void*)G->gs, &P->opts));
        if (!G->p2) SPG_TRY(spg_plan_create(&G->p2, (void*)G->gs, &P->opts));
        G->p1->opts = G->p2->opts = P->opts;
        G->p1->stream = G->p2->stream = G->gs;
        G->p1->opts.profile = G->p2->opts.profile = 0;
        G->p1->frozen = G->p2->frozen = false;
        SPG_TRY(galerkin_sequence(P, G, true));
        // first entry of each instance in C (host copy of the row pointers)
        std::vector<int64_t> crp((size_t)G->rows_rt + 1);
        HIP_TRY(hipMemcpyAsync(crp.data(), G->c_rp.p, 8 * crp.size(), hipMemcpyDeviceToHost, G->gs));
        HIP_TRY(hipStreamSynchronize(G->gs));
        G->c_base.resize((size_t)nb + 1);
        for (int b = 0; b < nb; ++b) G->c_base[b] = crp[(size_t)G->h_desc[3 * nb + b].row_off];
        G->c_base[nb] = crp[(size_t)G->rows_rt];
        G->valid = true;
        if (use_graph) SPG_TRY(galerkin_capture(P, G));  // for later calls; this one ran eagerly
    } else if (use_graph) {
        if (!G->exec) SPG_TRY(galerkin_capture(P, G));
        HIP_TRY(hipGraphLaunch(G->exec, G->gs));
    } else {
        G->p1->frozen = G->p2->frozen = true;
        spg_status st = galerkin_sequence(P, G, false);
        G->p1->frozen = G->p2->frozen = false;
        SPG_TRY(st);
    }
    return SPG_OK;
}

extern "C" spg_status spgemm_galerkin_copy(spg_plan P, int64_t* row_ptr, int32_t* col, void* val) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    GalerkinState* G = galerkin_state(P);
    if (!G || !G->valid) return fail(SPG_ERR_STATE, "no batched Galerkin result on this plan");
    const size_t w = G->sr == SPG_SR_OR_AND_BOOL ? 1 : 8;
    if (!row_ptr) return fail(SPG_ERR_ARG, "row_ptr is NULL");
    HIP_TRY(hipMemcpyAsync(row_ptr, G->out_rp.p, 8 * (size_t)(G->rows_rt + G->nb), hipMemcpyDeviceToDevice, P->stream));
    if (G->nnz_c > 0) {
        if (!col) return fail(SPG_ERR_ARG, "col is NULL");
        HIP_TRY(hipMemcpyAsync(col, G->c_col.p, 4 * (size_t)G->nnz_c, hipMemcpyDeviceToDevice, P->stream));
        if (val) HIP_TRY(hipMemcpyAsync(val, G->c_val.p, w * (size_t)G->nnz_c, hipMemcpyDeviceToDevice, P->stream));
    }
    return SPG_OK;
}

// per-plan Galerkin state (owned by the plan, freed with it)
static GalerkinState* galerkin_state(spg_plan P) {
    if (!P->galerkin) P->galerkin = new (std::nothrow) GalerkinState();
    return P->galerkin;
}
static void galerkin_free(GalerkinState* G) {
    if (!G) return;
    if (G->exec) hipGraphExecDestroy(G->exec);
    if (G->graph) hipGraphDestroy(G->graph);
    for (DevBuf* b : {&G->desc, &G->rt_rp, &G->rt_col, &G->rt_val, &G->a_rp, &G->a_col, &G->a_val, &G->r_rp, &G->r_col,
                      &G->r_val, &G->t_rp, &G->t_col, &G->t_val, &G->c_rp, &G->c_col, &G->c_val, &G->out_rp})
        b->release();
    if (G->p1) spg_plan_destroy(G->p1);
    if (G->p2) spg_plan_destroy(G->p2);
    if (G->gs) {
        hipStreamSynchronize(G->gs);
        hipStreamDestroy(G->gs);
    }
    if (G->ev_in) hipEventDestroy(G->ev_in);
    if (G->ev_out) hipEventDestroy(G->ev_out);
    delete G;
}
void spg_release_galerkin(spg_plan P) {
    galerkin_free(P->galerkin);
    P->galerkin = nullptr;
}

// ---------------------------------------------------------------------------
// autotuner of the batched Galerkin products
// ---------------------------------------------------------------------------
#include <chrono>
#include <cstdio>
#include <fstream>

namespace {

// knobs the tuner varies, with their candidate values
struct TuneKnob {
    const char* name;
    int32_t spg_opts::*field;
    std::vector<int32_t> values;
};

std::vector<TuneKnob> tune_knobs() {
    return {
        {"small_max_flops", &spg_opts::small_max_flops, {16, 32, 64}},
        {"streams", &spg_opts::streams, {1, 2, 4}},
        {"gather_map", &spg_opts::gather_map, {1, 2}},
        {"unroll", &spg_opts::unroll, {4, 8}},
        {"sym_gather_map", &spg_opts::sym_gather_map, {1, 2}},
        {"hash_max_nnz", &spg_opts::hash_max_nnz, {2048, 4096}},
    };
}

// device and workload key of a cache entry: architecture, CU count, the
// semiring and every instance's sizes (folded into a 64-bit FNV-1a hash)
std::string tune_key(int device, spg_semiring sr, int32_t nb, const spg_csr* RT, const spg_csr* A,
                     const spg_csr* R) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (char& ch : arch)
        if (ch == '"' || ch == ' ' || ch == ':') ch = '_';
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    int64_t tot = 0;
    for (int b = 0; b < nb; ++b) {
        for (const spg_csr* M : {&RT[b], &A[b], &R[b]}) {
            mix(M->nrows);
            mix(M->ncols);
            mix(M->nnz);
            tot += M->nnz;
        }
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "galerkin:%s:cu%d:sr%d:nb%d:nnz%lld:%016llx", arch.c_str(), cus, (int)sr, (int)nb,
                  (long long)tot, (unsigned long long)h);
    return buf;
}

// one JSON object per line: {"key": "...", "ms": t, "opts": {"name": v, ...}}
bool tune_cache_lookup(const char* path, const std::string& key, spg_opts* o) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line, want = "\"key\": \"" + key + "\"";
    bool found = false;
    while (std::getline(f, line)) {
        if (line.find(want) == std::string::npos) continue;
        spg_opts t = *o;
        bool ok = true;
        for (const TuneKnob& k : tune_knobs()) {
            const std::string field = "\"" + std::string(k.name) + "\": ";
            size_t p = line.find(field);
            if (p == std::string::npos) {
                ok = false;
                break;
            }
            t.*(k.field) = (int32_t)std::strtol(line.c_str() + p + field.size(), nullptr, 10);
        }
        if (ok) {
            *o = t;  // the last matching line wins
            found = true;
        }
    }
    return found;
}

bool tune_cache_store(const char* path, const std::string& key, const spg_opts& o, double ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return false;
    std::fprintf(f, "{\"key\": \"%s\", \"ms\": %.4f, \"opts\": {", key.c_str(), ms);
    bool first = true;
    for (const TuneKnob& k : tune_knobs()) {
        std::fprintf(f, "%s\"%s\": %d", first ? "" : ", ", k.name, (int)(o.*(k.field)));
        first = false;
    }
    std::fprintf(f, "}}\n");
    return std::fclose(f) == 0;
}

}  // namespace

// Time one candidate: a fresh plan on the caller's stream, one eager call
// (which captures the graph), one warm replay, then `reps` replays between
// two events.
static spg_status tune_time(spg_plan P, const spg_opts& o, spg_semiring sr, int32_t nb, const spg_csr* RT,
                            const spg_csr* A, const spg_csr* R, spg_csr* out, int reps, float* ms) {
    spg_plan T = nullptr;
    SPG_TRY(spg_plan_create(&T, (void*)P->stream, &o));
    spg_status st = spgemm_galerkin_batched(T, sr, nb, RT, A, R, out, 1);
    if (st == SPG_OK) st = spgemm_galerkin_batched(T, sr, nb, RT, A, R, out, 1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == SPG_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(SPG_ERR_HIP, "hipEventCreate failed");
    if (st == SPG_OK) {
        hipEventRecord(e0, P->stream);
        for (int r = 0; r < reps && st == SPG_OK; ++r) st = spgemm_galerkin_batched(T, sr, nb, RT, A, R, out, 1);
        hipEventRecord(e1, P->stream);
        if (hipEventSynchronize(e1) != hipSuccess) st = fail(SPG_ERR_HIP, "timing event failed");
        float t = 0.f;
        if (st == SPG_OK) {
            hipEventElapsedTime(&t, e0, e1);
            *ms = t / (float)reps;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    spg_plan_destroy(T);
    return st;
}

extern "C" spg_status spg_autotune_galerkin(spg_plan P, spg_semiring sr, int32_t nb, const spg_csr* RT,
                                            const spg_csr* A, const spg_csr* R, const char* cache_path,
                                            int32_t budget_ms, spg_opts* best, int32_t* from_cache) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    if (nb < 1 || !RT || !A || !R) return fail(SPG_ERR_ARG, "need nb >= 1 and non-NULL arrays");
    if (from_cache) *from_cache = 0;
    const std::string key = tune_key(P->device, sr, nb, RT, A, R);
    spg_opts cur = P->opts;
    cur.profile = 0;
    if (cache_path && tune_cache_lookup(cache_path, key, &cur)) {
        if (from_cache) *from_cache = 1;
    } else {
        std::vector<spg_csr> out((size_t)nb);
        const auto t_start = std::chrono::steady_clock::now();
        auto elapsed_ms = [&] {
            return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        };
        float best_ms = 0.f;
        SPG_TRY(tune_time(P, cur, sr, nb, RT, A, R, out.data(), 5, &best_ms));
        // coordinate descent: each knob over its candidates, the others
        // held at the best so far; two sweeps or until the budget is spent
        for (int sweep = 0; sweep < 2; ++sweep) {
            bool improved = false;
            for (const TuneKnob& k : tune_knobs()) {
                for (int32_t v : k.values) {
                    if (budget_ms > 0 && elapsed_ms() > budget_ms) break;
                    if (cur.*(k.field) == v) continue;
                    spg_opts cand = cur;
                    cand.*(k.field) = v;
                    if (cand.chunk_min_nnz > cand.hash_max_nnz) cand.chunk_min_nnz = cand.hash_max_nnz;
                    float t = 0.f;
                    SPG_TRY(tune_time(P, cand, sr, nb, RT, A, R, out.data(), 5, &t));
                    if (t < 0.98f * best_ms) {  // a clear gain only
                        best_ms = t;
                        cur = cand;
                        improved = true;
                    }
                }
            }
            if (!improved) break;
        }
        if (cache_path && !tune_cache_store(cache_path, key, cur, best_ms))
            return fail(SPG_ERR_ARG, std::string("cannot append to the tuning cache ") + cache_path);
    }
    // the plan takes the chosen options; its batched state starts afresh
    const int32_t prof = P->opts.profile, val = P->opts.validate;
    spg_release_galerkin(P);
    P->opts = cur;
    P->opts.profile = prof;
    P->opts.validate = val;
    if (best) *best = cur;
    return SPG_OK;
}

// ---------------------------------------------------------------------------
// distance-2 maximal independent set, aggregation, restriction operator
// ---------------------------------------------------------------------------
static const int32_t MIS_MAX_ROUNDS = 4096;

static unsigned grid_rows(int64_t n) { return grid_for(n * MIS_LANES, 256); }

extern "C" spg_status spg_mis2_aggregate(spg_plan P, const spg_csr* A, uint64_t seed, uint8_t* in_mis, int32_t* agg,
                                         int64_t* n_agg, int32_t* rounds) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->cur = nullptr;
    SPG_TRY(check_csr(A, "A", SPG_SR_OR_AND_BOOL, false));
    if (A->nrows != A->ncols) return fail(SPG_ERR_SHAPE, "A must be square (a graph)");
    if (!in_mis || !agg || !n_agg) return fail(SPG_ERR_ARG, "in_mis, agg and n_agg must not be NULL");
    const int64_t n = A->nrows;
    if (rounds) *rounds = 0;
    *n_agg = 0;
    if (n == 0) return SPG_OK;
    if (P->opts.validate) SPG_TRY(validate_csr(P, A, "A"));
    SPG_TRY(P->mis_key.ensure(8 * (size_t)n, "MIS-2 keys"));
    SPG_TRY(P->mis_m1.ensure(8 * (size_t)n, "MIS-2 minima"));
    SPG_TRY(P->mis_cand.ensure((size_t)n, "MIS-2 candidates"));
    SPG_TRY(P->mis_new.ensure((size_t)n, "MIS-2 new vertices"));
    SPG_TRY(P->mis_a1.ensure((size_t)n, "MIS-2 neighbourhood"));
    SPG_TRY(P->mis_flags.ensure(8 * (size_t)(n + 1), "MIS-2 root numbers"));
    SPG_TRY(P->mis_agg1.ensure(4 * (size_t)n, "aggregates"));
    SPG_TRY(P->mis_ctr.ensure(64, "counters"));
    Csr a = view(A);
    uint8_t* cand = P->mis_cand.as<uint8_t>();
    uint8_t* news = P->mis_new.as<uint8_t>();
    uint8_t* a1 = P->mis_a1.as<uint8_t>();
    uint64_t* key = P->mis_key.as<uint64_t>();
    uint64_t* m1 = P->mis_m1.as<uint64_t>();
    int32_t* ctr = P->mis_ctr.as<int32_t>();
    // fill kernels, not memsets (the sequence may be captured)
    auto fill_u8 = [&](uint8_t* p, uint8_t v) -> spg_status {
        return launch(P, "fill", [&] { k_fill_bytes<<<grid_for(n, 256), 256, 0, cs(P)>>>(p, n, v); });
    };
    SPG_TRY(fill_u8(cand, 1));
    SPG_TRY(fill_u8(in_mis, 0));
    int32_t r = 0;
    for (;; ++r) {
        if (r >= MIS_MAX_ROUNDS) return fail(SPG_ERR_STATE, "MIS-2 did not finish (pattern not symmetric?)");
        SPG_TRY(fill_i32(P, ctr, 1, 0));
        SPG_TRY(launch(P, "mis_keys", [&] {
            k_mis_keys<<<grid_for(n, 256), 256, 0, cs(P)>>>(n, cand, seed, r, key);
        }));
        SPG_TRY(launch(P, "mis_row_min", [&] { k_mis_row_min<<<grid_rows(n), 256, 0, cs(P)>>>(a, key, m1); }));
        SPG_TRY(launch(P, "mis_select", [&] { k_mis_select<<<grid_rows(n), 256, 0, cs(P)>>>(a, key, m1, cand, news); }));
        SPG_TRY(launch(P, "mis_row_any", [&] { k_mis_row_any<<<grid_rows(n), 256, 0, cs(P)>>>(a, news, a1); }));
        SPG_TRY(launch(P, "mis_prune", [&] {
            k_mis_prune<<<grid_rows(n), 256, 0, cs(P)>>>(a, a1, news, cand, in_mis, ctr);
        }));
        int32_t left = 0;
        HIP_TRY(hipMemcpyAsync(&left, ctr, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
        HIP_TRY(hipStreamSynchronize(P->stream));
        if (left == 0) break;
    }
    if (rounds) *rounds = r + 1;
    // aggregates: roots numbered in vertex order, then their neighbours, then the rest
    int64_t* flags = P->mis_flags.as<int64_t>();
    SPG_TRY(launch(P, "mis_flags", [&] { k_mis_flags<<<grid_for(n, 256), 256, 0, cs(P)>>>(n, in_mis, flags); }));
    SPG_TRY(scan_counts(P, flags, n));
    int32_t* agg1 = P->mis_agg1.as<int32_t>();
    SPG_TRY(launch(P, "agg_roots", [&] { k_agg_roots<<<grid_rows(n), 256, 0, cs(P)>>>(a, in_mis, flags, agg1); }));
    SPG_TRY(fill_i32(P, ctr + 1, 1, 0));
    SPG_TRY(launch(P, "agg_rest", [&] { k_agg_rest<<<grid_rows(n), 256, 0, cs(P)>>>(a, agg1, seed, agg, ctr + 1); }));
    int64_t h[2] = {0, 0};
    int32_t un = 0;
    HIP_TRY(hipMemcpyAsync(&h[0], flags + n, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipMemcpyAsync(&un, ctr + 1, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    if (un) return fail(SPG_ERR_STATE, "some vertices are farther than two hops from the independent set");
    *n_agg = h[0];
    return SPG_OK;
}

template <int SR>
static spg_status restriction_sr(spg_plan P, int64_t n, int64_t na, const int32_t* agg, int64_t* r_rp, int32_t* r_col,
                                 void* r_val, int64_t* rt_rp, int32_t* rt_col, void* rt_val) {
    SPG_TRY(fill_i64(P, rt_rp, na + 1, 0));
    if (n == 0) return fill_i64(P, r_rp, 1, 0);
    SPG_TRY(launch(P, "restrict_rows", [&] {
        k_restrict_rows<SR><<<grid_for(n + 1, 256), 256, 0, cs(P)>>>(n, agg, r_rp, r_col, r_val, rt_rp);
    }));
    SPG_TRY(scan_counts(P, rt_rp, na));
    SPG_TRY(P->mis_flags.ensure(8 * (size_t)(na + 1), "restriction cursors"));
    int64_t* cursor = P->mis_flags.as<int64_t>();
    SPG_TRY(fill_i64(P, cursor, na, 0));
    SPG_TRY(launch(P, "restrict_cols", [&] {
        k_restrict_cols<SR><<<grid_for(n, 256), 256, 0, cs(P)>>>(n, agg, rt_rp, cursor, rt_col, rt_val);
    }));
    SPG_TRY(P->mis_ctr.ensure(64, "counters"));
    int32_t* ctr = P->mis_ctr.as<int32_t>();
    SPG_TRY(fill_i32(P, ctr + 2, 1, 0));
    SPG_TRY(launch(P, "sort_row_cols", [&] {
        k_sort_row_cols<<<(unsigned)na, 64, 0, cs(P)>>>(na, rt_rp, rt_col, ctr + 2);
    }));
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, ctr + 2, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    if (bad) return fail(SPG_ERR_CAPACITY, "an aggregate has more than 4096 vertices");
    return SPG_OK;
}

extern "C" spg_status spg_restriction(spg_plan P, spg_semiring sr, int64_t n, int64_t n_agg, const int32_t* agg,
                                      int64_t* r_rp, int32_t* r_col, void* r_val, int64_t* rt_rp, int32_t* rt_col,
                                      void* rt_val) {
    if (!P) return fail(SPG_ERR_ARG, "plan is NULL");
    P->cur = nullptr;
    if ((int)sr < 0 || (int)sr > 2) return fail(SPG_ERR_ARG, "unknown semiring");
    if (n < 0 || n_agg < 0 || (n > 0 && n_agg < 1) || n >= (1ll << 31) || n_agg > n)
        return fail(SPG_ERR_ARG, "need 0 <= n < 2^31 and 1 <= n_agg <= n");
    if (!r_rp || !rt_rp || (n > 0 && (!agg || !r_col || !rt_col)))
        return fail(SPG_ERR_ARG, "NULL output or aggregate array");
    if (n > 0 && n_agg > (int64_t)UINT32_MAX) return fail(SPG_ERR_INDEX_RANGE, "too many aggregates");
    switch (sr) {
        case SPG_SR_PLUS_TIMES_F64: return restriction_sr<SR_F64>(P, n, n_agg, agg, r_rp, r_col, r_val, rt_rp, rt_col, rt_val);
        case SPG_SR_PLUS_TIMES_I64: return restriction_sr<SR_I64>(P, n, n_agg, agg, r_rp, r_col, r_val, rt_rp, rt_col, rt_val);
        case SPG_SR_OR_AND_BOOL: return restriction_sr<SR_BOOL>(P, n, n_agg, agg, r_rp, r_col, r_val, rt_rp, rt_col, rt_val);
    }
    return fail(SPG_ERR_ARG, "unknown semiring");
}
