// cse_api.hip -- host runtime of libcse: the C ABI declared in include/cse.h.
//
// A context owns loaded schemes (input systems as column bitsets in HBM),
// jobs (per-unit state and programs of one scheme run) and batches (the
// jobs that share launches).  A batch is executed by launch groups: one
// step-kernel launch per (row-word count W, state placement) covering the
// units of all its jobs' components, described by a segment table in device
// memory.  With sharing (Sec. 3.5.2) the host runs rounds: every group
// advances its units by at most share_every steps, each component pool
// counts its active units, ranks them and copies prefixes, and the host
// reads the counts.  A server is a batch whose job set changes between
// rounds: jobs are admitted as device memory frees up and join the next
// round's launches (continuous batching); every job keeps its own round
// counter, so its results are those of running alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cse.h"
#include "cse_flip.hpp"
#include "cse_input.hpp"
#include "cse_kernels.hpp"
#include "cse_share.hpp"
#include "cse_step.hpp"

// Working memory of cse_reduce_static, for callers that cannot allocate:
// a file-scope device array, one copy per GPU, kept until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returned for the current device, recorded once per
// device by cse_ctx_create.
static constexpr size_t kStaticScratchBytes = CSE_STATIC_SCRATCH_BYTES;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

namespace {

constexpr int kMaxRows = 512;          // W <= 8 row words
constexpr int kMaxVars = 32767;        // 15-bit variable ids
constexpr int kMaskBudgetWords = 1024; // gi masks: at most 8 KB per unit (64-bit words)
// LDS of one gfx950 CU.  A unit (one wave) whose state would let fewer than
// four units share a CU, one per SIMD, keeps the bulk of it in HBM (one slot
// per unit) and only the variable lists in LDS.
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr int kMinUnitsPerCu = 4;
// Cancellation flags (pinned host memory read by the kernels): jobs alive at once.
constexpr int kCancelSlots = 1 << 16;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct DevComp {
    int n_e = 0, n_x = 0, n_fmax = 0, W = 0, m_cap = 0, naive0 = 0, newc_cap = 0, m_words = 0, m0 = 0;
    bool gs = false;   // bulk state in HBM
    bool adj = false;  // gi over per-variable ranges (large candidate sets)
    bool tl = false;   // with gs and adj: the range tables in LDS
    int nw = 1;        // waves per unit (1, 2 or 4; more than one with adj)
    int kbits = 1;     // weight bit-planes per ordering
    long long occ0 = 0;
    int8_t* d_A = nullptr;        // the input, rows x cols row-major
    uint64_t* d_P = nullptr;
    uint64_t* d_N = nullptr;
    uint64_t* d_cand0 = nullptr;  // candidates of the input system, canonical order
    uint32_t* d_tl0 = nullptr;    // the same by (second, first, sign)
    uint64_t* d_cand0_g = nullptr;  // the same two lists counted on the matrix cores
    uint32_t* d_tl0_g = nullptr;
};

struct SchemeRec {
    int n_comp = 0;
    DevComp comp[3];
};

struct CompJob {
    csek::UnitState st{};
    void* block = nullptr;  // one allocation for all per-unit arrays
    size_t bytes = 0;
};

struct JobRec {
    int scheme = -1;
    cse_run_cfg cfg{};
    int n_comp = 0;
    CompJob cj[3];
    int batch = -1;
    unsigned long long* d_t0 = nullptr;  // device clock at the start of the latest run
    int32_t* d_share = nullptr;          // sharing scratch of its pools
    int budget = -1;                     // selection steps per launch (< 0: to completion)
    uint32_t round = 0;                  // rounds completed in the latest run
    bool done = false;                   // every unit finished (round-driven runs)
    bool allocated = false;
    bool server = false;                 // owned by a server
    int state = CSE_JOB_DONE;            // CSE_JOB_* (server jobs)
    int cancel_slot = -1;                // its flag in the context's cancellation array
    bool cancelled = false;
    int32_t* d_best = nullptr;           // per-component best cost (cse_poll)
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    size_t bytes = 0;                    // device footprint
    // Outer iterations (cse_run_driver): each component's best program so far.
    bool driver = false;
    bool driver_running = false;
    uint32_t* d_bestprog = nullptr;          // per component max(1, n_fmax) keys
    unsigned long long* d_key = nullptr;     // per component argmin key
    int32_t best_cost[3] = {-1, -1, -1}, best_iter[3] = {0, 0, 0}, best_proc[3] = {0, 0, 0};
    std::vector<uint32_t> best_keys[3];
    std::vector<int32_t> totals;             // best total after each iteration
    std::vector<uint64_t> iter_ns;           // host time from the driver start to each iteration's end
};

struct LaunchGroup {
    int W = 0;
    bool gs = false;
    bool adj = false;
    bool tl = false;
    int nw = 1;                     // waves per unit
    bool gp = false;                // some job gives Greedy-Potential a weight
    uint32_t n_grid = 0;
    size_t lds = 0;
    int seg_begin = 0, n_segs = 0;  // slice of the batch's segment table
    size_t order_begin = 0;         // slice of the batch's dispatch order
};

struct Pool {  // the units of one component of one job
    int job = 0, comp = 0;
    uint32_t n = 0, n_src = 0;
    bool shares = false;
    int32_t* scratch = nullptr;
};

struct BatchRec {
    std::vector<int> jobs;            // jobs launched by this batch (unfinished ones for a server)
    std::vector<csek::Segment> segs;  // host copy of the segment table
    std::vector<int> seg_job;         // job of each segment
    csek::Segment* d_segs = nullptr;
    size_t segs_cap = 0;
    std::vector<LaunchGroup> groups;
    std::vector<Pool> pools;
    std::vector<uint32_t> order;      // dispatch order of every group, concatenated
    uint32_t* d_order = nullptr;
    size_t order_cap = 0;
    bool built = false;               // tables match the current jobs and configurations
    bool rounds = false;  // host-driven rounds (sharing or server)
    hipStream_t stream = nullptr;
    hipEvent_t ev_done = nullptr;
    bool finished = true;
    int* d_err = nullptr;
    int32_t* d_counts = nullptr;  // active units per pool
    int32_t* h_counts = nullptr;  // pinned copy
    size_t counts_cap = 0;
    bool is_server = false;
    cse_server* owner = nullptr;      // the server running this batch
    // Round-driven batches: the pools' table, and one round (every group's
    // launch, the pool kernels, the count copy) captured as a graph and
    // replayed on an internal stream.
    csek::PoolDev* d_pools = nullptr;
    std::vector<csek::PoolDev> hpools;  // host copy of the pools' table
    size_t dpools_cap = 0;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_order = nullptr;
    // The groups of a launch run side by side: group g > 0 on side[g - 1],
    // forked from the launching stream by ev_fork and joined back by
    // ev_join[g - 1] (also inside a captured round, where they become edges).
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint32_t pool_grid_x = 1;
    // Kernel timing (context switch): two events per launch group, the
    // groups' launches not yet read, and device time per class (W, layout)
    // since the run started.
    std::vector<hipEvent_t> tev;
    std::vector<int> t_pending;
    std::map<std::pair<int, int>, std::pair<int32_t, uint64_t>> t_class;
};

}  // namespace

// A random-flip run (Sec. 3.5.3): the best variant found, with its
// matrices, component costs and programs, and the best total per iteration.
struct FlipRun {
    int n = 0, m = 0, p = 0, r = 0;
    std::vector<int8_t> U, V, W;
    int32_t best_cost[3] = {-1, -1, -1};
    int32_t best_total = -1, variant = -1, iteration = -1;
    std::vector<uint32_t> keys[3];
    std::vector<int32_t> totals;
};

struct cse_ctx {
    int device = 0;
    std::string err;
    std::map<int, SchemeRec> schemes;
    std::map<int, JobRec> jobs;
    std::map<int, BatchRec> batches;
    std::map<int, FlipRun> flips;
    int next_scheme = 1, next_job = 1, next_batch = 1, next_flip = 1;
    size_t lds_max = 65536;
    uint64_t tick_hz = 100000000ull;
    bool timing = false;          // step-kernel launches bracketed by events
    int32_t* h_cancel = nullptr;  // kCancelSlots flags, pinned host memory
    int32_t* d_cancel = nullptr;  // the same as seen by the device
    std::vector<int> free_slots;
};

struct cse_server {
    cse_ctx* ctx = nullptr;
    int batch = -1;
    uint64_t max_bytes = 0, used_bytes = 0;
    uint32_t round_steps = 32;
    std::deque<int> queue;
    bool dirty = true;  // job set changed since the segment table was built
};

namespace {

int fail(cse_ctx* ctx, int code, const char* fmt, ...) {
    // A failed runtime call (an allocation beyond device memory, say) stays
    // HIP's last error until read; later launch checks must not see it.
    if (code == CSE_EHIP) (void)hipGetLastError();
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, expr)                                                                          \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail((ctx), CSE_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t bulk_bytes(const DevComp& c) {
    // Units of several waves keep 32-bit candidate entries.
    return csek::bulk_layout(c.n_x + c.n_fmax, c.W, c.m_cap, c.newc_cap, c.m_words, c.adj ? 1 : 0, c.kbits,
                             c.nw > 1 ? 4 : 8)
        .bytes;
}
size_t lds_bytes(const DevComp& c) {
    const int n_vmax = c.n_x + c.n_fmax;
    if (c.gs && c.tl) return csek::table_layout(n_vmax, c.m_cap, c.kbits).bytes;
    // Units of several waves keep the new-pair table after the lists, and
    // with HBM state the LDS budget for gi's per-step tables.
    const size_t multi = c.nw > 1 ? csek::newpair_table_bytes(n_vmax) + (c.gs ? csek::kGsTableBudget : 0) : 0;
    return (c.gs ? 0 : bulk_bytes(c)) + csek::list_bytes(n_vmax) + multi;
}

void free_component(DevComp& c) {
    for (void* p : {(void*)c.d_A, (void*)c.d_P, (void*)c.d_N, (void*)c.d_cand0, (void*)c.d_tl0,
                    (void*)c.d_cand0_g, (void*)c.d_tl0_g})
        if (p) (void)hipFree(p);
    c.d_A = nullptr;
    c.d_P = c.d_N = c.d_cand0 = c.d_cand0_g = nullptr;
    c.d_tl0 = c.d_tl0_g = nullptr;
}

// Analysis of the input system on the device (Sec. 3.3), synchronous: pair
// counts by popcounts of the column bitsets, or (gram) from the int8 Gram
// matrix [P N]^T [P N] on the matrix cores; then the candidate list in
// canonical order and the second ordering.  *m receives the candidate count.
int analyse_input(cse_ctx* ctx, const DevComp& c, bool gram, uint64_t** cand_out, uint32_t** tl_out, int* m) {
    const int n = c.n_x;
    int32_t* buf = nullptr;  // row_n, col_n, row_off, col_off, totals
    int8_t* X = nullptr;
    int32_t* G = nullptr;
    uint64_t* cand = nullptr;
    uint32_t* tl = nullptr;
    int rc = CSE_OK;
    int32_t tot[2] = {0, 0};
    const int F = (2 * n + 31) / 32 * 32, Kp = (c.n_e + 15) / 16 * 16;
    csek::PairSource src{c.d_P, c.d_N, c.W, nullptr, F, n};
    auto cleanup = [&]() {
        if (buf) (void)hipFree(buf);
        if (X) (void)hipFree(X);
        if (G) (void)hipFree(G);
    };
#define IN_TRY(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            rc = fail(ctx, CSE_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                          \
            cleanup();                                                                                 \
            if (cand) (void)hipFree(cand);                                                             \
            if (tl) (void)hipFree(tl);                                                                 \
            return rc;                                                                                 \
        }                                                                                              \
    } while (0)
    IN_TRY(hipMalloc((void**)&buf, sizeof(int32_t) * (4 * (size_t)n + 4)));
    int32_t* row_n = buf;
    int32_t* col_n = buf + n;
    int32_t* row_off = buf + 2 * n;
    int32_t* col_off = buf + 3 * n + 1;
    int32_t* d_tot = buf + 4 * n + 2;
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, nullptr, buf, 2 * n, 0);
    if (gram) {
        IN_TRY(hipMalloc((void**)&X, (size_t)F * Kp));
        IN_TRY(hipMalloc((void**)&G, (size_t)F * F * 4));
        const size_t nx = (size_t)F * Kp;
        hipLaunchKernelGGL(csek::input_features_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, nullptr,
                           c.d_A, c.n_e, n, Kp, F, X);
        hipLaunchKernelGGL(csek::input_gram_kernel, dim3(F / 32, F / 32), dim3(64), 0, nullptr, X, Kp, F, G);
        src.G = G;
    }
    hipLaunchKernelGGL(csek::input_count_kernel, dim3(n), dim3(csek::kInputBlock), 0, nullptr, src, row_n, col_n);
    hipLaunchKernelGGL(csek::input_scan_kernel, dim3(1), dim3(csek::kInputBlock), 0, nullptr, row_n, col_n, n,
                       row_off, col_off, d_tot);
    IN_TRY(hipGetLastError());
    IN_TRY(hipMemcpy(tot, d_tot, sizeof tot, hipMemcpyDeviceToHost));
    if (tot[0] != tot[1] || tot[0] < 0) {
        cleanup();
        return fail(ctx, CSE_EHIP, "input analysis: %d candidates by first variable, %d by second", tot[0], tot[1]);
    }
    IN_TRY(hipMalloc((void**)&cand, std::max<size_t>(1, tot[0]) * 8));
    IN_TRY(hipMalloc((void**)&tl, std::max<size_t>(1, tot[0]) * 4));
    hipLaunchKernelGGL(csek::input_rows_kernel, dim3(n), dim3(csek::kInputBlock), 0, nullptr, src, row_off, cand);
    hipLaunchKernelGGL(csek::input_cols_kernel, dim3(n), dim3(csek::kInputBlock), 0, nullptr, src, row_off, col_off,
                       cand, tl);
    IN_TRY(hipGetLastError());
    IN_TRY(hipStreamSynchronize(nullptr));
#undef IN_TRY
    cleanup();
    *cand_out = cand;
    *tl_out = tl;
    *m = tot[0];
    return CSE_OK;
}

// Candidate lists counted on the matrix cores, computed on first use; they
// must equal the popcount lists' size (the counts are the same integers).
int ensure_gram_lists(cse_ctx* ctx, DevComp& c) {
    if (c.d_cand0_g) return CSE_OK;
    int m = 0;
    int rc = analyse_input(ctx, c, true, &c.d_cand0_g, &c.d_tl0_g, &m);
    if (rc) return rc;
    if (m != c.m0) return fail(ctx, CSE_EHIP, "matrix-core count path found %d candidates, popcounts %d", m, c.m0);
    return CSE_OK;
}

// Layout of a component (CSE_LAYOUT_*): bulk state in HBM slots instead of
// LDS, gi over per-variable ranges instead of masks, for HBM state with
// ranges the range tables in LDS, and the waves per unit (1, 2 or 4; more
// than one only with ranges).  Results do not depend on it.
constexpr int kLayoutMax = CSE_LAYOUT_HBM | CSE_LAYOUT_RANGE | CSE_LAYOUT_LDS_TABLES | CSE_LAYOUT_WAVES4;
// Waves per unit that loading gives HBM-state range-form components.
constexpr int kDefaultHbmRangeWaves = 4;
bool layout_valid(int layout) {
    if (layout < 0 || layout > kLayoutMax) return false;
    const int wb = (layout >> CSE_LAYOUT_WAVES_SHIFT) & 3;
    if (wb == 3 || (wb && !(layout & CSE_LAYOUT_RANGE))) return false;
    return !(layout & CSE_LAYOUT_LDS_TABLES) || (layout & (CSE_LAYOUT_HBM | CSE_LAYOUT_RANGE)) ==
                                                      (CSE_LAYOUT_HBM | CSE_LAYOUT_RANGE);
}
int waves_bits(int nw) { return nw == 4 ? CSE_LAYOUT_WAVES4 : nw == 2 ? CSE_LAYOUT_WAVES2 : 0; }
int layout_code(const DevComp& c) {
    return (c.gs ? CSE_LAYOUT_HBM : 0) | (c.adj ? CSE_LAYOUT_RANGE : 0) | (c.tl ? CSE_LAYOUT_LDS_TABLES : 0) |
           waves_bits(c.nw);
}
void set_layout(DevComp& c, int layout) {
    c.gs = (layout & CSE_LAYOUT_HBM) != 0;
    c.adj = (layout & CSE_LAYOUT_RANGE) != 0;
    c.tl = (layout & CSE_LAYOUT_LDS_TABLES) != 0;
    c.nw = 1 << ((layout >> CSE_LAYOUT_WAVES_SHIFT) & 3);
}

// Sizes of a component from its nonzeros, pair occurrences and naive count
// (Sec. 3.2.1); n_e and n_x are set.  Host arithmetic only.
int size_component(cse_ctx* ctx, DevComp& c, long long nnz, long long occ, long long naive) {
    const int rows = c.n_e, cols = c.n_x;
    // Each substitution removes c >= 2 nonzeros and no row empties, so at
    // most floor((nnz - n_e) / 2) fresh variables; every candidate uses at
    // least two of the pair occurrences, whose number never grows.
    c.n_fmax = (int)((nnz - rows) / 2);
    if ((long long)cols + c.n_fmax > kMaxVars)
        return fail(ctx, CSE_EINVAL, "variables %lld exceed %d", (long long)cols + c.n_fmax, kMaxVars);
    c.W = (rows + 63) / 64;
    c.occ0 = occ;
    // The range form of gi packs candidate indices in 23 bits.
    if (occ / 2 >= (1ll << 23)) return fail(ctx, CSE_EINVAL, "%lld candidates exceed 2^23", occ / 2);
    c.m_cap = (int)std::max<long long>(1, occ / 2);
    c.kbits = csek::weight_bits(rows);
    c.naive0 = (int)naive;
    c.newc_cap = std::max(1, std::min(c.m_cap, 2 * (cols + c.n_fmax)));
    return CSE_OK;
}

// Layout of a component once the input's candidate count c.m0 is known.
int pick_layout(cse_ctx* ctx, DevComp& c) {
    const int cols = c.n_x, n_vmax = c.n_x + c.n_fmax;
    // Large candidate sets walk per-variable ranges in gi instead of masks.
    c.adj = (long long)cols * ((c.m0 + 63) / 64) > kMaskBudgetWords * 3 / 4;
    // Mask capacity: twice the input's need (live variables x 32-bit words of
    // candidates), at least 1 KB, at most the budget; a step that needs more
    // takes the exact O(m^2) form.
    const long long full32 = (long long)n_vmax * ((c.m_cap + 31) / 32);
    const long long want32 = std::max<long long>(2ll * cols * ((c.m0 + 31) / 32), 256);
    const long long words32 = std::min<long long>({full32, want32, 2ll * kMaskBudgetWords});
    c.m_words = (int)std::max<long long>(1, (words32 + 1) / 2);
    // Too large for four units per CU: state in HBM, and gi over ranges, which
    // touches far less of that state per step than building masks does.
    if (kMinUnitsPerCu * (bulk_bytes(c) + csek::list_bytes(n_vmax)) > kLdsPerCu) c.gs = c.adj = true;
    // Those units wait on memory; they run on several waves (whose 32-bit
    // candidate entries hold variable ids below 2048).
    c.nw = c.gs && c.adj && n_vmax <= csek::kCompactMaxVars ? kDefaultHbmRangeWaves : 1;
    // Every layout keeps the variable lists in LDS.
    if (lds_bytes(c) > ctx->lds_max)
        return fail(ctx, CSE_ENOMEM, "%d variables need %zu B of LDS for their lists (max %zu)", n_vmax,
                    lds_bytes(c), ctx->lds_max);
    return CSE_OK;
}

// A component from an input already copied to c->d_A (rows x cols int8)
// and its sizes: nonzeros, pair occurrences and naive count (Sec. 3.2.1).
// Builds the bitsets, analyses the input and picks the layout; frees the
// component on error.
int finish_component(cse_ctx* ctx, DevComp& c, long long nnz, long long occ, long long naive, DevComp* out) {
    const int rows = c.n_e, cols = c.n_x;
    int rc = size_component(ctx, c, nnz, occ, naive);
    if (rc) {
        free_component(c);
        return rc;
    }
    const size_t col_bytes = (size_t)cols * c.W * 8;
    hipError_t e = hipMalloc(&c.d_P, col_bytes);
    if (e == hipSuccess) e = hipMalloc(&c.d_N, col_bytes);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(csek::input_columns_kernel, dim3((cols * c.W + 255) / 256), dim3(256), 0, nullptr,
                           c.d_A, rows, cols, c.W, c.d_P, c.d_N);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        free_component(c);
        return fail(ctx, CSE_EHIP, "loading a %d x %d system: %s", rows, cols, hipGetErrorString(e));
    }
    // The input's candidates, shared by every unit at its first step.
    rc = analyse_input(ctx, c, false, &c.d_cand0, &c.d_tl0, &c.m0);
    if (rc == CSE_OK) rc = pick_layout(ctx, c);
    if (rc) {
        free_component(c);
        return rc;
    }
    *out = c;
    return CSE_OK;
}

// A component from a host matrix (copied; the caller keeps it).
int load_component(cse_ctx* ctx, const int8_t* A, int rows, int cols, DevComp* out) {
    if (!A || rows < 1 || cols < 1) return fail(ctx, CSE_EINVAL, "empty system (%d x %d)", rows, cols);
    if (rows > kMaxRows) return fail(ctx, CSE_EINVAL, "rows %d exceed %d", rows, kMaxRows);
    long long nnz = 0, occ = 0, naive = 0;
    for (int i = 0; i < rows; ++i) {
        long long r = 0;
        for (int j = 0; j < cols; ++j) {
            const int8_t v = A[(size_t)i * cols + j];
            if (v < -1 || v > 1) return fail(ctx, CSE_EINVAL, "entry (%d,%d) = %d not ternary", i, j, v);
            r += v != 0;
        }
        if (r == 0) return fail(ctx, CSE_EINVAL, "row %d is all zero", i);
        nnz += r;
        occ += r * (r - 1) / 2;
        naive += r - 1;
    }
    DevComp c;
    c.n_e = rows;
    c.n_x = cols;
    hipError_t e = hipMalloc(&c.d_A, (size_t)rows * cols);
    if (e == hipSuccess) e = hipMemcpy(c.d_A, A, (size_t)rows * cols, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_component(c);
        return fail(ctx, CSE_EHIP, "loading a %d x %d system: %s", rows, cols, hipGetErrorString(e));
    }
    return finish_component(ctx, c, nnz, occ, naive, out);
}

// A component from a device matrix (copied on `stream` after the caller's
// work there; the caller keeps it), validated and sized on the device.
int load_component_device(cse_ctx* ctx, const int8_t* dA, int rows, int cols, hipStream_t stream,
                          unsigned long long* d_st, DevComp* out) {
    if (!dA || rows < 1 || cols < 1) return fail(ctx, CSE_EINVAL, "empty system (%d x %d)", rows, cols);
    if (rows > kMaxRows) return fail(ctx, CSE_EINVAL, "rows %d exceed %d", rows, kMaxRows);
    DevComp c;
    c.n_e = rows;
    c.n_x = cols;
    unsigned long long st[5] = {0, 0, 0, 0, 0};
    hipError_t e = hipMalloc(&c.d_A, (size_t)rows * cols);
    if (e == hipSuccess) e = hipMemcpyAsync(c.d_A, dA, (size_t)rows * cols, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, stream, (int32_t*)d_st, 10, 0);
        hipLaunchKernelGGL(csek::input_stats_kernel, dim3((rows + 255) / 256), dim3(256), 0, stream, c.d_A, rows, cols,
                           d_st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(st, d_st, sizeof st, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        free_component(c);
        return fail(ctx, CSE_EHIP, "loading a %d x %d device system: %s", rows, cols, hipGetErrorString(e));
    }
    if (st[3] || st[4]) {
        free_component(c);
        return fail(ctx, CSE_EINVAL, "device system %d x %d: %llu entries not ternary, %llu all-zero rows", rows, cols,
                    st[3], st[4]);
    }
    return finish_component(ctx, c, (long long)st[0], (long long)st[1], (long long)st[2], out);
}

bool shares(const cse_run_cfg& c) { return c.share_every > 0 && c.share_src_pm > 0 && c.share_max_rounds > 0; }

int validate_cfg(cse_ctx* ctx, const cse_run_cfg* cfg) {
    if (!cfg) return fail(ctx, CSE_EINVAL, "null configuration");
    if (cfg->n_proc < 1 || cfg->n_proc > (1u << 24)) return fail(ctx, CSE_EINVAL, "n_proc %u out of range", cfg->n_proc);
    unsigned long long tw = 0;
    for (int i = 0; i < 7; ++i) tw += cfg->weights[i];
    if (tw == 0 || tw > 0xFFFFFFFFull) return fail(ctx, CSE_EINVAL, "strategy weights must sum to 1..2^32-1");
    unsigned long long mw = 0;
    for (int i = 0; i < 4; ++i) mw += cfg->mix_weights[i];
    if (cfg->weights[CSE_STRAT_MIX] && (mw == 0 || mw > 0xFFFFFFFFull))
        return fail(ctx, CSE_EINVAL, "mix weights must sum to 1..2^32-1");
    if (cfg->gr_p_q16 > 65536) return fail(ctx, CSE_EINVAL, "gr_p_q16 > 65536");
    if (cfg->share_max_rounds > 1023) return fail(ctx, CSE_EINVAL, "share_max_rounds > 1023");
    if (cfg->share_every > 65535) return fail(ctx, CSE_EINVAL, "share_every > 65535");
    if (cfg->share_src_pm > 1000 || cfg->share_dst_pm > 1000) return fail(ctx, CSE_EINVAL, "per mille > 1000");
    if (cfg->count_path > CSE_COUNT_MFMA) return fail(ctx, CSE_EINVAL, "unknown count path");
    if (cfg->reserved[0] || cfg->reserved[1] || cfg->reserved[2]) return fail(ctx, CSE_EINVAL, "reserved fields must be 0");
    return CSE_OK;
}

// Expected relative work of a unit: steps ~ n_fmax, each scanning the
// candidates (~m_cap / 64 chunks); gi scores every intersecting pair.
double unit_cost(const DevComp& c, uint32_t strat) {
    const double scan = (double)c.n_fmax * (1.0 + c.m_cap / 64.0);
    if (strat == CSE_STRAT_GP) return 4.0 * scan * (1.0 + c.n_fmax / 16.0);
    return strat == CSE_STRAT_GI ? 4.0 * scan : strat == CSE_STRAT_MIX ? 2.6 * scan : scan;
}

csek::RunArgs run_args(cse_ctx* ctx, const JobRec& J) {
    const cse_run_cfg& cfg = J.cfg;
    csek::RunArgs R{};
    R.seed = cfg.seed;
    for (int i = 0; i < 7; ++i) R.weights[i] = cfg.weights[i];
    for (int i = 0; i < 4; ++i) R.mix_weights[i] = cfg.mix_weights[i];
    R.proc0_greedy = cfg.proc0_greedy;
    R.gr_p_q16 = cfg.gr_p_q16;
    R.step_cap = cfg.step_cap;
    R.iteration = cfg.iteration;
    R.budget = J.budget;
    R.n_units = cfg.n_proc;
    R.cancel = J.cancel_slot >= 0 ? ctx->d_cancel + J.cancel_slot : nullptr;
    return R;
}

// gram: the initial lists counted on the matrix cores (count_path MFMA).
csek::CompArgs comp_args(const DevComp& c, int comp, bool gram) {
    csek::CompArgs C{};
    C.P0 = c.d_P;
    C.N0 = c.d_N;
    C.cand0 = gram ? c.d_cand0_g : c.d_cand0;
    C.tl0 = gram ? c.d_tl0_g : c.d_tl0;
    C.m0 = c.m0;
    C.adj = c.adj ? 1 : 0;
    C.n_e = c.n_e;
    C.n_x = c.n_x;
    C.n_fmax = c.n_fmax;
    C.m_cap = c.m_cap;
    C.naive0 = c.naive0;
    C.comp = (uint32_t)comp;
    C.prog_stride = std::max(1, c.n_fmax);
    C.newc_cap = c.newc_cap;
    C.m_words = c.m_words;
    C.kbits = c.kbits;
    return C;
}

// An HBM slot holds a unit's bulk state and, in its last 16 bytes, the
// record of which state that is (256 bytes keep slots aligned).
size_t slot_bytes(const DevComp& c) { return bulk_bytes(c) + 256; }

size_t comp_job_bytes(const DevComp& c, uint32_t n) {
    const size_t prog = (size_t)n * std::max(1, c.n_fmax) * 4;
    const size_t gs = c.gs ? (size_t)n * slot_bytes(c) : 0;
    return gs + prog + 7 * (size_t)n * 4 + 2 * (size_t)n * 8 + 64 * 11;
}

size_t job_bytes(cse_ctx* ctx, int scheme, const cse_run_cfg& cfg) {
    const SchemeRec& sc = ctx->schemes[scheme];
    size_t b = 128;
    for (int c = 0; c < sc.n_comp; ++c) {
        b += comp_job_bytes(sc.comp[c], cfg.n_proc);
        if (shares(cfg)) b += csek::share_scratch_bytes(cfg.n_proc);
    }
    return b;
}

int alloc_comp_job(cse_ctx* ctx, const DevComp& c, uint32_t n, CompJob* cj) {
    const size_t prog = (size_t)n * std::max(1, c.n_fmax) * 4;
    const size_t i32 = (size_t)n * 4;
    const size_t u64 = (size_t)n * 8;
    const size_t gs = c.gs ? (size_t)n * slot_bytes(c) : 0;
    const size_t total = comp_job_bytes(c, n);
    char* base = nullptr;
    HIP_TRY(ctx, hipMalloc((void**)&base, total));
    cj->block = base;
    cj->bytes = total;
    auto take = [&](size_t bytes) { char* p = base; base += (bytes + 63) & ~size_t(63); return p; };
    csek::UnitState& S = cj->st;
    S.gs_base = c.gs ? take(gs) : nullptr;
    S.gs_stride = c.gs ? slot_bytes(c) : 0;
    S.ops = (unsigned long long*)take(u64);
    S.finish = (unsigned long long*)take(u64);
    S.prog = (uint32_t*)take(prog);
    S.t = (int32_t*)take(i32);
    S.cost = (int32_t*)take(i32);
    S.executed = (int32_t*)take(i32);
    S.epoch = (int32_t*)take(i32);
    S.k0 = (int32_t*)take(i32);
    S.active = (int32_t*)take(i32);
    S.strat = (int32_t*)take(i32);
    return CSE_OK;
}

void free_job_device(cse_ctx* ctx, JobRec& J) {
    for (int c = 0; c < J.n_comp; ++c) {
        if (J.cj[c].block) (void)hipFree(J.cj[c].block);
        J.cj[c].block = nullptr;
    }
    if (J.d_t0) (void)hipFree(J.d_t0);
    if (J.d_share) (void)hipFree(J.d_share);
    if (J.d_best) (void)hipFree(J.d_best);
    if (J.d_bestprog) (void)hipFree(J.d_bestprog);
    if (J.d_key) (void)hipFree(J.d_key);
    J.d_t0 = nullptr;
    J.d_share = nullptr;
    J.d_best = nullptr;
    J.d_bestprog = nullptr;
    J.d_key = nullptr;
    if (J.cancel_slot >= 0) ctx->free_slots.push_back(J.cancel_slot);
    J.cancel_slot = -1;
    J.allocated = false;
}

// Device memory of one job: unit arrays per component, start stamp,
// sharing scratch.
int alloc_job(cse_ctx* ctx, JobRec& J) {
    const SchemeRec& sc = ctx->schemes[J.scheme];
    J.n_comp = sc.n_comp;
    J.allocated = true;
    for (int c = 0; c < sc.n_comp; ++c) {
        int rc = alloc_comp_job(ctx, sc.comp[c], J.cfg.n_proc, &J.cj[c]);
        if (rc) return rc;
        J.cj[c].st.t0 = nullptr;
    }
    HIP_TRY(ctx, hipMalloc((void**)&J.d_t0, 64));  // start stamp (8 B), round counter (4 B)
    HIP_TRY(ctx, hipMalloc((void**)&J.d_best, 16));
    if (!ctx->free_slots.empty()) {
        J.cancel_slot = ctx->free_slots.back();
        ctx->free_slots.pop_back();
        __atomic_store_n(&ctx->h_cancel[J.cancel_slot], 0, __ATOMIC_SEQ_CST);
    }
    J.cancelled = false;
    for (int c = 0; c < sc.n_comp; ++c) {
        J.cj[c].st.t0 = J.d_t0;
        J.cj[c].st.round = (int32_t*)((char*)J.d_t0 + 8);
    }
    if (shares(J.cfg))
        HIP_TRY(ctx, hipMalloc((void**)&J.d_share, csek::share_scratch_bytes(J.cfg.n_proc) * sc.n_comp));
    J.bytes = job_bytes(ctx, J.scheme, J.cfg);
    return CSE_OK;
}

void free_batch_device(BatchRec& B) {
    for (hipEvent_t e : B.tev)
        if (e) (void)hipEventDestroy(e);
    B.tev.clear();
    B.t_pending.clear();
    if (B.gexec) (void)hipGraphExecDestroy(B.gexec);
    if (B.gstream) (void)hipStreamDestroy(B.gstream);
    if (B.ev_order) (void)hipEventDestroy(B.ev_order);
    for (hipStream_t x : B.side)
        if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t x : B.ev_join)
        if (x) (void)hipEventDestroy(x);
    if (B.ev_fork) (void)hipEventDestroy(B.ev_fork);
    B.side.clear();
    B.ev_join.clear();
    B.ev_fork = nullptr;
    if (B.d_pools) (void)hipFree(B.d_pools);
    B.gexec = nullptr;
    B.gstream = nullptr;
    B.ev_order = nullptr;
    B.d_pools = nullptr;
    B.dpools_cap = 0;
    if (B.d_segs) (void)hipFree(B.d_segs);
    if (B.d_order) (void)hipFree(B.d_order);
    if (B.d_err) (void)hipFree(B.d_err);
    if (B.d_counts) (void)hipFree(B.d_counts);
    if (B.h_counts) (void)hipHostFree(B.h_counts);
    if (B.ev_done) (void)hipEventDestroy(B.ev_done);
    B.d_segs = nullptr;
    B.d_order = nullptr;
    B.d_err = nullptr;
    B.d_counts = nullptr;
    B.h_counts = nullptr;
    B.ev_done = nullptr;
    B.segs_cap = B.counts_cap = B.order_cap = 0;
}

// The step kernel of a class (row words W, layout, waves per unit); the
// kernels of each W are compiled in their own translation unit.
const void* step_kernel_ptr(const LaunchGroup& G) {
    switch (G.W) {
    case 1: return csek_step_kernel_w1(G.gs, G.adj, G.tl, G.nw);
    case 2: return csek_step_kernel_w2(G.gs, G.adj, G.tl, G.nw);
    case 3: return csek_step_kernel_w3(G.gs, G.adj, G.tl, G.nw);
    case 4: return csek_step_kernel_w4(G.gs, G.adj, G.tl, G.nw);
    case 5: return csek_step_kernel_w5(G.gs, G.adj, G.tl, G.nw);
    case 6: return csek_step_kernel_w6(G.gs, G.adj, G.tl, G.nw);
    case 7: return csek_step_kernel_w7(G.gs, G.adj, G.tl, G.nw);
    case 8: return csek_step_kernel_w8(G.gs, G.adj, G.tl, G.nw);
    default: return nullptr;
    }
}
int group_layout(const LaunchGroup& G) {
    return (G.gs ? CSE_LAYOUT_HBM : 0) | (G.adj ? CSE_LAYOUT_RANGE : 0) | (G.tl ? CSE_LAYOUT_LDS_TABLES : 0) |
           waves_bits(G.nw);
}

// Dynamic LDS above 64 KB must be allowed per kernel before launches (and
// before a launch is captured into a graph).
int set_lds_limit(cse_ctx* ctx, const LaunchGroup& G) {
    if (G.lds <= 65536) return CSE_OK;
    const void* k = step_kernel_ptr(G);
    if (!k) return fail(ctx, CSE_EINVAL, "no step kernel for row words %d, layout %d", G.W, group_layout(G));
    HIP_TRY(ctx, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.lds));
    return CSE_OK;
}

// Segment table, launch groups and pools of the batch's unfinished jobs:
// components grouped by row-word count W and state placement (the kernel is
// specialised on both), then uploaded on the batch's stream.
int build_segments(cse_ctx* ctx, BatchRec& B) {
    for (int jid : B.jobs) {
        JobRec& J = ctx->jobs[jid];
        if (J.done || J.cfg.count_path != CSE_COUNT_MFMA) continue;
        SchemeRec& sc = ctx->schemes[J.scheme];
        for (int c = 0; c < sc.n_comp; ++c) {
            int rc = ensure_gram_lists(ctx, sc.comp[c]);
            if (rc) return rc;
        }
    }
    B.segs.clear();
    B.seg_job.clear();
    B.groups.clear();
    B.pools.clear();
    // Classes (W, placement, gi form, tables, waves per unit): the kernel is
    // specialised on each.
    for (int cls = 0; cls < 120; ++cls) {
        const int W = 1 + cls / 15, k = cls % 15 / 3, nw = 1 << (cls % 3);
        const bool gs = k == 1 || k >= 3, adj = k >= 2, tl = k == 4;
        if (nw > 1 && !adj) continue;
        LaunchGroup G;
        G.W = W;
        G.gs = gs;
        G.adj = adj;
        G.tl = tl;
        G.nw = nw;
        G.seg_begin = (int)B.segs.size();
        uint32_t unit = 0;
        for (int jid : B.jobs) {
            JobRec& J = ctx->jobs[jid];
            if (J.done) continue;
            const SchemeRec& sc = ctx->schemes[J.scheme];
            for (int c = 0; c < J.n_comp; ++c) {
                const DevComp& dc = sc.comp[c];
                if (dc.W != W || dc.gs != gs || dc.adj != adj || dc.tl != tl || dc.nw != nw) continue;
                csek::Segment s{};
                s.C = comp_args(dc, c, J.cfg.count_path == CSE_COUNT_MFMA);
                s.R = run_args(ctx, J);
                s.S = J.cj[c].st;
                s.unit_begin = unit;
                unit += J.cfg.n_proc;
                G.lds = std::max(G.lds, lds_bytes(dc));
                B.segs.push_back(s);
                B.seg_job.push_back(jid);
            }
        }
        G.n_segs = (int)B.segs.size() - G.seg_begin;
        G.n_grid = unit;
        if (!G.n_segs) continue;
        // The kernel's Greedy-Potential body is entered only where a job
        // gives gp a weight.
        for (int si = G.seg_begin; si < G.seg_begin + G.n_segs; ++si)
            G.gp |= ctx->jobs[B.seg_job[si]].cfg.weights[CSE_STRAT_GP] != 0;
        B.groups.push_back(G);
    }
    // Longest expected work first, so that the long units do not form the
    // tail of the launch (unit results do not depend on the order).  Each
    // process's strategy comes from the kernels' own process draw.
    std::map<int, std::vector<int32_t>> strat_of;
    {
        uint32_t nmax = 0;
        for (int jid : B.jobs)
            if (!ctx->jobs[jid].done) nmax = std::max(nmax, ctx->jobs[jid].cfg.n_proc);
        int32_t* d_strat = nullptr;
        if (nmax) HIP_TRY(ctx, hipMalloc((void**)&d_strat, sizeof(int32_t) * nmax));
        hipError_t e = hipSuccess;
        for (int jid : B.jobs) {
            JobRec& J = ctx->jobs[jid];
            if (J.done || e != hipSuccess) continue;
            std::vector<int32_t>& st = strat_of[jid];
            st.resize(J.cfg.n_proc);
            hipLaunchKernelGGL(csek::proc_strategy_kernel, dim3((J.cfg.n_proc + 255) / 256), dim3(256), 0, B.stream,
                               run_args(ctx, J), J.cfg.n_proc, d_strat);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = hipMemcpyAsync(st.data(), d_strat, sizeof(int32_t) * J.cfg.n_proc, hipMemcpyDeviceToHost,
                                   B.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(B.stream);
        }
        if (d_strat) (void)hipFree(d_strat);
        if (e != hipSuccess) return fail(ctx, CSE_EHIP, "process strategies: %s", hipGetErrorString(e));
    }
    B.order.clear();
    for (LaunchGroup& G : B.groups) {
        G.order_begin = B.order.size();
        std::vector<std::pair<double, uint32_t>> key;
        key.reserve(G.n_grid);
        for (int si = G.seg_begin; si < G.seg_begin + G.n_segs; ++si) {
            const csek::Segment& sg = B.segs[si];
            const JobRec* Jp = &ctx->jobs[B.seg_job[si]];
            const DevComp& dc = ctx->schemes[Jp->scheme].comp[sg.C.comp];
            const std::vector<int32_t>& st = strat_of[B.seg_job[si]];
            for (uint32_t p = 0; p < sg.R.n_units; ++p)
                key.emplace_back(-unit_cost(dc, (uint32_t)st[p]), sg.unit_begin + p);
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<double, uint32_t>& a, const std::pair<double, uint32_t>& b) {
                             return a.first < b.first;
                         });
        for (auto& k : key) B.order.push_back(k.second);
    }
    for (int jid : B.jobs) {
        JobRec& J = ctx->jobs[jid];
        if (J.done) continue;
        for (int c = 0; c < J.n_comp; ++c) {
            Pool P;
            P.job = jid;
            P.comp = c;
            P.n = J.cfg.n_proc;
            P.shares = shares(J.cfg);
            uint32_t n_src = (uint32_t)(((unsigned long long)P.n * J.cfg.share_src_pm + 999) / 1000);
            P.n_src = std::max(1u, std::min(n_src, P.n));
            P.scratch = P.shares ? (int32_t*)((char*)J.d_share + csek::share_scratch_bytes(P.n) * c) : nullptr;
            B.pools.push_back(P);
        }
    }
    for (const LaunchGroup& G : B.groups) {
        if (G.lds > ctx->lds_max)
            return fail(ctx, CSE_ENOMEM, "unit state needs %zu B of LDS (max %zu)", G.lds, ctx->lds_max);
        int rc = set_lds_limit(ctx, G);
        if (rc) return rc;
    }
    if (B.rounds) {
        std::vector<csek::PoolDev> pd;
        uint32_t nmax = 1;
        for (size_t i = 0; i < B.pools.size(); ++i) {
            const Pool& P = B.pools[i];
            const JobRec& J = ctx->jobs[P.job];
            csek::PoolDev d{};
            d.S = J.cj[P.comp].st;
            if (P.shares) d.sc = csek::share_scratch(P.scratch, P.n);
            d.seed = J.cfg.seed;
            d.n = P.n;
            d.n_src = P.n_src;
            d.comp = (uint32_t)P.comp;
            d.dst_pm = J.cfg.share_dst_pm;
            d.max_rounds = J.cfg.share_max_rounds;
            d.shares = P.shares ? 1u : 0u;
            d.n_fmax = ctx->schemes[J.scheme].comp[P.comp].n_fmax;
            d.first_of_job = P.comp == 0 ? 1u : 0u;
            d.iteration = J.cfg.iteration;
            pd.push_back(d);
            nmax = std::max(nmax, P.n);
        }
        B.pool_grid_x = (nmax + 255) / 256;
        if (pd.size() > B.dpools_cap) {
            if (B.d_pools) HIP_TRY(ctx, hipFree(B.d_pools));
            B.d_pools = nullptr;
            B.dpools_cap = std::max(pd.size(), 2 * B.dpools_cap);
            HIP_TRY(ctx, hipMalloc((void**)&B.d_pools, sizeof(csek::PoolDev) * B.dpools_cap));
        }
        B.hpools = pd;
        if (!pd.empty())
            HIP_TRY(ctx, hipMemcpyAsync(B.d_pools, B.hpools.data(), sizeof(csek::PoolDev) * pd.size(),
                                        hipMemcpyHostToDevice, B.stream));
        if (B.gexec) HIP_TRY(ctx, hipGraphExecDestroy(B.gexec));
        B.gexec = nullptr;  // the captured round no longer matches
    }
    if (B.segs.size() > B.segs_cap) {
        if (B.d_segs) HIP_TRY(ctx, hipFree(B.d_segs));
        B.d_segs = nullptr;
        B.segs_cap = std::max<size_t>(B.segs.size(), 2 * B.segs_cap);
        HIP_TRY(ctx, hipMalloc((void**)&B.d_segs, sizeof(csek::Segment) * B.segs_cap));
    }
    if (B.rounds && B.pools.size() > B.counts_cap) {
        if (B.d_counts) HIP_TRY(ctx, hipFree(B.d_counts));
        if (B.h_counts) HIP_TRY(ctx, hipHostFree(B.h_counts));
        B.d_counts = nullptr;
        B.h_counts = nullptr;
        B.counts_cap = std::max<size_t>(B.pools.size(), 2 * B.counts_cap);
        HIP_TRY(ctx, hipMalloc((void**)&B.d_counts, sizeof(int32_t) * B.counts_cap));
        HIP_TRY(ctx, hipHostMalloc((void**)&B.h_counts, sizeof(int32_t) * B.counts_cap, hipHostMallocDefault));
    }
    if (B.order.size() > B.order_cap) {
        if (B.d_order) HIP_TRY(ctx, hipFree(B.d_order));
        B.d_order = nullptr;
        B.order_cap = std::max<size_t>(B.order.size(), 2 * B.order_cap);
        HIP_TRY(ctx, hipMalloc((void**)&B.d_order, sizeof(uint32_t) * B.order_cap));
    }
    if (!B.segs.empty())
        HIP_TRY(ctx, hipMemcpyAsync(B.d_segs, B.segs.data(), sizeof(csek::Segment) * B.segs.size(),
                                    hipMemcpyHostToDevice, B.stream));
    if (!B.order.empty())
        HIP_TRY(ctx, hipMemcpyAsync(B.d_order, B.order.data(), sizeof(uint32_t) * B.order.size(),
                                    hipMemcpyHostToDevice, B.stream));
    B.built = true;
    return CSE_OK;
}

// Move a built single-job batch to outer iteration `it`: only the run
// arguments' and pools' iteration fields change, in place in device memory,
// so the dispatch order and a captured round stay valid (the order only
// affects timing; the draws are keyed by the iteration).
int set_iteration(cse_ctx* ctx, BatchRec& B, uint32_t it) {
    for (csek::Segment& sg : B.segs) sg.R.iteration = it;
    for (csek::PoolDev& pd : B.hpools) pd.iteration = it;
    if (!B.segs.empty())
        HIP_TRY(ctx, hipMemcpyAsync(B.d_segs, B.segs.data(), sizeof(csek::Segment) * B.segs.size(),
                                    hipMemcpyHostToDevice, B.stream));
    if (B.rounds && !B.hpools.empty())
        HIP_TRY(ctx, hipMemcpyAsync(B.d_pools, B.hpools.data(), sizeof(csek::PoolDev) * B.hpools.size(),
                                    hipMemcpyHostToDevice, B.stream));
    return CSE_OK;
}

// One group's step-kernel launch: a workgroup of 64 nw lanes per grid unit.
int launch_group(cse_ctx* ctx, const LaunchGroup& G, const csek::Segment* d_segs, const uint32_t* d_order,
                 int* d_err, hipStream_t s) {
    if (G.lds > ctx->lds_max)
        return fail(ctx, CSE_ENOMEM, "unit state needs %zu B of LDS (max %zu)", G.lds, ctx->lds_max);
    const void* k = step_kernel_ptr(G);
    if (!k) return fail(ctx, CSE_EINVAL, "no step kernel for row words %d, layout %d", G.W, group_layout(G));
    const csek::Segment* segs = d_segs + G.seg_begin;
    int n_segs = G.n_segs;
    const uint32_t* order = d_order ? d_order + G.order_begin : nullptr;
    uint32_t n_grid = G.n_grid;
    int any_gp = G.gp ? 1 : 0;
    void* args[] = {(void*)&segs, (void*)&n_segs, (void*)&order, (void*)&n_grid, (void*)&d_err, (void*)&any_gp};
    HIP_TRY(ctx, hipLaunchKernel(k, dim3(G.n_grid), dim3(csek::kWave * G.nw), args, G.lds, s));
    return CSE_OK;
}

// Device time of the timed launches queued since the last call, added to
// their classes (call once the stream holding them has been synchronised).
int collect_times(cse_ctx* ctx, BatchRec& B) {
    for (int g : B.t_pending) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, B.tev[2 * g], B.tev[2 * g + 1]));
        const LaunchGroup& G = B.groups[g];
        auto& slot = B.t_class[std::make_pair(G.W, group_layout(G))];
        slot.first += 1;
        slot.second += (uint64_t)((double)ms * 1e6 + 0.5);
    }
    B.t_pending.clear();
    return CSE_OK;
}

// Every group's launch.  Groups hold disjoint units, so they run side by
// side: the first on s, the others on the batch's side streams, forked from
// s before and joined back into s after (a round's tail of long units in one
// class then overlaps the other classes).
int launch_groups(cse_ctx* ctx, BatchRec& B, hipStream_t s, bool timed = false) {
    if (timed && !B.t_pending.empty()) {
        // Launches of an earlier run not read yet (a relaunch queued behind
        // it on the same stream): read them before their events are reused.
        for (int g : B.t_pending) HIP_TRY(ctx, hipEventSynchronize(B.tev[2 * g + 1]));
        int rc = collect_times(ctx, B);
        if (rc) return rc;
    }
    if (timed && B.tev.size() < 2 * B.groups.size()) {
        size_t have = B.tev.size();
        B.tev.resize(2 * B.groups.size(), nullptr);
        for (size_t i = have; i < B.tev.size(); ++i) HIP_TRY(ctx, hipEventCreate(&B.tev[i]));
    }
    const size_t n_side = B.groups.empty() ? 0 : B.groups.size() - 1;
    while (B.side.size() < n_side) {
        hipStream_t x = nullptr;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        B.side.push_back(x);
        hipEvent_t ev = nullptr;
        HIP_TRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        B.ev_join.push_back(ev);
    }
    if (n_side) {
        if (!B.ev_fork) HIP_TRY(ctx, hipEventCreateWithFlags(&B.ev_fork, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventRecord(B.ev_fork, s));
        for (size_t i = 0; i < n_side; ++i) HIP_TRY(ctx, hipStreamWaitEvent(B.side[i], B.ev_fork, 0));
    }
    for (size_t gi = 0; gi < B.groups.size(); ++gi) {
        const LaunchGroup& G = B.groups[gi];
        const hipStream_t gs = gi == 0 ? s : B.side[gi - 1];
        if (timed) HIP_TRY(ctx, hipEventRecord(B.tev[2 * gi], gs));
        int rc = launch_group(ctx, G, B.d_segs, B.d_order, B.d_err, gs);
        if (rc) return rc;
        if (timed) {
            HIP_TRY(ctx, hipEventRecord(B.tev[2 * gi + 1], gs));
            B.t_pending.push_back((int)gi);
        }
    }
    for (size_t i = 0; i < n_side; ++i) {
        HIP_TRY(ctx, hipEventRecord(B.ev_join[i], B.side[i]));
        HIP_TRY(ctx, hipStreamWaitEvent(s, B.ev_join[i], 0));
    }
    return CSE_OK;
}

int check_err(cse_ctx* ctx, BatchRec& B) {
    int herr = 0;
    HIP_TRY(ctx, hipMemcpy(&herr, B.d_err, sizeof herr, hipMemcpyDeviceToHost));
    if (herr) return fail(ctx, CSE_EHIP, "device consistency check failed (flags 0x%x)", herr);
    return CSE_OK;
}

int wait_batch(cse_ctx* ctx, BatchRec& B) {
    if (!B.finished) {
        HIP_TRY(ctx, hipEventSynchronize(B.ev_done));
        B.finished = true;
        int rc = collect_times(ctx, B);
        if (rc) return rc;
        return check_err(ctx, B);
    }
    return CSE_OK;
}

BatchRec* batch_of(cse_ctx* ctx, int job_id, JobRec** job = nullptr) {
    auto it = ctx->jobs.find(job_id);
    if (it == ctx->jobs.end()) return nullptr;
    if (job) *job = &it->second;
    auto bt = ctx->batches.find(it->second.batch);
    return bt == ctx->batches.end() ? nullptr : &bt->second;
}

// Reset the unit arrays of a job and stamp its start on the stream.
int init_job(cse_ctx* ctx, JobRec& J, hipStream_t s) {
    for (int c = 0; c < J.n_comp; ++c)
        hipLaunchKernelGGL(csek::init_units_kernel, dim3((J.cfg.n_proc + 255) / 256), dim3(256), 0, s,
                           J.cj[c].st, J.cfg.n_proc, c == 0 ? 1 : 0);
    HIP_TRY(ctx, hipGetLastError());
    J.round = 0;
    J.done = false;
    return CSE_OK;
}

// One round for every unfinished job of the batch (Sec. 3.5.2): one launch
// per group advances each active unit by at most its job's budget; then every
// pool counts its active units and, if its job shares and is below
// share_max_rounds, ranks its units and copies prefixes into targets; each
// job's round counter advances.  The round is captured once as a graph (its
// arguments never change: budgets, pools and round counters live in device
// memory) and replayed on the batch's internal stream, after the work the
// caller queued on the batch's stream.  The host waits for the counts; a job
// with no active unit left is done.
// One round's work on stream s: every group's launch, then the pool kernels
// and the copy of the active counts to pinned host memory.
int enqueue_round(cse_ctx* ctx, BatchRec& B, hipStream_t s, bool timed) {
    const int n_pools = (int)B.pools.size();
    int rc = launch_groups(ctx, B, s, timed);
    if (rc) return rc;
    const dim3 pg(B.pool_grid_x, (unsigned)n_pools), blk(256);
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3((n_pools + 255) / 256), blk, 0, s, B.d_counts, n_pools, 0);
    hipLaunchKernelGGL(csek::pools_count_kernel, pg, blk, 0, s, B.d_pools, B.d_counts);
    hipLaunchKernelGGL(csek::pools_rank_kernel, pg, blk, 0, s, B.d_pools);
    hipLaunchKernelGGL(csek::pools_target_kernel, pg, blk, 0, s, B.d_pools);
    hipLaunchKernelGGL(csek::pools_round_kernel, dim3(1), blk, 0, s, B.d_pools, n_pools);
    hipError_t e = hipMemcpyAsync(B.h_counts, B.d_counts, sizeof(int32_t) * n_pools, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail(ctx, CSE_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
    return CSE_OK;
}

int capture_round(cse_ctx* ctx, BatchRec& B) {
    HIP_TRY(ctx, hipStreamBeginCapture(B.gstream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_round(ctx, B, B.gstream, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B.gstream, &g);
    if (rc == CSE_OK && e != hipSuccess) rc = fail(ctx, CSE_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (rc == CSE_OK) {
        e = hipGraphInstantiate(&B.gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(ctx, CSE_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    if (g) (void)hipGraphDestroy(g);
    return rc;
}

int round_once(cse_ctx* ctx, BatchRec& B) {
    if (!B.gstream) HIP_TRY(ctx, hipStreamCreateWithFlags(&B.gstream, hipStreamNonBlocking));
    if (!B.ev_order) HIP_TRY(ctx, hipEventCreateWithFlags(&B.ev_order, hipEventDisableTiming));
    // Timed rounds are launched directly, each step-kernel launch between
    // two events; otherwise the round is a captured graph.
    if (!ctx->timing && !B.gexec) {
        int rc = capture_round(ctx, B);
        if (rc) return rc;
    }
    HIP_TRY(ctx, hipEventRecord(B.ev_order, B.stream));
    HIP_TRY(ctx, hipStreamWaitEvent(B.gstream, B.ev_order, 0));
    if (ctx->timing) {
        int rc = enqueue_round(ctx, B, B.gstream, true);
        if (rc) return rc;
    } else {
        HIP_TRY(ctx, hipGraphLaunch(B.gexec, B.gstream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(B.gstream));
    if (ctx->timing) {
        int rc = collect_times(ctx, B);
        if (rc) return rc;
    }
    const int n_pools = (int)B.pools.size();
    std::map<int, long long> active;
    for (int p = 0; p < n_pools; ++p) active[B.pools[p].job] += B.h_counts[p];
    for (auto& kv : active) {
        JobRec& J = ctx->jobs[kv.first];
        J.round++;
        if (kv.second == 0) J.done = true;
    }
    return CSE_OK;
}

// Enqueue a batch's run on its stream.  Without sharing one launch per group
// runs every unit to completion asynchronously; with sharing the host runs
// rounds until no job has an active unit.  fresh = false continues the units
// as they are (the driver's later iterations): only the round counters
// restart.
int run_batch(cse_ctx* ctx, BatchRec& B, bool fresh = true) {
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, B.stream, B.d_err, 1, 0);
    for (int jid : B.jobs) {
        JobRec& J = ctx->jobs[jid];
        J.budget = shares(J.cfg) ? (int)J.cfg.share_every : -1;
        if (fresh) {
            int rc = init_job(ctx, J, B.stream);
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, B.stream, J.cj[0].st.round, 1, 0);
            HIP_TRY(ctx, hipGetLastError());
            J.round = 0;
            J.done = false;
        }
    }
    int rc = B.built ? CSE_OK : build_segments(ctx, B);
    if (rc) return rc;
    if (!B.rounds) return launch_groups(ctx, B, B.stream, ctx->timing);
    for (;;) {
        rc = round_once(ctx, B);
        if (rc) return rc;
        bool any = false;
        for (int jid : B.jobs) any |= !ctx->jobs[jid].done;
        if (!any) return CSE_OK;
    }
}

void drop_batch(cse_ctx* ctx, int bid) {
    auto it = ctx->batches.find(bid);
    if (it == ctx->batches.end()) return;
    BatchRec& B = it->second;
    if (!B.finished && B.ev_done) (void)hipEventSynchronize(B.ev_done);
    std::vector<int> owned;
    for (auto& kv : ctx->jobs)
        if (kv.second.batch == bid) owned.push_back(kv.first);
    for (int jid : owned) {
        free_job_device(ctx, ctx->jobs[jid]);
        ctx->jobs.erase(jid);
    }
    free_batch_device(B);
    ctx->batches.erase(it);
}

int new_batch(cse_ctx* ctx, hipStream_t stream, int* bid) {
    const int id = ctx->next_batch++;
    BatchRec& B = ctx->batches[id];
    B.stream = stream;
    HIP_TRY(ctx, hipMalloc((void**)&B.d_err, 64));
    HIP_TRY(ctx, hipEventCreateWithFlags(&B.ev_done, hipEventDisableTiming));
    *bid = id;
    return CSE_OK;
}

// A job's results may be read once its batch has finished and, for server
// jobs, once the job itself is done.
int readable(cse_ctx* ctx, int job_id, JobRec** J, int comp) {
    BatchRec* B = batch_of(ctx, job_id, J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (comp < -1 || comp >= (*J)->n_comp) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    if ((*J)->server && (*J)->state == CSE_JOB_FAILED)
        return fail(ctx, CSE_ENOMEM, "job %d failed at admission; it has no results", job_id);
    if ((*J)->server && (*J)->state != CSE_JOB_DONE) return fail(ctx, CSE_EBUSY, "job %d is not done", job_id);
    if (!(*J)->allocated) return fail(ctx, CSE_EBUSY, "job %d has no results", job_id);
    return wait_batch(ctx, *B);
}

}  // namespace

extern "C" {

int32_t cse_version(void) { return 1; }

int32_t cse_ctx_create(int32_t device, cse_ctx** out) {
    if (!out) return CSE_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return CSE_EHIP;
    if (hipSetDevice(device) != hipSuccess) return CSE_EHIP;
    cse_ctx* ctx = new (std::nothrow) cse_ctx();
    if (!ctx) return CSE_ENOMEM;
    ctx->device = device;
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            // On failure the address stays unset and cse_reduce_static
            // reports it; every other entry point works without the array.
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
                g_scratch_ptr[device] = ptr;
            else
                (void)hipGetLastError();
        }
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess)
        ctx->lds_max = std::max<size_t>(prop.sharedMemPerBlock, 65536);
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        ctx->tick_hz = (uint64_t)khz * 1000ull;
    // Cancellation flags: coherent pinned host memory, read by the kernels.
    if (hipHostMalloc((void**)&ctx->h_cancel, sizeof(int32_t) * kCancelSlots,
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&ctx->d_cancel, ctx->h_cancel, 0) != hipSuccess) {
        if (ctx->h_cancel) (void)hipHostFree(ctx->h_cancel);
        delete ctx;
        return CSE_EHIP;
    }
    std::memset(ctx->h_cancel, 0, sizeof(int32_t) * kCancelSlots);
    ctx->free_slots.reserve(kCancelSlots);
    for (int i = kCancelSlots - 1; i >= 0; --i) ctx->free_slots.push_back(i);
    *out = ctx;
    return CSE_OK;
}

void cse_ctx_destroy(cse_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    std::vector<int> bids;
    for (auto& kv : ctx->batches) bids.push_back(kv.first);
    for (int b : bids) drop_batch(ctx, b);
    for (auto& kv : ctx->schemes)
        for (int c = 0; c < kv.second.n_comp; ++c) free_component(kv.second.comp[c]);
    if (ctx->h_cancel) (void)hipHostFree(ctx->h_cancel);
    delete ctx;
}

const char* cse_last_error(const cse_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t cse_system_load(cse_ctx* ctx, const int8_t* A, int32_t rows, int32_t cols, int32_t* scheme_id) {
    if (!ctx || !scheme_id) return CSE_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    SchemeRec s;
    s.n_comp = 1;
    int rc = load_component(ctx, A, rows, cols, &s.comp[0]);
    if (rc) return rc;
    const int id = ctx->next_scheme++;
    ctx->schemes[id] = s;
    *scheme_id = id;
    return CSE_OK;
}

int32_t cse_scheme_load(cse_ctx* ctx, const int8_t* U, int32_t u_rows, int32_t u_cols,
                        const int8_t* V, int32_t v_rows, int32_t v_cols,
                        const int8_t* Wt, int32_t w_rows, int32_t w_cols, int32_t* scheme_id) {
    if (!ctx || !scheme_id) return CSE_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    SchemeRec s;
    s.n_comp = 3;
    const int8_t* mats[3] = {U, V, Wt};
    const int rows[3] = {u_rows, v_rows, w_rows}, cols[3] = {u_cols, v_cols, w_cols};
    for (int c = 0; c < 3; ++c) {
        int rc = load_component(ctx, mats[c], rows[c], cols[c], &s.comp[c]);
        if (rc) {
            for (int k = 0; k < c; ++k) free_component(s.comp[k]);
            return rc;
        }
    }
    const int id = ctx->next_scheme++;
    ctx->schemes[id] = s;
    *scheme_id = id;
    return CSE_OK;
}

int32_t cse_scheme_load_device(cse_ctx* ctx, const int8_t* U, int32_t u_rows, int32_t u_cols, const int8_t* V,
                               int32_t v_rows, int32_t v_cols, const int8_t* Wt, int32_t w_rows, int32_t w_cols,
                               void* stream, int32_t* scheme_id) {
    if (!ctx || !scheme_id) return CSE_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int8_t* mats[3] = {U, V, Wt};
    const int rows[3] = {u_rows, v_rows, w_rows}, cols[3] = {u_cols, v_cols, w_cols};
    const int n = (V || Wt) ? 3 : 1;
    if (n == 3 && (!V || !Wt)) return fail(ctx, CSE_EINVAL, "V and W^T are both given or both null");
    unsigned long long* d_st = nullptr;
    HIP_TRY(ctx, hipMalloc((void**)&d_st, 64));
    SchemeRec s;
    s.n_comp = n;
    int rc = CSE_OK;
    for (int c = 0; c < n && rc == CSE_OK; ++c) {
        rc = load_component_device(ctx, mats[c], rows[c], cols[c], (hipStream_t)stream, d_st, &s.comp[c]);
        if (rc)
            for (int k = 0; k < c; ++k) free_component(s.comp[k]);
    }
    (void)hipFree(d_st);
    if (rc) return rc;
    const int id = ctx->next_scheme++;
    ctx->schemes[id] = s;
    *scheme_id = id;
    return CSE_OK;
}

int32_t cse_scheme_info(cse_ctx* ctx, int32_t scheme_id, int32_t* n_comp, int32_t info[12]) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->schemes.find(scheme_id);
    if (it == ctx->schemes.end()) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_id);
    if (n_comp) *n_comp = it->second.n_comp;
    if (info)
        for (int c = 0; c < it->second.n_comp; ++c) {
            const DevComp& d = it->second.comp[c];
            info[4 * c + 0] = d.n_e;
            info[4 * c + 1] = d.n_x;
            info[4 * c + 2] = d.n_fmax;
            info[4 * c + 3] = d.naive0;
        }
    return CSE_OK;
}

int32_t cse_scheme_free(cse_ctx* ctx, int32_t scheme_id) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->schemes.find(scheme_id);
    if (it == ctx->schemes.end()) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_id);
    for (auto& kv : ctx->jobs)
        if (kv.second.scheme == scheme_id)
            return fail(ctx, CSE_EBUSY, "scheme %d still has job %d; release it first", scheme_id, kv.first);
    for (int c = 0; c < it->second.n_comp; ++c) free_component(it->second.comp[c]);
    ctx->schemes.erase(it);
    return CSE_OK;
}

int32_t cse_launch(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, void* stream, int32_t* job_id) {
    return cse_launch_batch(ctx, &scheme_id, cfg, 1, stream, job_id);
}

}  // extern "C"

namespace {
bool scheme_busy(cse_ctx* ctx, int scheme_id) {
    for (auto& kv : ctx->jobs)
        if (kv.second.scheme == scheme_id) return true;
    return false;
}

// Time one layout of a component: a job on a temporary one-component scheme
// that shares the component's device buffers, launched once, then two timed
// relaunches on the stream.
// relaunches on the stream.  A layout whose first launch already takes more
// than three times `bound` ms is not timed further (*ms = that time).
int probe_layout(cse_ctx* ctx, const DevComp& probe, const cse_run_cfg& pc, hipStream_t s, float bound,
                 float* ms) {
    const int sid = ctx->next_scheme++;
    SchemeRec& tmp = ctx->schemes[sid];
    tmp.n_comp = 1;
    tmp.comp[0] = probe;
    int32_t job = -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        ctx->schemes.erase(sid);
        return fail(ctx, CSE_EHIP, "hipEventCreate failed");
    }
    int rc = hipEventRecord(e0, s) == hipSuccess ? CSE_OK : fail(ctx, CSE_EHIP, "hipEventRecord failed");
    if (rc == CSE_OK) rc = cse_launch(ctx, sid, &pc, s, &job);
    if (rc == CSE_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(ms, e0, e1) != hipSuccess))
        rc = fail(ctx, CSE_EHIP, "probe timing failed");
    if (rc == CSE_OK) rc = cse_wait(ctx, job);
    if (rc == CSE_OK && !(bound > 0.f && *ms > 3.f * bound)) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = fail(ctx, CSE_EHIP, "hipEventRecord failed");
        for (int r = 0; r < 2 && rc == CSE_OK; ++r) rc = cse_relaunch(ctx, job, nullptr, s);
        if (rc == CSE_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(ms, e0, e1) != hipSuccess))
            rc = fail(ctx, CSE_EHIP, "probe timing failed");
        if (rc == CSE_OK) rc = cse_wait(ctx, job);
        *ms *= 0.5f;
    }
    std::string keep = ctx->err;
    if (job >= 0) (void)cse_job_release(ctx, job);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx->schemes.erase(sid);  // the buffers belong to the real component
    ctx->err = keep;
    return rc;
}
}  // namespace

extern "C" {

int32_t cse_scheme_layout(cse_ctx* ctx, int32_t scheme_id, int32_t comp, int32_t layout, int32_t* current) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->schemes.find(scheme_id);
    if (it == ctx->schemes.end()) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_id);
    if (comp < 0 || comp >= it->second.n_comp) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    DevComp& dc = it->second.comp[comp];
    if (current) *current = layout_code(dc);
    if (layout < 0) return CSE_OK;
    if (!layout_valid(layout)) return fail(ctx, CSE_EINVAL, "unknown layout %d", layout);
    if (scheme_busy(ctx, scheme_id)) return fail(ctx, CSE_EBUSY, "scheme %d has jobs; release them first", scheme_id);
    DevComp probe = dc;
    set_layout(probe, layout);
    if (probe.nw > 1 && dc.n_x + dc.n_fmax > csek::kCompactMaxVars)
        return fail(ctx, CSE_EINVAL, "layout %d: several waves per unit need at most %d variables (%d)", layout,
                    csek::kCompactMaxVars, dc.n_x + dc.n_fmax);
    if (lds_bytes(probe) > ctx->lds_max)
        return fail(ctx, CSE_ENOMEM, "layout %d needs %zu B of LDS per unit (max %zu)", layout, lds_bytes(probe),
                    ctx->lds_max);
    set_layout(dc, layout);
    return CSE_OK;
}

int32_t cse_autotune(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, void* stream, int32_t layouts[3]) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->schemes.find(scheme_id);
    if (it == ctx->schemes.end()) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_id);
    int rc = validate_cfg(ctx, cfg);
    if (rc) return rc;
    if (scheme_busy(ctx, scheme_id)) return fail(ctx, CSE_EBUSY, "scheme %d has jobs; release them first", scheme_id);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // A bounded probe: at most 1024 processes, 32 steps each, no sharing.
    cse_run_cfg pc = *cfg;
    pc.n_proc = std::min<uint32_t>(cfg->n_proc, 1024);
    pc.step_cap = cfg->step_cap ? std::min<uint32_t>(cfg->step_cap, 32) : 32;
    pc.share_every = pc.share_src_pm = pc.share_dst_pm = pc.share_max_rounds = 0;
    pc.count_path = CSE_COUNT_POPCOUNT;
    for (int c = 0; c < it->second.n_comp; ++c) {
        DevComp& dc = ctx->schemes[scheme_id].comp[c];
        int best = layout_code(dc);
        float best_ms = -1.f;
        // The mask form of gi is skipped where the input's masks already
        // exceed their capacity (its steps would take the O(m^2) form).
        const bool masks_fit = (long long)dc.n_x * ((dc.m0 + 31) / 32) <= 2ll * dc.m_words;
        // Range tables in LDS are not probed: a one-component probe cannot
        // show what their LDS footprint costs when the components of a job
        // share the CUs (on 6x6x6 it would pick them and lose 3%).
        // Waves per unit (threads per process) are tuned with the range form:
        // one, two or four.
        for (int code = 0; code < 12; ++code) {
            const int base = code & 3, wb = code >> 2;
            if (wb && !(base & CSE_LAYOUT_RANGE)) continue;
            const int lay = base | (wb << CSE_LAYOUT_WAVES_SHIFT);
            DevComp probe = dc;
            set_layout(probe, lay);
            if (lds_bytes(probe) > ctx->lds_max) continue;
            if (probe.nw > 1 && dc.n_x + dc.n_fmax > csek::kCompactMaxVars) continue;
            if (!probe.adj && !masks_fit) continue;
            float ms = 0.f;
            rc = probe_layout(ctx, probe, pc, (hipStream_t)stream, best_ms, &ms);
            if (rc) return rc;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = lay;
            }
        }
        set_layout(dc, best);
        if (layouts) layouts[c] = best;
    }
    return CSE_OK;
}

}  // extern "C"

namespace {
// A batch of new jobs with their device state, not yet started; on error
// nothing is left behind.
int create_batch(cse_ctx* ctx, const int32_t* scheme_ids, const cse_run_cfg* cfgs, int32_t n, void* stream,
                 int* bid_out) {
    for (int i = 0; i < n; ++i) {
        if (!ctx->schemes.count(scheme_ids[i])) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_ids[i]);
        int rc = validate_cfg(ctx, &cfgs[i]);
        if (rc) return rc;
    }
    int bid = -1;
    int rc = new_batch(ctx, (hipStream_t)stream, &bid);
    BatchRec& B = ctx->batches[bid];
    for (int i = 0; i < n && rc == CSE_OK; ++i) {
        const int jid = ctx->next_job++;
        JobRec& J = ctx->jobs[jid];
        J.scheme = scheme_ids[i];
        J.cfg = cfgs[i];
        J.batch = bid;
        B.jobs.push_back(jid);
        B.rounds |= shares(J.cfg);
        rc = alloc_job(ctx, J);
    }
    if (rc != CSE_OK) {
        std::string keep = ctx->err;
        drop_batch(ctx, bid);
        ctx->err = keep;
        return rc;
    }
    *bid_out = bid;
    return CSE_OK;
}

// Run a created batch on its stream (asynchronous unless it has rounds);
// on error the batch is dropped.
int start_batch(cse_ctx* ctx, int bid) {
    BatchRec& B = ctx->batches[bid];
    B.finished = false;
    int rc = run_batch(ctx, B);
    if (rc == CSE_OK) {
        hipError_t e = hipEventRecord(B.ev_done, B.stream);
        if (e != hipSuccess) rc = fail(ctx, CSE_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
    }
    if (rc != CSE_OK) {
        std::string keep = ctx->err;
        (void)hipStreamSynchronize(B.stream);
        B.finished = true;
        drop_batch(ctx, bid);
        ctx->err = keep;
    }
    return rc;
}
}  // namespace

extern "C" {

int32_t cse_launch_batch(cse_ctx* ctx, const int32_t* scheme_ids, const cse_run_cfg* cfgs, int32_t n,
                         void* stream, int32_t* job_ids) {
    if (!ctx || !scheme_ids || !cfgs || !job_ids || n < 1) return CSE_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int bid = -1;
    int rc = create_batch(ctx, scheme_ids, cfgs, n, stream, &bid);
    if (rc) return rc;
    std::vector<int> ids = ctx->batches[bid].jobs;
    rc = start_batch(ctx, bid);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) job_ids[i] = ids[i];
    return CSE_OK;
}

int32_t cse_relaunch(cse_ctx* ctx, int32_t job_id, const cse_run_cfg* cfg, void* stream) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (B->is_server) return fail(ctx, CSE_EINVAL, "server jobs cannot be relaunched");
    if (J->driver) return fail(ctx, CSE_EINVAL, "driver jobs cannot be relaunched");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // On the batch's own stream the earlier run is ordered before the new
    // one; elsewhere, and whenever the host drives rounds, wait for it.
    int rc = CSE_OK;
    if ((hipStream_t)stream != B->stream || B->rounds) rc = wait_batch(ctx, *B);
    if (rc) return rc;
    if (cfg) {
        rc = validate_cfg(ctx, cfg);
        if (rc) return rc;
        if (B->jobs.size() != 1) return fail(ctx, CSE_EINVAL, "a batched job is relaunched with its batch's configurations");
        if (cfg->n_proc != J->cfg.n_proc) return fail(ctx, CSE_EINVAL, "n_proc cannot change on relaunch");
        if (shares(*cfg) != shares(J->cfg)) return fail(ctx, CSE_EINVAL, "relaunch cannot switch sharing on or off");
        rc = wait_batch(ctx, *B);
        if (rc) return rc;
        J->cfg = *cfg;
        B->built = false;
    }
    for (int jid : B->jobs) {
        JobRec& Jb = ctx->jobs[jid];
        if (Jb.cancel_slot >= 0) __atomic_store_n(&ctx->h_cancel[Jb.cancel_slot], 0, __ATOMIC_SEQ_CST);
        Jb.cancelled = false;
    }
    B->stream = (hipStream_t)stream;
    B->finished = false;
    rc = run_batch(ctx, *B);
    if (rc) return rc;
    HIP_TRY(ctx, hipEventRecord(B->ev_done, B->stream));
    return CSE_OK;
}

int32_t cse_resume(cse_ctx* ctx, int32_t job_id, void* stream) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (B->is_server) return fail(ctx, CSE_EINVAL, "server jobs cannot be resumed");
    if (J->driver) return fail(ctx, CSE_EINVAL, "driver jobs cannot be resumed");
    if (B->rounds) return fail(ctx, CSE_EINVAL, "jobs with sharing rounds cannot be resumed");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = wait_batch(ctx, *B);
    if (rc) return rc;
    for (int jid : B->jobs) {
        JobRec& Jb = ctx->jobs[jid];
        if (Jb.cancel_slot >= 0) __atomic_store_n(&ctx->h_cancel[Jb.cancel_slot], 0, __ATOMIC_SEQ_CST);
        Jb.cancelled = false;
    }
    B->stream = (hipStream_t)stream;
    B->finished = false;
    // Unit state is kept: each active unit replays its prefix (or takes its
    // HBM slot record) and continues with the draws of its epoch and step.
    rc = run_batch(ctx, *B, false);
    if (rc) return rc;
    HIP_TRY(ctx, hipEventRecord(B->ev_done, B->stream));
    return CSE_OK;
}

int32_t cse_poll(cse_ctx* ctx, int32_t job_id, int32_t* done, int32_t best_cost[3]) {
    if (!ctx || !done) return CSE_EINVAL;
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (best_cost) best_cost[0] = best_cost[1] = best_cost[2] = -1;
    *done = 0;
    if (J->server) {
        if (J->state != CSE_JOB_DONE && J->state != CSE_JOB_FAILED) return CSE_OK;
    } else if (!B->finished) {
        hipError_t e = hipEventQuery(B->ev_done);
        if (e == hipErrorNotReady) return CSE_OK;
        if (e != hipSuccess) return fail(ctx, CSE_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
        B->finished = true;
        int rc = check_err(ctx, *B);
        if (rc) return rc;
    }
    *done = 1;
    if (!best_cost || !J->allocated) return CSE_OK;
    // The best of each pool (Sec. 3.5): a min over the units on the device.
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, B->stream, J->d_best, 4, 0x7FFFFFFF);
    for (int c = 0; c < J->n_comp; ++c)
        hipLaunchKernelGGL(csek::best_cost_kernel, dim3((J->cfg.n_proc + 255) / 256), dim3(256), 0, B->stream,
                           J->cj[c].st.cost, J->cfg.n_proc, J->d_best + c);
    HIP_TRY(ctx, hipGetLastError());
    int32_t h[4];
    HIP_TRY(ctx, hipMemcpyAsync(h, J->d_best, sizeof h, hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(ctx, hipStreamSynchronize(B->stream));
    for (int c = 0; c < J->n_comp; ++c) best_cost[c] = h[c];
    return CSE_OK;
}

int32_t cse_wait(cse_ctx* ctx, int32_t job_id) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (J->server && J->state == CSE_JOB_FAILED)
        return fail(ctx, CSE_ENOMEM, "server job %d failed at admission", job_id);
    if (J->server && J->state != CSE_JOB_DONE) return fail(ctx, CSE_EBUSY, "server job %d is not done", job_id);
    int rc = J->server ? CSE_OK : wait_batch(ctx, *B);
    if (rc) return rc;
    if (J->cancelled) return fail(ctx, CSE_ECANCELED, "job %d was cancelled", job_id);
    return CSE_OK;
}

int32_t cse_cancel(cse_ctx* ctx, int32_t job_id) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (J->server) {
        if (J->state == CSE_JOB_DONE || J->state == CSE_JOB_FAILED) return CSE_OK;
        J->cancelled = true;
        if (J->state == CSE_JOB_QUEUED && B->owner) {
            auto& q = B->owner->queue;
            q.erase(std::remove(q.begin(), q.end(), job_id), q.end());
            J->state = CSE_JOB_DONE;
            J->t_done = now_ns();
        }
        return CSE_OK;  // a running server job stops at the end of the current round
    }
    if (__atomic_load_n(&J->driver_running, __ATOMIC_SEQ_CST)) {
        // The driver stops after the running iteration, whose units stop early.
        if (J->cancel_slot >= 0) __atomic_store_n(&ctx->h_cancel[J->cancel_slot], 1, __ATOMIC_SEQ_CST);
        __atomic_store_n(&J->cancelled, true, __ATOMIC_SEQ_CST);
        return CSE_OK;
    }
    if (B->finished) return CSE_OK;
    hipError_t e = hipEventQuery(B->ev_done);
    if (e == hipSuccess) return CSE_OK;
    if (e != hipErrorNotReady) return fail(ctx, CSE_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
    if (J->cancel_slot < 0) return fail(ctx, CSE_EINVAL, "job %d has no cancellation flag", job_id);
    __atomic_store_n(&ctx->h_cancel[J->cancel_slot], 1, __ATOMIC_SEQ_CST);
    J->cancelled = true;
    return CSE_OK;
}

int32_t cse_get_unit_results(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t n, int32_t* cost,
                             int32_t* steps, int32_t* executed, int32_t* epoch, int32_t* k0, int64_t* ops,
                             int32_t* strat, uint64_t* finish) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    int rc = readable(ctx, job_id, &J, comp);
    if (rc) return rc;
    if (comp < 0) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    if (n != (int32_t)J->cfg.n_proc) return fail(ctx, CSE_ERANGE, "n must equal n_proc (%u)", J->cfg.n_proc);
    const csek::UnitState& S = J->cj[comp].st;
    const size_t b4 = (size_t)n * 4, b8 = (size_t)n * 8;
    if (cost) HIP_TRY(ctx, hipMemcpy(cost, S.cost, b4, hipMemcpyDeviceToHost));
    if (steps) HIP_TRY(ctx, hipMemcpy(steps, S.t, b4, hipMemcpyDeviceToHost));
    if (executed) HIP_TRY(ctx, hipMemcpy(executed, S.executed, b4, hipMemcpyDeviceToHost));
    if (epoch) HIP_TRY(ctx, hipMemcpy(epoch, S.epoch, b4, hipMemcpyDeviceToHost));
    if (k0) HIP_TRY(ctx, hipMemcpy(k0, S.k0, b4, hipMemcpyDeviceToHost));
    if (ops) HIP_TRY(ctx, hipMemcpy(ops, S.ops, b8, hipMemcpyDeviceToHost));
    if (strat) HIP_TRY(ctx, hipMemcpy(strat, S.strat, b4, hipMemcpyDeviceToHost));
    if (finish) HIP_TRY(ctx, hipMemcpy(finish, S.finish, b8, hipMemcpyDeviceToHost));
    return CSE_OK;
}

int32_t cse_get_programs(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t n, int32_t* triples, int32_t cap) {
    if (!ctx || !triples) return CSE_EINVAL;
    JobRec* J = nullptr;
    int rc = readable(ctx, job_id, &J, comp);
    if (rc) return rc;
    if (comp < 0) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    if (n != (int32_t)J->cfg.n_proc) return fail(ctx, CSE_ERANGE, "n must equal n_proc (%u)", J->cfg.n_proc);
    const DevComp& dc = ctx->schemes[J->scheme].comp[comp];
    if (cap < dc.n_fmax) return fail(ctx, CSE_ERANGE, "cap %d < n_fmax %d", cap, dc.n_fmax);
    const int nf = std::max(1, dc.n_fmax);
    std::vector<uint32_t> keys((size_t)n * nf);
    std::vector<int32_t> len(n);
    HIP_TRY(ctx, hipMemcpy(keys.data(), J->cj[comp].st.prog, keys.size() * 4, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(len.data(), J->cj[comp].st.t, (size_t)n * 4, hipMemcpyDeviceToHost));
    for (int u = 0; u < n; ++u) {
        int32_t* dst = triples + (size_t)u * cap * 3;
        std::memset(dst, 0, sizeof(int32_t) * 3 * (size_t)cap);
        for (int i = 0; i < len[u]; ++i) {
            const uint32_t k = keys[(size_t)u * nf + i];
            dst[3 * i + 0] = (int32_t)(k >> 16);
            dst[3 * i + 1] = (int32_t)((k >> 1) & 0x7FFFu);
            dst[3 * i + 2] = (k & 1u) ? -1 : 1;
        }
    }
    return CSE_OK;
}

int32_t cse_get_program(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t proc, int32_t* triples, int32_t cap,
                        int32_t* n_fresh, int32_t* cost, int32_t* needed) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    int rc = readable(ctx, job_id, &J, comp);
    if (rc) return rc;
    if (comp < 0) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    const int n = (int)J->cfg.n_proc;
    if (proc < -1 || proc >= n) return fail(ctx, CSE_EINVAL, "process %d out of range", proc);
    std::vector<int32_t> costs(n), len(n);
    HIP_TRY(ctx, hipMemcpy(costs.data(), J->cj[comp].st.cost, (size_t)n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(len.data(), J->cj[comp].st.t, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (proc < 0) {
        proc = 0;
        for (int u = 1; u < n; ++u)
            if (costs[u] < costs[proc]) proc = u;
    }
    if (n_fresh) *n_fresh = len[proc];
    if (cost) *cost = costs[proc];
    if (needed) *needed = len[proc];
    if (cap < len[proc] || (!triples && len[proc] > 0)) return fail(ctx, CSE_ERANGE, "cap %d < %d", cap, len[proc]);
    const DevComp& dc = ctx->schemes[J->scheme].comp[comp];
    std::vector<uint32_t> keys(std::max(1, len[proc]));
    if (len[proc] > 0)
        HIP_TRY(ctx, hipMemcpy(keys.data(), J->cj[comp].st.prog + (size_t)proc * std::max(1, dc.n_fmax),
                               (size_t)len[proc] * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < len[proc]; ++i) {
        triples[3 * i + 0] = (int32_t)(keys[i] >> 16);
        triples[3 * i + 1] = (int32_t)((keys[i] >> 1) & 0x7FFFu);
        triples[3 * i + 2] = (keys[i] & 1u) ? -1 : 1;
    }
    return CSE_OK;
}

int32_t cse_ctx_set_timing(cse_ctx* ctx, int32_t on) {
    if (!ctx) return CSE_EINVAL;
    ctx->timing = on != 0;
    return CSE_OK;
}

int32_t cse_kernel_times(cse_ctx* ctx, int32_t job_id, cse_kernel_time* out, int32_t cap, int32_t* n,
                         int32_t reset) {
    if (!ctx || !n) return CSE_EINVAL;
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (!J->server) {
        int rc = wait_batch(ctx, *B);
        if (rc) return rc;
    }
    *n = (int32_t)B->t_class.size();
    if (out && cap < *n) return fail(ctx, CSE_ERANGE, "cap %d < %d", cap, *n);
    int i = 0;
    for (const auto& kv : B->t_class) {
        if (out) {
            out[i].row_words = kv.first.first;
            out[i].layout = kv.first.second;
            out[i].launches = kv.second.first;
            out[i].reserved = 0;
            out[i].device_ns = kv.second.second;
        }
        ++i;
    }
    if (reset) B->t_class.clear();
    return CSE_OK;
}

int32_t cse_job_timing(cse_ctx* ctx, int32_t job_id, uint64_t* ticks, uint64_t* tick_hz) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    int rc = readable(ctx, job_id, &J, -1);
    if (rc) return rc;
    uint64_t last = 0;
    const int n = (int)J->cfg.n_proc;
    std::vector<unsigned long long> f(n);
    for (int c = 0; c < J->n_comp; ++c) {
        HIP_TRY(ctx, hipMemcpy(f.data(), J->cj[c].st.finish, (size_t)n * 8, hipMemcpyDeviceToHost));
        for (int u = 0; u < n; ++u) last = std::max<uint64_t>(last, f[u]);
    }
    if (ticks) *ticks = last;
    if (tick_hz) *tick_hz = ctx->tick_hz;
    return CSE_OK;
}

}  // extern "C"

namespace {
// Offset of component c's best program in a driver job's buffer.
size_t best_offset(const SchemeRec& sc, int c) {
    size_t o = 0;
    for (int i = 0; i < c; ++i) o += (size_t)std::max(1, sc.comp[i].n_fmax);
    return o;
}

// After an iteration of a driver job: each component's best unit (lowest
// cost, then process) replaces the best program so far when its cost is
// strictly lower.  Returns the best total.
int driver_update_best(cse_ctx* ctx, JobRec& J, hipStream_t s, int32_t* total) {
    const SchemeRec& sc = ctx->schemes[J.scheme];
    const uint32_t n = J.cfg.n_proc;
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)J.d_key, 2 * J.n_comp, -1);
    for (int c = 0; c < J.n_comp; ++c)
        hipLaunchKernelGGL(csek::driver_argmin_kernel, dim3((n + 255) / 256), dim3(256), 0, s, J.cj[c].st.cost, n,
                           J.d_key + c);
    HIP_TRY(ctx, hipGetLastError());
    unsigned long long key[3];
    HIP_TRY(ctx, hipMemcpyAsync(key, J.d_key, sizeof(unsigned long long) * J.n_comp, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const int it = (int)J.cfg.iteration;
    int32_t sum = 0;
    for (int c = 0; c < J.n_comp; ++c) {
        const int32_t cost = (int32_t)(key[c] >> 32);
        const int32_t proc = (int32_t)(key[c] & 0xFFFFFFFFu);
        if (J.best_cost[c] < 0 || cost < J.best_cost[c]) {
            const int nf = std::max(1, sc.comp[c].n_fmax);
            int32_t len = 0;
            HIP_TRY(ctx, hipMemcpy(&len, J.cj[c].st.t + proc, 4, hipMemcpyDeviceToHost));
            if (len < 0 || len > sc.comp[c].n_fmax) return fail(ctx, CSE_EHIP, "program length %d out of range", len);
            uint32_t* dst = J.d_bestprog + best_offset(sc, c);
            const uint32_t* src = J.cj[c].st.prog + (size_t)proc * nf;
            J.best_keys[c].assign((size_t)len, 0u);
            if (len > 0) {
                HIP_TRY(ctx, hipMemcpy(dst, src, (size_t)len * 4, hipMemcpyDeviceToDevice));
                HIP_TRY(ctx, hipMemcpy(J.best_keys[c].data(), src, (size_t)len * 4, hipMemcpyDeviceToHost));
            }
            J.best_cost[c] = cost;
            J.best_iter[c] = it;
            J.best_proc[c] = proc;
        }
        sum += J.best_cost[c];
    }
    *total = sum;
    return CSE_OK;
}
}  // namespace

extern "C" {

int32_t cse_run_driver(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, const cse_driver_cfg* dcfg,
                       void* stream, int32_t* job_id, int32_t* iterations) {
    if (!ctx || !cfg || !dcfg || !job_id) return CSE_EINVAL;
    if (dcfg->reinit_pm > 1000 || dcfg->max_iterations < 1 || dcfg->max_iterations > 1024 || dcfg->reserved)
        return fail(ctx, CSE_EINVAL, "driver configuration out of range");
    if (cfg->iteration != 0) return fail(ctx, CSE_EINVAL, "the driver starts at iteration 0");
    if (iterations) *iterations = 0;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const uint64_t t_start = now_ns();
    int bid = -1;
    int rc = create_batch(ctx, &scheme_id, cfg, 1, stream, &bid);
    if (rc) return rc;
    const int32_t jid = ctx->batches[bid].jobs[0];
    {
        // Marked as a running driver before its id is published, so a
        // cse_cancel from another thread always takes the driver's path.
        JobRec& J0 = ctx->jobs[jid];
        J0.driver = true;
        __atomic_store_n(&J0.driver_running, true, __ATOMIC_SEQ_CST);
    }
    __atomic_store_n(job_id, jid, __ATOMIC_SEQ_CST);
    rc = start_batch(ctx, bid);  // iteration 0
    if (rc) {
        __atomic_store_n(job_id, -1, __ATOMIC_SEQ_CST);  // the job was dropped
        return rc;
    }
    JobRec& J = ctx->jobs[jid];
    BatchRec& B = ctx->batches[J.batch];
    const SchemeRec& sc = ctx->schemes[J.scheme];
    hipError_t e = hipMalloc((void**)&J.d_bestprog, 4 * best_offset(sc, sc.n_comp));
    if (e == hipSuccess) e = hipMalloc((void**)&J.d_key, sizeof(unsigned long long) * 3);
    if (e != hipSuccess) rc = fail(ctx, CSE_EHIP, "hipMalloc: %s", hipGetErrorString(e));
    int it = 0, unchanged = 0;
    while (rc == CSE_OK) {
        rc = wait_batch(ctx, B);
        if (rc) break;
        int32_t total = 0;
        rc = driver_update_best(ctx, J, B.stream, &total);
        if (rc) break;
        unchanged = (!J.totals.empty() && total == J.totals.back()) ? unchanged + 1 : 0;
        J.totals.push_back(total);
        J.iter_ns.push_back(now_ns() - t_start);
        ++it;
        if (__atomic_load_n(&J.cancelled, __ATOMIC_SEQ_CST)) {
            rc = fail(ctx, CSE_ECANCELED, "job %d was cancelled", jid);
            break;
        }
        if (unchanged >= (int)dcfg->patience || it >= (int)dcfg->max_iterations) break;
        // Restart every unit, then run iteration `it` with its own draws.
        for (int c = 0; c < J.n_comp; ++c)
            hipLaunchKernelGGL(csek::driver_reinit_kernel, dim3((J.cfg.n_proc + 255) / 256), dim3(256), 0, B.stream,
                               J.cj[c].st, J.cfg.n_proc, J.cfg.seed, (uint32_t)c, (uint32_t)it, dcfg->reinit_pm,
                               J.d_bestprog + best_offset(sc, c), (int)J.best_keys[c].size(),
                               std::max(1, sc.comp[c].n_fmax));
        e = hipGetLastError();
        if (e != hipSuccess) {
            rc = fail(ctx, CSE_EHIP, "driver_reinit_kernel: %s", hipGetErrorString(e));
            break;
        }
        J.cfg.iteration = (uint32_t)it;
        rc = B.built ? set_iteration(ctx, B, (uint32_t)it) : CSE_OK;
        if (rc) break;
        B.finished = false;
        rc = run_batch(ctx, B, false);
        if (rc) break;
        e = hipEventRecord(B.ev_done, B.stream);
        if (e != hipSuccess) rc = fail(ctx, CSE_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
    }
    if (!B.finished) (void)hipStreamSynchronize(B.stream);
    B.finished = true;
    __atomic_store_n(&J.driver_running, false, __ATOMIC_SEQ_CST);
    if (iterations) *iterations = it;
    return rc;
}

int32_t cse_driver_best(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t* triples, int32_t cap,
                        int32_t* n_fresh, int32_t* cost, int32_t* iteration, int32_t* proc, int32_t* needed) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = nullptr;
    int rc = readable(ctx, job_id, &J, comp);
    if (rc) return rc;
    if (!J->driver) return fail(ctx, CSE_EINVAL, "job %d did not run the driver", job_id);
    if (comp < 0) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    if (J->best_cost[comp] < 0) return fail(ctx, CSE_ENOENT, "job %d has no completed iteration", job_id);
    const std::vector<uint32_t>& k = J->best_keys[comp];
    const int len = (int)k.size();
    if (n_fresh) *n_fresh = len;
    if (cost) *cost = J->best_cost[comp];
    if (iteration) *iteration = J->best_iter[comp];
    if (proc) *proc = J->best_proc[comp];
    if (needed) *needed = len;
    if (cap < len || (!triples && len > 0)) return fail(ctx, CSE_ERANGE, "cap %d < %d", cap, len);
    for (int i = 0; i < len; ++i) {
        triples[3 * i + 0] = (int32_t)(k[i] >> 16);
        triples[3 * i + 1] = (int32_t)((k[i] >> 1) & 0x7FFFu);
        triples[3 * i + 2] = (k[i] & 1u) ? -1 : 1;
    }
    return CSE_OK;
}

int32_t cse_hybrid_best(cse_ctx* ctx, const int32_t* job_ids, int32_t n, int32_t best_cost[3], int32_t best_job[3],
                        int32_t best_proc[3]) {
    if (!ctx || !job_ids || n < 1 || !best_cost) return CSE_EINVAL;
    int n_comp = -1, scheme = -1;
    for (int i = 0; i < n; ++i) {
        JobRec* J = nullptr;
        int rc = readable(ctx, job_ids[i], &J, -1);
        if (rc) return rc;
        // Components of different runs combine only within one scheme.
        if (scheme >= 0 && J->scheme != scheme)
            return fail(ctx, CSE_EINVAL, "job %d reduces scheme %d, job %d scheme %d", job_ids[i], J->scheme,
                        job_ids[0], scheme);
        scheme = J->scheme;
        n_comp = J->n_comp;
    }
    for (int c = 0; c < 3; ++c) {
        best_cost[c] = -1;
        if (best_job) best_job[c] = -1;
        if (best_proc) best_proc[c] = -1;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (int i = 0; i < n; ++i) {
        JobRec& J = ctx->jobs[job_ids[i]];
        int32_t cost[3], proc[3];
        if (J.driver && J.best_cost[0] >= 0) {
            for (int c = 0; c < n_comp; ++c) {
                cost[c] = J.best_cost[c];
                proc[c] = J.best_proc[c];
            }
        } else {
            // The best unit of each component: a device argmin over (cost, process).
            unsigned long long* d_key = nullptr;
            HIP_TRY(ctx, hipMalloc((void**)&d_key, sizeof(unsigned long long) * 3));
            hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, nullptr, (int32_t*)d_key, 6, -1);
            for (int c = 0; c < n_comp; ++c)
                hipLaunchKernelGGL(csek::driver_argmin_kernel, dim3((J.cfg.n_proc + 255) / 256), dim3(256), 0,
                                   nullptr, J.cj[c].st.cost, J.cfg.n_proc, d_key + c);
            unsigned long long key[3];
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpy(key, d_key, sizeof key, hipMemcpyDeviceToHost);
            (void)hipFree(d_key);
            if (e != hipSuccess) return fail(ctx, CSE_EHIP, "best units: %s", hipGetErrorString(e));
            for (int c = 0; c < n_comp; ++c) {
                cost[c] = (int32_t)(key[c] >> 32);
                proc[c] = (int32_t)(key[c] & 0xFFFFFFFFu);
            }
        }
        for (int c = 0; c < n_comp; ++c) {
            if (best_cost[c] >= 0 && cost[c] >= best_cost[c]) continue;
            best_cost[c] = cost[c];
            if (best_job) best_job[c] = job_ids[i];
            if (best_proc) best_proc[c] = proc[c];
        }
    }
    return CSE_OK;
}

int32_t cse_driver_totals(cse_ctx* ctx, int32_t job_id, int32_t* totals, uint64_t* elapsed_ns, int32_t cap,
                          int32_t* n) {
    if (!ctx || !n) return CSE_EINVAL;
    JobRec* J = nullptr;
    int rc = readable(ctx, job_id, &J, -1);
    if (rc) return rc;
    if (!J->driver) return fail(ctx, CSE_EINVAL, "job %d did not run the driver", job_id);
    *n = (int32_t)J->totals.size();
    if (!totals && !elapsed_ns) return CSE_OK;
    if (cap < *n) return fail(ctx, CSE_ERANGE, "cap %d < %d", cap, *n);
    for (int32_t i = 0; i < *n; ++i) {
        if (totals) totals[i] = J->totals[(size_t)i];
        if (elapsed_ns) elapsed_ns[i] = J->iter_ns[(size_t)i];
    }
    return CSE_OK;
}

}  // extern "C"

namespace {
int release_job(cse_ctx* ctx, int32_t job_id) {
    JobRec* J = nullptr;
    BatchRec* B = batch_of(ctx, job_id, &J);
    if (!B) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    const int bid = J->batch;
    if (!B->finished) (void)wait_batch(ctx, *B);
    B->jobs.erase(std::remove(B->jobs.begin(), B->jobs.end(), job_id), B->jobs.end());
    free_job_device(ctx, *J);
    ctx->jobs.erase(job_id);
    B->built = false;
    if (!B->is_server && B->jobs.empty()) drop_batch(ctx, bid);
    return CSE_OK;
}
}  // namespace

extern "C" {

int32_t cse_job_release(cse_ctx* ctx, int32_t job_id) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->jobs.find(job_id);
    if (it == ctx->jobs.end()) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (it->second.server) return fail(ctx, CSE_EINVAL, "server job %d is released with cse_server_release", job_id);
    return release_job(ctx, job_id);
}

// ---------------------------------------------------------------------------
// Server: continuous batching of reduction jobs.
// ---------------------------------------------------------------------------

int32_t cse_server_create(cse_ctx* ctx, uint64_t max_state_bytes, uint32_t round_steps, void* stream,
                          cse_server** out) {
    if (!ctx || !out || round_steps == 0) return CSE_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    cse_server* s = new (std::nothrow) cse_server();
    if (!s) return CSE_ENOMEM;
    s->ctx = ctx;
    s->max_bytes = max_state_bytes;
    s->round_steps = round_steps;
    int bid = -1;
    int rc = new_batch(ctx, (hipStream_t)stream, &bid);
    if (rc) { delete s; return rc; }
    BatchRec& B = ctx->batches[bid];
    B.is_server = true;
    B.owner = s;
    B.rounds = true;
    s->batch = bid;
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, B.stream, B.d_err, 1, 0);
    *out = s;
    return CSE_OK;
}

int32_t cse_server_submit(cse_server* s, int32_t scheme_id, const cse_run_cfg* cfg, int32_t* job_id) {
    if (!s || !job_id) return CSE_EINVAL;
    cse_ctx* ctx = s->ctx;
    if (!ctx->schemes.count(scheme_id)) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_id);
    int rc = validate_cfg(ctx, cfg);
    if (rc) return rc;
    if (job_bytes(ctx, scheme_id, *cfg) > s->max_bytes)
        return fail(ctx, CSE_ENOMEM, "job needs %zu B, server budget %llu B", job_bytes(ctx, scheme_id, *cfg),
                    (unsigned long long)s->max_bytes);
    // A job whose unit state cannot fit a workgroup's LDS in its layout
    // would fail every round's launch: refused here.
    const SchemeRec& sc = ctx->schemes[scheme_id];
    for (int c = 0; c < sc.n_comp; ++c)
        if (lds_bytes(sc.comp[c]) > ctx->lds_max)
            return fail(ctx, CSE_ENOMEM, "component %d needs %zu B of LDS per unit (max %zu)", c,
                        lds_bytes(sc.comp[c]), ctx->lds_max);
    const int jid = ctx->next_job++;
    JobRec& J = ctx->jobs[jid];
    J.scheme = scheme_id;
    J.cfg = *cfg;
    J.batch = s->batch;
    J.server = true;
    J.state = CSE_JOB_QUEUED;
    J.t_submit = now_ns();
    J.n_comp = ctx->schemes[scheme_id].n_comp;
    s->queue.push_back(jid);
    *job_id = jid;
    return CSE_OK;
}

int32_t cse_server_tick(cse_server* s, int32_t* n_running, int32_t* n_queued) {
    if (!s) return CSE_EINVAL;
    cse_ctx* ctx = s->ctx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    BatchRec& B = ctx->batches[s->batch];
    // Admission: first come, first served, while the footprint fits.
    while (!s->queue.empty()) {
        JobRec& J = ctx->jobs[s->queue.front()];
        const size_t need = job_bytes(ctx, J.scheme, J.cfg);
        if (s->used_bytes + need > s->max_bytes) break;
        int rc = alloc_job(ctx, J);
        if (rc) {
            // Retired as failed; the queue and the running jobs go on.
            free_job_device(ctx, J);
            J.state = CSE_JOB_FAILED;
            J.t_done = now_ns();
            s->queue.pop_front();
            continue;
        }
        s->used_bytes += J.bytes;
        J.budget = shares(J.cfg) ? (int)J.cfg.share_every : (int)s->round_steps;
        rc = init_job(ctx, J, B.stream);
        if (rc) return rc;
        J.state = CSE_JOB_RUNNING;
        J.t_admit = now_ns();
        B.jobs.push_back(s->queue.front());
        s->queue.pop_front();
        s->dirty = true;
    }
    if (!B.jobs.empty()) {
        if (s->dirty) {
            int rc = build_segments(ctx, B);
            if (rc) return rc;
            s->dirty = false;
        }
        B.finished = false;
        int rc = round_once(ctx, B);
        B.finished = true;
        if (rc) return rc;
        rc = check_err(ctx, B);
        if (rc) return rc;
        const uint64_t t = now_ns();
        std::vector<int> still;
        for (int jid : B.jobs) {
            JobRec& J = ctx->jobs[jid];
            if (J.done || J.cancelled) {
                J.state = CSE_JOB_DONE;
                J.t_done = t;
                s->dirty = true;
            } else {
                still.push_back(jid);
            }
        }
        B.jobs.swap(still);
    }
    if (n_running) *n_running = (int32_t)B.jobs.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return CSE_OK;
}

int32_t cse_server_job_info(cse_server* s, int32_t job_id, int32_t* state, uint64_t times_ns[3]) {
    if (!s) return CSE_EINVAL;
    cse_ctx* ctx = s->ctx;
    auto it = ctx->jobs.find(job_id);
    if (it == ctx->jobs.end() || !it->second.server) return fail(ctx, CSE_ENOENT, "unknown server job %d", job_id);
    if (state) *state = it->second.state;
    if (times_ns) {
        times_ns[0] = it->second.t_submit;
        times_ns[1] = it->second.t_admit;
        times_ns[2] = it->second.t_done;
    }
    return CSE_OK;
}

int32_t cse_server_release(cse_server* s, int32_t job_id) {
    if (!s) return CSE_EINVAL;
    cse_ctx* ctx = s->ctx;
    auto it = ctx->jobs.find(job_id);
    if (it == ctx->jobs.end() || !it->second.server) return fail(ctx, CSE_ENOENT, "unknown server job %d", job_id);
    if (it->second.state != CSE_JOB_DONE && it->second.state != CSE_JOB_FAILED)
        return fail(ctx, CSE_EBUSY, "server job %d is not done", job_id);
    if (it->second.state == CSE_JOB_FAILED) {
        ctx->jobs.erase(it);  // holds no device memory
        return CSE_OK;
    }
    s->used_bytes -= std::min<uint64_t>(s->used_bytes, it->second.bytes);
    return release_job(ctx, job_id);
}

void cse_server_destroy(cse_server* s) {
    if (!s) return;
    cse_ctx* ctx = s->ctx;
    (void)hipSetDevice(ctx->device);
    drop_batch(ctx, s->batch);
    delete s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Random flips of a scheme (Sec. 3.5.3).
// ---------------------------------------------------------------------------
namespace {

int validate_flip(cse_ctx* ctx, const int8_t* U, const int8_t* V, const int8_t* W, int32_t rank,
                  const cse_flip_cfg* f) {
    if (!U || !V || !W || !f || rank < 1) return fail(ctx, CSE_EINVAL, "null scheme or configuration");
    if (f->n < 1 || f->m < 1 || f->p < 1 || f->n * f->m > 4096 || f->m * f->p > 4096 || f->n * f->p > 4096)
        return fail(ctx, CSE_EINVAL, "format %d x %d x %d out of range", f->n, f->m, f->p);
    if (f->n_variants < 1 || f->n_variants > 4096) return fail(ctx, CSE_EINVAL, "n_variants %d out of range", f->n_variants);
    if (f->max_flips < 1 || f->max_flips > 65534) return fail(ctx, CSE_EINVAL, "max_flips %d out of range", f->max_flips);
    if (f->reserved) return fail(ctx, CSE_EINVAL, "reserved field must be 0");
    const int len[3] = {f->n * f->m, f->m * f->p, f->n * f->p};
    for (int x = 0; x < 3; ++x) {
        const int8_t* M = x == 0 ? U : x == 1 ? V : W;
        for (size_t k = 0; k < (size_t)rank * len[x]; ++k)
            if (M[k] < -1 || M[k] > 1) return fail(ctx, CSE_EINVAL, "scheme coefficient not ternary");
    }
    if (csek::flip_lds_bytes(rank, len[0], len[1], len[2]) > ctx->lds_max)
        return fail(ctx, CSE_ENOMEM, "a %d-product scheme needs %zu B of LDS to flip (max %zu)", rank,
                    csek::flip_lds_bytes(rank, len[0], len[1], len[2]), ctx->lds_max);
    return CSE_OK;
}

// Device buffers of one flip generation: the scheme and all its variants.
struct FlipBufs {
    int8_t* base = nullptr;  // U | V | W
    int8_t* var = nullptr;   // M x (U | V | W) then M x W^T
    int32_t* n_done = nullptr;
    ~FlipBufs() {
        if (base) (void)hipFree(base);
        if (var) (void)hipFree(var);
        if (n_done) (void)hipFree(n_done);
    }
};

int flip_generate(cse_ctx* ctx, const int8_t* U, const int8_t* V, const int8_t* W, int r, const cse_flip_cfg* f,
                  uint64_t seed, uint32_t iteration, hipStream_t s, FlipBufs& B, csek::FlipArgs* out) {
    const int len[3] = {f->n * f->m, f->m * f->p, f->n * f->p};
    const size_t per = (size_t)r * (len[0] + len[1] + len[2]);
    const int Mv = f->n_variants;
    if (!B.base) {
        HIP_TRY(ctx, hipMalloc((void**)&B.base, per));
        HIP_TRY(ctx, hipMalloc((void**)&B.var, per * Mv + (size_t)Mv * r * len[2]));
        HIP_TRY(ctx, hipMalloc((void**)&B.n_done, sizeof(int32_t) * Mv));
        HIP_TRY(ctx, hipMemcpyAsync(B.base, U, (size_t)r * len[0], hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(B.base + (size_t)r * len[0], V, (size_t)r * len[1], hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(B.base + (size_t)r * (len[0] + len[1]), W, (size_t)r * len[2],
                                    hipMemcpyHostToDevice, s));
    }
    csek::FlipArgs A{};
    A.U = B.base;
    A.V = B.base + (size_t)r * len[0];
    A.W = B.base + (size_t)r * (len[0] + len[1]);
    A.outU = B.var;
    A.outV = B.var + (size_t)Mv * r * len[0];
    A.outW = B.var + (size_t)Mv * r * (len[0] + len[1]);
    A.outWt = B.var + per * Mv;
    A.n_done = B.n_done;
    A.r = r;
    for (int x = 0; x < 3; ++x) A.len[x] = len[x];
    A.max_flips = (uint32_t)f->max_flips;
    A.iteration = iteration;
    A.seed = seed;
    const size_t lds = csek::flip_lds_bytes(r, len[0], len[1], len[2]);
    if (lds > 65536)
        HIP_TRY(ctx, hipFuncSetAttribute((const void*)csek::flip_variants_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(csek::flip_variants_kernel, dim3(Mv), dim3(csek::kWave), lds, s, A);
    HIP_TRY(ctx, hipGetLastError());
    *out = A;
    return CSE_OK;
}

}  // namespace

extern "C" {

int32_t cse_flip_variants(cse_ctx* ctx, const int8_t* U, const int8_t* V, const int8_t* W, int32_t rank,
                          const cse_flip_cfg* fcfg, uint64_t seed, uint32_t iteration, int8_t* outU, int8_t* outV,
                          int8_t* outW, int32_t* n_flips) {
    if (!ctx) return CSE_EINVAL;
    int rc = validate_flip(ctx, U, V, W, rank, fcfg);
    if (rc) return rc;
    if (!outU || !outV || !outW) return fail(ctx, CSE_EINVAL, "null output");
    if (iteration > 1023) return fail(ctx, CSE_EINVAL, "iteration %u exceeds 1023", iteration);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    FlipBufs B;
    csek::FlipArgs A{};
    rc = flip_generate(ctx, U, V, W, rank, fcfg, seed, iteration, nullptr, B, &A);
    if (rc) return rc;
    const size_t Mv = (size_t)fcfg->n_variants;
    HIP_TRY(ctx, hipMemcpy(outU, A.outU, Mv * rank * A.len[0], hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(outV, A.outV, Mv * rank * A.len[1], hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(outW, A.outW, Mv * rank * A.len[2], hipMemcpyDeviceToHost));
    if (n_flips) HIP_TRY(ctx, hipMemcpy(n_flips, A.n_done, sizeof(int32_t) * Mv, hipMemcpyDeviceToHost));
    return CSE_OK;
}

int32_t cse_run_flips(cse_ctx* ctx, const int8_t* U, const int8_t* V, const int8_t* W, int32_t rank,
                      const cse_flip_cfg* fcfg, const cse_run_cfg* cfg, int32_t patience, int32_t max_iterations,
                      void* stream, int32_t* run_id, int32_t* iterations) {
    if (!ctx || !run_id) return CSE_EINVAL;
    int rc = validate_flip(ctx, U, V, W, rank, fcfg);
    if (rc) return rc;
    rc = validate_cfg(ctx, cfg);
    if (rc) return rc;
    if (cfg->iteration != 0) return fail(ctx, CSE_EINVAL, "the flip mode starts at iteration 0");
    if (max_iterations < 1 || max_iterations > 1024 || patience < 0)
        return fail(ctx, CSE_EINVAL, "iterations out of range");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const hipStream_t s = (hipStream_t)stream;
    const int Mv = fcfg->n_variants;
    const int len[3] = {fcfg->n * fcfg->m, fcfg->m * fcfg->p, fcfg->n * fcfg->p};
    FlipRun R;
    R.n = fcfg->n;
    R.m = fcfg->m;
    R.p = fcfg->p;
    R.r = rank;
    FlipBufs B;
    unsigned long long* d_st = nullptr;
    unsigned long long* d_key = nullptr;
    HIP_TRY(ctx, hipMalloc((void**)&d_st, 64));
    if (hipMalloc((void**)&d_key, sizeof(unsigned long long) * 3 * Mv) != hipSuccess) {
        (void)hipFree(d_st);
        return fail(ctx, CSE_EHIP, "hipMalloc of %d argmin keys failed", 3 * Mv);
    }
    int it = 0, unchanged = 0;
    std::vector<int32_t> sids, jobs;
    auto cleanup = [&]() {
        for (int j : jobs) (void)release_job(ctx, j);
        for (int sid : sids) {
            for (int c = 0; c < ctx->schemes[sid].n_comp; ++c) free_component(ctx->schemes[sid].comp[c]);
            ctx->schemes.erase(sid);
        }
        jobs.clear();
        sids.clear();
    };
    while (rc == CSE_OK) {
        csek::FlipArgs A{};
        rc = flip_generate(ctx, U, V, W, rank, fcfg, cfg->seed, (uint32_t)it, s, B, &A);
        if (rc) break;
        // Each variant as a scheme: U_v, V_v and W_v^T, analysed on the device.
        for (int v = 0; v < Mv && rc == CSE_OK; ++v) {
            SchemeRec sc;
            sc.n_comp = 3;
            const int8_t* comp[3] = {A.outU + (size_t)v * rank * len[0], A.outV + (size_t)v * rank * len[1],
                                     A.outWt + (size_t)v * rank * len[2]};
            const int rows[3] = {rank, rank, len[2]}, cols[3] = {len[0], len[1], rank};
            int c = 0;
            for (; c < 3 && rc == CSE_OK; ++c)
                rc = load_component_device(ctx, comp[c], rows[c], cols[c], s, d_st, &sc.comp[c]);
            if (rc) {
                for (int k = 0; k + 1 < c; ++k) free_component(sc.comp[k]);
                break;
            }
            const int id = ctx->next_scheme++;
            ctx->schemes[id] = sc;
            sids.push_back(id);
        }
        if (rc) break;
        // All variants in one batch: variant v with seed + v and this iteration's draws.
        std::vector<cse_run_cfg> cfgs((size_t)Mv, *cfg);
        for (int v = 0; v < Mv; ++v) {
            cfgs[v].seed = cfg->seed + (uint64_t)v;
            cfgs[v].iteration = (uint32_t)it;
        }
        int bid = -1;
        rc = create_batch(ctx, sids.data(), cfgs.data(), Mv, stream, &bid);
        if (rc) break;
        jobs = ctx->batches[bid].jobs;
        rc = start_batch(ctx, bid);
        if (rc) {
            jobs.clear();  // dropped with the batch
            break;
        }
        rc = wait_batch(ctx, ctx->batches[bid]);
        if (rc) break;
        // Each variant's best unit per component: (cost, process) argmin.
        hipLaunchKernelGGL(csek::fill_i32_kernel, dim3((6 * Mv + 255) / 256), dim3(256), 0, s, (int32_t*)d_key,
                           6 * Mv, -1);
        for (int v = 0; v < Mv; ++v)
            for (int c = 0; c < 3; ++c)
                hipLaunchKernelGGL(csek::driver_argmin_kernel, dim3((cfg->n_proc + 255) / 256), dim3(256), 0, s,
                                   ctx->jobs[jobs[v]].cj[c].st.cost, cfg->n_proc, d_key + 3 * v + c);
        std::vector<unsigned long long> key((size_t)3 * Mv);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(key.data(), d_key, sizeof(unsigned long long) * 3 * Mv, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = fail(ctx, CSE_EHIP, "variant bests: %s", hipGetErrorString(e));
            break;
        }
        int best_v = 0;
        int32_t best_t = -1;
        for (int v = 0; v < Mv; ++v) {
            int32_t t = 0;
            for (int c = 0; c < 3; ++c) t += (int32_t)(key[3 * v + c] >> 32);
            if (best_t < 0 || t < best_t) {
                best_t = t;
                best_v = v;
            }
        }
        if (R.best_total < 0 || best_t < R.best_total) {
            R.best_total = best_t;
            R.variant = best_v;
            R.iteration = it;
            R.U.resize((size_t)rank * len[0]);
            R.V.resize((size_t)rank * len[1]);
            R.W.resize((size_t)rank * len[2]);
            e = hipMemcpy(R.U.data(), A.outU + (size_t)best_v * rank * len[0], R.U.size(), hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = hipMemcpy(R.V.data(), A.outV + (size_t)best_v * rank * len[1], R.V.size(), hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = hipMemcpy(R.W.data(), A.outW + (size_t)best_v * rank * len[2], R.W.size(), hipMemcpyDeviceToHost);
            const JobRec& J = ctx->jobs[jobs[best_v]];
            for (int c = 0; c < 3 && e == hipSuccess; ++c) {
                const uint32_t proc = (uint32_t)(key[3 * best_v + c] & 0xFFFFFFFFu);
                const int nf = std::max(1, ctx->schemes[sids[best_v]].comp[c].n_fmax);
                int32_t L = 0;
                R.best_cost[c] = (int32_t)(key[3 * best_v + c] >> 32);
                e = hipMemcpy(&L, J.cj[c].st.t + proc, 4, hipMemcpyDeviceToHost);
                R.keys[c].assign((size_t)std::max(0, L), 0u);
                if (e == hipSuccess && L > 0)
                    e = hipMemcpy(R.keys[c].data(), J.cj[c].st.prog + (size_t)proc * nf, (size_t)L * 4,
                                  hipMemcpyDeviceToHost);
            }
            if (e != hipSuccess) {
                rc = fail(ctx, CSE_EHIP, "best variant readback: %s", hipGetErrorString(e));
                break;
            }
        }
        unchanged = (!R.totals.empty() && R.best_total == R.totals.back()) ? unchanged + 1 : 0;
        R.totals.push_back(R.best_total);
        cleanup();
        ++it;
        if (unchanged >= patience || it >= max_iterations) break;
    }
    cleanup();
    (void)hipFree(d_st);
    (void)hipFree(d_key);
    if (iterations) *iterations = it;
    if (rc) return rc;
    const int id = ctx->next_flip++;
    ctx->flips[id] = std::move(R);
    *run_id = id;
    return CSE_OK;
}

int32_t cse_flip_best(cse_ctx* ctx, int32_t run_id, int8_t* U, int8_t* V, int8_t* W, int32_t best_cost[3],
                      int32_t* variant, int32_t* iteration, int32_t* totals, int32_t cap, int32_t* n_iter) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->flips.find(run_id);
    if (it == ctx->flips.end()) return fail(ctx, CSE_ENOENT, "unknown flip run %d", run_id);
    const FlipRun& R = it->second;
    if (U) std::memcpy(U, R.U.data(), R.U.size());
    if (V) std::memcpy(V, R.V.data(), R.V.size());
    if (W) std::memcpy(W, R.W.data(), R.W.size());
    if (best_cost)
        for (int c = 0; c < 3; ++c) best_cost[c] = R.best_cost[c];
    if (variant) *variant = R.variant;
    if (iteration) *iteration = R.iteration;
    if (n_iter) *n_iter = (int32_t)R.totals.size();
    if (totals) {
        if (cap < (int32_t)R.totals.size()) return fail(ctx, CSE_ERANGE, "cap %d < %zu", cap, R.totals.size());
        for (size_t i = 0; i < R.totals.size(); ++i) totals[i] = R.totals[i];
    }
    return CSE_OK;
}

int32_t cse_flip_program(cse_ctx* ctx, int32_t run_id, int32_t comp, int32_t* triples, int32_t cap, int32_t* n_fresh,
                         int32_t* needed) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->flips.find(run_id);
    if (it == ctx->flips.end()) return fail(ctx, CSE_ENOENT, "unknown flip run %d", run_id);
    if (comp < 0 || comp > 2) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    const std::vector<uint32_t>& k = it->second.keys[comp];
    const int len = (int)k.size();
    if (n_fresh) *n_fresh = len;
    if (needed) *needed = len;
    if (cap < len || (!triples && len > 0)) return fail(ctx, CSE_ERANGE, "cap %d < %d", cap, len);
    for (int i = 0; i < len; ++i) {
        triples[3 * i + 0] = (int32_t)(k[i] >> 16);
        triples[3 * i + 1] = (int32_t)((k[i] >> 1) & 0x7FFFu);
        triples[3 * i + 2] = (k[i] & 1u) ? -1 : 1;
    }
    return CSE_OK;
}

int32_t cse_flip_release(cse_ctx* ctx, int32_t run_id) {
    if (!ctx) return CSE_EINVAL;
    if (!ctx->flips.erase(run_id)) return fail(ctx, CSE_ENOENT, "unknown flip run %d", run_id);
    return CSE_OK;
}

}  // extern "C"

namespace {

// Bump allocation inside the static scratch array (256-byte aligned pieces).
struct ScratchCarve {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t bytes) {
        T* p = (T*)(base + off);
        off += (bytes + 255) & ~size_t(255);
        return p;
    }
};

}  // namespace

extern "C" {

int32_t cse_reduce_static(cse_ctx* ctx, const int8_t* A, int32_t rows, int32_t cols, int32_t comp,
                          const cse_run_cfg* cfg, void* stream, int32_t* cost, int32_t* length, uint32_t* prog,
                          int32_t prog_cap, int32_t* needed) {
    if (!ctx) return CSE_EINVAL;
    if (!A || rows < 1 || cols < 1) return fail(ctx, CSE_EINVAL, "empty system (%d x %d)", rows, cols);
    if (rows > kMaxRows) return fail(ctx, CSE_EINVAL, "rows %d exceed %d", rows, kMaxRows);
    if (comp < 0 || comp > 2) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    int rc = validate_cfg(ctx, cfg);
    if (rc) return rc;
    if (shares(*cfg)) return fail(ctx, CSE_EINVAL, "cse_reduce_static runs without sharing rounds");
    if (cfg->count_path == CSE_COUNT_MFMA)
        return fail(ctx, CSE_EINVAL, "cse_reduce_static counts the input by popcounts only");
    if (ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device])
        return fail(ctx, CSE_EHIP, "no static scratch address for device %d", ctx->device);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const hipStream_t s = (hipStream_t)stream;
    const uint32_t n = cfg->n_proc;
    ScratchCarve sc{(char*)g_scratch_ptr[ctx->device]};
    unsigned long long* d_st = sc.take<unsigned long long>(64);
    int* d_err = sc.take<int>(64);
    unsigned long long* d_t0 = sc.take<unsigned long long>(64);  // start stamp (8 B), round counter (4 B)
    csek::Segment* d_seg = sc.take<csek::Segment>(sizeof(csek::Segment));

    // Validation and sizes on the device (Sec. 3.2.1).
    unsigned long long st[5] = {0, 0, 0, 0, 0};
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)d_st, 10, 0);
    hipLaunchKernelGGL(csek::input_stats_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, A, rows, cols, d_st);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(st, d_st, sizeof st, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (st[3] || st[4])
        return fail(ctx, CSE_EINVAL, "system %d x %d: %llu entries not ternary, %llu all-zero rows", rows, cols, st[3],
                    st[4]);
    DevComp c;
    c.n_e = rows;
    c.n_x = cols;
    rc = size_component(ctx, c, (long long)st[0], (long long)st[1], (long long)st[2]);
    if (rc) return rc;
    const int pstride = std::max(1, c.n_fmax);
    if (needed) *needed = pstride;
    if (prog_cap < pstride || !cost || !length || !prog)
        return fail(ctx, CSE_ERANGE, "programs need %d entries per process (cap %d) and non-null outputs", pstride,
                    prog_cap);

    // The input's column bitsets and candidate lists (the pieces every unit
    // starts from), then the per-unit arrays the caller does not hold.
    const size_t col_bytes = (size_t)cols * c.W * 8;
    c.d_P = sc.take<uint64_t>(col_bytes);
    c.d_N = sc.take<uint64_t>(col_bytes);
    int32_t* buf = sc.take<int32_t>(((size_t)4 * cols + 4) * 4);
    c.d_cand0 = sc.take<uint64_t>((size_t)c.m_cap * 8);
    c.d_tl0 = sc.take<uint32_t>((size_t)c.m_cap * 4);
    if (sc.off > kStaticScratchBytes)
        return fail(ctx, CSE_ENOMEM, "%u processes of a %d x %d system need %zu B of scratch (max %zu)", n, rows,
                    cols, sc.off, kStaticScratchBytes);
    hipLaunchKernelGGL(csek::input_columns_kernel, dim3((cols * c.W + 255) / 256), dim3(256), 0, s, A, rows, cols,
                       c.W, c.d_P, c.d_N);
    const int nx = cols;
    int32_t* row_n = buf;
    int32_t* col_n = buf + nx;
    int32_t* row_off = buf + 2 * nx;
    int32_t* col_off = buf + 3 * nx + 1;
    int32_t* d_tot = buf + 4 * nx + 2;
    csek::PairSource src{c.d_P, c.d_N, c.W, nullptr, 0, nx};
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3((2 * nx + 255) / 256), dim3(256), 0, s, buf, 2 * nx, 0);
    hipLaunchKernelGGL(csek::input_count_kernel, dim3(nx), dim3(csek::kInputBlock), 0, s, src, row_n, col_n);
    hipLaunchKernelGGL(csek::input_scan_kernel, dim3(1), dim3(csek::kInputBlock), 0, s, row_n, col_n, nx, row_off,
                       col_off, d_tot);
    HIP_TRY(ctx, hipGetLastError());
    int32_t tot[2] = {0, 0};
    HIP_TRY(ctx, hipMemcpyAsync(tot, d_tot, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (tot[0] != tot[1] || tot[0] < 0 || tot[0] > c.m_cap)
        return fail(ctx, CSE_EHIP, "input analysis: %d candidates by first variable, %d by second (bound %d)", tot[0],
                    tot[1], c.m_cap);
    hipLaunchKernelGGL(csek::input_rows_kernel, dim3(nx), dim3(csek::kInputBlock), 0, s, src, row_off, c.d_cand0);
    hipLaunchKernelGGL(csek::input_cols_kernel, dim3(nx), dim3(csek::kInputBlock), 0, s, src, row_off, col_off,
                       c.d_cand0, c.d_tl0);
    HIP_TRY(ctx, hipGetLastError());
    c.m0 = tot[0];
    rc = pick_layout(ctx, c);
    if (rc) return rc;

    csek::UnitState S{};
    S.ops = sc.take<unsigned long long>((size_t)n * 8);
    S.finish = sc.take<unsigned long long>((size_t)n * 8);
    S.executed = sc.take<int32_t>((size_t)n * 4);
    S.epoch = sc.take<int32_t>((size_t)n * 4);
    S.k0 = sc.take<int32_t>((size_t)n * 4);
    S.active = sc.take<int32_t>((size_t)n * 4);
    S.strat = sc.take<int32_t>((size_t)n * 4);
    S.prog = prog;
    S.t = length;
    S.cost = cost;
    S.t0 = d_t0;
    S.round = (int32_t*)((char*)d_t0 + 8);
    if (sc.off > kStaticScratchBytes)
        return fail(ctx, CSE_ENOMEM, "%u processes need %zu B of scratch (max %zu)", n, sc.off, kStaticScratchBytes);
    if (c.gs) {
        const size_t slots = (size_t)n * slot_bytes(c);
        if (slots > kStaticScratchBytes - sc.off)
            return fail(ctx, CSE_ENOMEM, "%u processes need %zu B of HBM unit state beside %zu B (scratch max %zu)", n,
                        slots, sc.off, kStaticScratchBytes);
        S.gs_stride = slot_bytes(c);
        S.gs_base = sc.take<char>(slots);
    }

    JobRec J;
    J.cfg = *cfg;
    J.budget = -1;
    csek::Segment sg{};
    sg.C = comp_args(c, comp, false);
    sg.C.prog_stride = prog_cap;
    sg.R = run_args(ctx, J);
    sg.S = S;
    sg.unit_begin = 0;
    LaunchGroup G;
    G.W = c.W;
    G.gs = c.gs;
    G.adj = c.adj;
    G.tl = false;
    G.nw = c.nw;
    G.gp = cfg->weights[CSE_STRAT_GP] != 0;
    G.n_grid = n;
    G.lds = lds_bytes(c);
    G.seg_begin = 0;
    G.n_segs = 1;
    G.order_begin = 0;
    rc = set_lds_limit(ctx, G);
    if (rc) return rc;
    HIP_TRY(ctx, hipMemcpyAsync(d_seg, &sg, sizeof sg, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(csek::fill_i32_kernel, dim3(1), dim3(64), 0, s, d_err, 1, 0);
    hipLaunchKernelGGL(csek::init_units_kernel, dim3((n + 255) / 256), dim3(256), 0, s, S, n, 1);
    HIP_TRY(ctx, hipGetLastError());
    rc = launch_group(ctx, G, d_seg, nullptr, d_err, s);
    if (rc) return rc;
    int herr = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&herr, d_err, sizeof herr, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (herr) return fail(ctx, CSE_EHIP, "device consistency check failed (flags 0x%x)", herr);
    return CSE_OK;
}

}  // extern "C"

