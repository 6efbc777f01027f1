// cse_api.hip -- host runtime of libcse: the C ABI declared in include/cse.h.
//
// A context owns loaded schemes (input systems as column bitsets in HBM) and
// jobs (per-unit state and programs in HBM).  A job launches, per component,
// one workgroup per process; with sharing rounds (Sec. 3.5.2) the host
// alternates step launches of at most share_every steps with the sharing
// kernels until no unit of the job is active.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "cse.h"
#include "cse_kernels.hpp"
#include "cse_share.hpp"

namespace {

constexpr int kMaxRows = 512;   // W <= 8 row words
constexpr int kMaxVars = 32767; // 15-bit variable ids

struct DevComp {
    int n_e = 0, n_x = 0, n_fmax = 0, W = 0, m_cap = 0, naive0 = 0;
    long long occ0 = 0;
    uint64_t* d_P = nullptr;
    uint64_t* d_N = nullptr;
};

struct SchemeRec {
    int n_comp = 0;
    DevComp comp[3];
};

struct CompJob {
    csek::UnitState st{};
    void* block = nullptr;     // one allocation for all per-unit arrays
};

struct JobRec {
    int scheme = -1;
    cse_run_cfg cfg{};
    hipStream_t stream = nullptr;
    int n_comp = 0;
    CompJob cj[3];
    unsigned long long* d_t0 = nullptr;
    int* d_err = nullptr;
    hipEvent_t ev_done = nullptr;
    bool finished = false;
};

}  // namespace

struct cse_ctx {
    int device = 0;
    std::string err;
    std::map<int, SchemeRec> schemes;
    std::map<int, JobRec> jobs;
    int next_scheme = 1;
    int next_job = 1;
    size_t lds_max = 65536;
    uint64_t tick_hz = 100000000ull;
};

namespace {

int fail(cse_ctx* ctx, int code, const char* fmt, ...) {
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

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail((ctx), CSE_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t lds_bytes(const DevComp& c) {
    const size_t n_vmax = (size_t)c.n_x + c.n_fmax;
    return 2 * n_vmax * c.W * 8 + (size_t)c.m_cap * 8 + n_vmax * 4 + 16;
}

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
    // Each substitution removes c >= 2 nonzeros and no row empties, so at
    // most floor((nnz - n_e) / 2) fresh variables; candidates each use at
    // least two of the (never growing) pair occurrences.
    c.n_fmax = (int)((nnz - rows) / 2);
    if ((long long)cols + c.n_fmax > kMaxVars)
        return fail(ctx, CSE_EINVAL, "variables %lld exceed %d", (long long)cols + c.n_fmax, kMaxVars);
    c.W = (rows + 63) / 64;
    c.occ0 = occ;
    c.m_cap = (int)std::max<long long>(1, occ / 2);
    c.naive0 = (int)naive;
    std::vector<uint64_t> P((size_t)cols * c.W, 0), N((size_t)cols * c.W, 0);
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) {
            const int8_t v = A[(size_t)i * cols + j];
            if (v > 0) P[(size_t)j * c.W + i / 64] |= 1ull << (i % 64);
            if (v < 0) N[(size_t)j * c.W + i / 64] |= 1ull << (i % 64);
        }
    const size_t bytes = P.size() * 8;
    HIP_TRY(ctx, hipMalloc(&c.d_P, bytes));
    HIP_TRY(ctx, hipMalloc(&c.d_N, bytes));
    HIP_TRY(ctx, hipMemcpy(c.d_P, P.data(), bytes, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(c.d_N, N.data(), bytes, hipMemcpyHostToDevice));
    *out = c;
    return CSE_OK;
}

void free_component(DevComp& c) {
    if (c.d_P) (void)hipFree(c.d_P);
    if (c.d_N) (void)hipFree(c.d_N);
    c.d_P = c.d_N = nullptr;
}

int validate_cfg(cse_ctx* ctx, const cse_run_cfg* cfg) {
    if (!cfg) return fail(ctx, CSE_EINVAL, "null configuration");
    if (cfg->n_proc < 1 || cfg->n_proc > (1u << 24)) return fail(ctx, CSE_EINVAL, "n_proc %u out of range", cfg->n_proc);
    unsigned long long tw = 0;
    for (int i = 0; i < 7; ++i) tw += cfg->weights[i];
    if (tw == 0 || tw > 0xFFFFFFFFull) return fail(ctx, CSE_EINVAL, "strategy weights must sum to 1..2^32-1");
    if (cfg->weights[CSE_STRAT_GP] != 0) return fail(ctx, CSE_EINVAL, "greedy-potential is not available");
    unsigned long long mw = 0;
    for (int i = 0; i < 4; ++i) mw += cfg->mix_weights[i];
    if (cfg->weights[CSE_STRAT_MIX] && (mw == 0 || mw > 0xFFFFFFFFull))
        return fail(ctx, CSE_EINVAL, "mix weights must sum to 1..2^32-1");
    if (cfg->gr_p_q16 > 65536) return fail(ctx, CSE_EINVAL, "gr_p_q16 > 65536");
    if (cfg->share_max_rounds > 1023) return fail(ctx, CSE_EINVAL, "share_max_rounds > 1023");
    if (cfg->share_src_pm > 1000 || cfg->share_dst_pm > 1000) return fail(ctx, CSE_EINVAL, "per mille > 1000");
    if (cfg->count_path > CSE_COUNT_MFMA) return fail(ctx, CSE_EINVAL, "unknown count path");
    if (cfg->reserved[0] || cfg->reserved[1] || cfg->reserved[2]) return fail(ctx, CSE_EINVAL, "reserved fields must be 0");
    return CSE_OK;
}

csek::RunArgs run_args(const cse_run_cfg& cfg, int budget) {
    csek::RunArgs R{};
    R.seed = cfg.seed;
    for (int i = 0; i < 7; ++i) R.weights[i] = cfg.weights[i];
    for (int i = 0; i < 4; ++i) R.mix_weights[i] = cfg.mix_weights[i];
    R.proc0_greedy = cfg.proc0_greedy;
    R.gr_p_q16 = cfg.gr_p_q16;
    R.step_cap = cfg.step_cap;
    R.iteration = cfg.iteration;
    R.budget = budget;
    R.n_units = cfg.n_proc;
    return R;
}

csek::CompArgs comp_args(const DevComp& c, int comp) {
    csek::CompArgs C{};
    C.P0 = c.d_P;
    C.N0 = c.d_N;
    C.n_e = c.n_e;
    C.n_x = c.n_x;
    C.n_fmax = c.n_fmax;
    C.m_cap = c.m_cap;
    C.naive0 = c.naive0;
    C.comp = (uint32_t)comp;
    C.prog_stride = std::max(1, c.n_fmax);
    return C;
}

template <int W>
int launch_step_w(cse_ctx* ctx, const DevComp& c, const csek::CompArgs& C, const csek::RunArgs& R,
                  const csek::UnitState& S, int* d_err, hipStream_t s) {
    const size_t lds = lds_bytes(c);
    if (lds > ctx->lds_max) return fail(ctx, CSE_ENOMEM, "unit state needs %zu B of LDS (max %zu)", lds, ctx->lds_max);
    if (lds > 65536) HIP_TRY(ctx, hipFuncSetAttribute((const void*)csek::step_kernel<W>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(csek::step_kernel<W>, dim3(R.n_units), dim3(csek::kWave), lds, s, C, R, S, d_err);
    HIP_TRY(ctx, hipGetLastError());
    return CSE_OK;
}

int launch_step(cse_ctx* ctx, const DevComp& c, int comp, const cse_run_cfg& cfg, int budget,
                const csek::UnitState& S, int* d_err, hipStream_t s) {
    const csek::CompArgs C = comp_args(c, comp);
    const csek::RunArgs R = run_args(cfg, budget);
    switch (c.W) {
    case 1: return launch_step_w<1>(ctx, c, C, R, S, d_err, s);
    case 2: return launch_step_w<2>(ctx, c, C, R, S, d_err, s);
    case 3: return launch_step_w<3>(ctx, c, C, R, S, d_err, s);
    case 4: return launch_step_w<4>(ctx, c, C, R, S, d_err, s);
    case 5: return launch_step_w<5>(ctx, c, C, R, S, d_err, s);
    case 6: return launch_step_w<6>(ctx, c, C, R, S, d_err, s);
    case 7: return launch_step_w<7>(ctx, c, C, R, S, d_err, s);
    case 8: return launch_step_w<8>(ctx, c, C, R, S, d_err, s);
    default: return fail(ctx, CSE_EINVAL, "row words %d unsupported", c.W);
    }
}

int alloc_comp_job(cse_ctx* ctx, const DevComp& c, uint32_t n, unsigned long long* d_t0, CompJob* cj) {
    const size_t prog = (size_t)n * std::max(1, c.n_fmax) * 4;
    const size_t i32 = (size_t)n * 4;
    const size_t u64 = (size_t)n * 8;
    const size_t total = prog + 7 * i32 + 2 * u64 + 64 * 10;
    char* base = nullptr;
    HIP_TRY(ctx, hipMalloc((void**)&base, total));
    cj->block = base;
    auto take = [&](size_t bytes) { char* p = base; base += (bytes + 63) & ~size_t(63); return p; };
    csek::UnitState& S = cj->st;
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
    S.t0 = d_t0;
    return CSE_OK;
}

JobRec* find_job(cse_ctx* ctx, int id) {
    auto it = ctx->jobs.find(id);
    return it == ctx->jobs.end() ? nullptr : &it->second;
}

int check_err(cse_ctx* ctx, JobRec& J) {
    int herr = 0;
    HIP_TRY(ctx, hipMemcpy(&herr, J.d_err, sizeof herr, hipMemcpyDeviceToHost));
    if (herr) return fail(ctx, CSE_EHIP, "device consistency check failed (flags 0x%x)", herr);
    return CSE_OK;
}

int wait_job(cse_ctx* ctx, JobRec& J) {
    if (!J.finished) {
        HIP_TRY(ctx, hipEventSynchronize(J.ev_done));
        J.finished = true;
        return check_err(ctx, J);
    }
    return CSE_OK;
}

// Sharing rounds (Sec. 3.5.2): every component advances by at most
// share_every steps per round, then each component pool runs one sharing
// event; the host reads the number of still-active units after each round
// and stops when none is left.  After share_max_rounds events the remaining
// units run to completion without sharing.
int run_sharing_rounds(cse_ctx* ctx, JobRec& J, const SchemeRec& sc) {
    const cse_run_cfg& cfg = J.cfg;
    const uint32_t n = cfg.n_proc;
    uint32_t n_src = (uint32_t)(((unsigned long long)n * cfg.share_src_pm + 999) / 1000);
    n_src = std::max(1u, std::min(n_src, n));
    int32_t* h_active = nullptr;
    int32_t* d_scratch = nullptr;
    const size_t per = csek::share_scratch_bytes(n);
    HIP_TRY(ctx, hipHostMalloc((void**)&h_active, 64 * sizeof(int32_t), hipHostMallocDefault));
    if (hipMalloc((void**)&d_scratch, per * J.n_comp) != hipSuccess) {
        (void)hipHostFree(h_active);
        return fail(ctx, CSE_ENOMEM, "sharing scratch of %zu B", per * J.n_comp);
    }
    bool live[3] = {true, true, true};
    int rc = CSE_OK;
    const dim3 blk(256), grd((n + 255) / 256);
    for (uint32_t r = 0; rc == CSE_OK; ++r) {
        const bool last = r >= cfg.share_max_rounds;
        for (int c = 0; c < J.n_comp && rc == CSE_OK; ++c)
            if (live[c]) rc = launch_step(ctx, sc.comp[c], c, cfg, last ? -1 : (int)cfg.share_every,
                                          J.cj[c].st, J.d_err, J.stream);
        if (rc || last) break;
        bool any = false;
        for (int c = 0; c < J.n_comp; ++c) {
            if (!live[c]) continue;
            csek::ShareScratch ss = csek::share_scratch(
                (int32_t*)((char*)d_scratch + per * c), n);
            hipLaunchKernelGGL(csek::share_clear_kernel, dim3(1), dim3(64), 0, J.stream, ss);
            hipLaunchKernelGGL(csek::share_rank_kernel, grd, blk, 0, J.stream, J.cj[c].st, n, n_src, ss);
            hipLaunchKernelGGL(csek::share_target_kernel, grd, blk, 0, J.stream, J.cj[c].st, n, n_src,
                               sc.comp[c].n_fmax, (uint32_t)c, cfg.seed, cfg.share_dst_pm, r, ss);
            if (hipGetLastError() != hipSuccess) { rc = fail(ctx, CSE_EHIP, "sharing launch failed"); break; }
            if (hipMemcpyAsync(h_active + c, ss.counter, sizeof(int32_t), hipMemcpyDeviceToHost, J.stream)
                != hipSuccess) { rc = fail(ctx, CSE_EHIP, "active count copy failed"); break; }
            any = true;
        }
        if (rc || !any) break;
        if (hipStreamSynchronize(J.stream) != hipSuccess) { rc = fail(ctx, CSE_EHIP, "round sync failed"); break; }
        bool more = false;
        for (int c = 0; c < J.n_comp; ++c) {
            if (live[c] && h_active[c] == 0) live[c] = false;
            more |= live[c];
        }
        if (!more) break;
    }
    (void)hipStreamSynchronize(J.stream);
    (void)hipFree(d_scratch);
    (void)hipHostFree(h_active);
    return rc;
}

// Enqueue every launch of one job on its stream.
int run_job(cse_ctx* ctx, JobRec& J, const SchemeRec& sc) {
    const cse_run_cfg& cfg = J.cfg;
    const uint32_t n = cfg.n_proc;
    for (int c = 0; c < J.n_comp; ++c) {
        hipLaunchKernelGGL(csek::init_units_kernel, dim3((n + 255) / 256), dim3(256), 0, J.stream,
                           J.cj[c].st, n, c == 0 ? 1 : 0);
        HIP_TRY(ctx, hipGetLastError());
    }
    const bool sharing = cfg.share_every > 0 && cfg.share_src_pm > 0 && cfg.share_max_rounds > 0;
    if (sharing) return run_sharing_rounds(ctx, J, sc);
    for (int c = 0; c < J.n_comp; ++c) {
        int rc = launch_step(ctx, sc.comp[c], c, cfg, -1, J.cj[c].st, J.d_err, J.stream);
        if (rc) return rc;
    }
    return CSE_OK;
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
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->lds_max = std::max<size_t>(prop.sharedMemPerBlock, 65536);
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        ctx->tick_hz = (uint64_t)khz * 1000ull;
    *out = ctx;
    return CSE_OK;
}

void cse_ctx_destroy(cse_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (auto& kv : ctx->jobs) {
        JobRec& J = kv.second;
        if (!J.finished) (void)hipEventSynchronize(J.ev_done);
        for (int c = 0; c < J.n_comp; ++c) (void)hipFree(J.cj[c].block);
        (void)hipFree(J.d_t0);
        (void)hipFree(J.d_err);
        (void)hipEventDestroy(J.ev_done);
    }
    for (auto& kv : ctx->schemes)
        for (int c = 0; c < kv.second.n_comp; ++c) free_component(kv.second.comp[c]);
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
        if (kv.second.scheme == scheme_id && !kv.second.finished) (void)wait_job(ctx, kv.second);
    for (int c = 0; c < it->second.n_comp; ++c) free_component(it->second.comp[c]);
    ctx->schemes.erase(it);
    return CSE_OK;
}

int32_t cse_launch(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, void* stream, int32_t* job_id) {
    return cse_launch_batch(ctx, &scheme_id, cfg, 1, stream, job_id);
}

int32_t cse_launch_batch(cse_ctx* ctx, const int32_t* scheme_ids, const cse_run_cfg* cfgs, int32_t n,
                         void* stream, int32_t* job_ids) {
    if (!ctx || !scheme_ids || !cfgs || !job_ids || n < 1) return CSE_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (int i = 0; i < n; ++i) {
        if (!ctx->schemes.count(scheme_ids[i])) return fail(ctx, CSE_ENOENT, "unknown scheme %d", scheme_ids[i]);
        int rc = validate_cfg(ctx, &cfgs[i]);
        if (rc) return rc;
    }
    for (int i = 0; i < n; ++i) {
        const SchemeRec& sc = ctx->schemes[scheme_ids[i]];
        JobRec J;
        J.scheme = scheme_ids[i];
        J.cfg = cfgs[i];
        J.stream = (hipStream_t)stream;
        J.n_comp = sc.n_comp;
        HIP_TRY(ctx, hipMalloc((void**)&J.d_t0, 64));
        HIP_TRY(ctx, hipMalloc((void**)&J.d_err, 64));
        HIP_TRY(ctx, hipMemsetAsync(J.d_err, 0, 64, J.stream));
        for (int c = 0; c < sc.n_comp; ++c) {
            int rc = alloc_comp_job(ctx, sc.comp[c], J.cfg.n_proc, J.d_t0, &J.cj[c]);
            if (rc) return rc;
        }
        HIP_TRY(ctx, hipEventCreateWithFlags(&J.ev_done, hipEventDisableTiming));
        int rc = run_job(ctx, J, sc);
        if (rc) return rc;
        HIP_TRY(ctx, hipEventRecord(J.ev_done, J.stream));
        const int id = ctx->next_job++;
        ctx->jobs[id] = J;
        job_ids[i] = id;
    }
    return CSE_OK;
}

int32_t cse_poll(cse_ctx* ctx, int32_t job_id, int32_t* done) {
    if (!ctx || !done) return CSE_EINVAL;
    JobRec* J = find_job(ctx, job_id);
    if (!J) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (J->finished) { *done = 1; return CSE_OK; }
    hipError_t e = hipEventQuery(J->ev_done);
    if (e == hipErrorNotReady) { *done = 0; return CSE_OK; }
    if (e != hipSuccess) return fail(ctx, CSE_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
    J->finished = true;
    *done = 1;
    return check_err(ctx, *J);
}

int32_t cse_wait(cse_ctx* ctx, int32_t job_id) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = find_job(ctx, job_id);
    if (!J) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    return wait_job(ctx, *J);
}

int32_t cse_get_unit_results(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t n, int32_t* cost,
                             int32_t* steps, int32_t* executed, int32_t* epoch, int32_t* k0, int64_t* ops,
                             int32_t* strat, uint64_t* finish) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = find_job(ctx, job_id);
    if (!J) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (comp < 0 || comp >= J->n_comp) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    if (n != (int32_t)J->cfg.n_proc) return fail(ctx, CSE_ERANGE, "n must equal n_proc (%u)", J->cfg.n_proc);
    int rc = wait_job(ctx, *J);
    if (rc) return rc;
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
    JobRec* J = find_job(ctx, job_id);
    if (!J) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (comp < 0 || comp >= J->n_comp) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    if (n != (int32_t)J->cfg.n_proc) return fail(ctx, CSE_ERANGE, "n must equal n_proc (%u)", J->cfg.n_proc);
    const DevComp& dc = ctx->schemes[J->scheme].comp[comp];
    if (cap < dc.n_fmax) return fail(ctx, CSE_ERANGE, "cap %d < n_fmax %d", cap, dc.n_fmax);
    int rc = wait_job(ctx, *J);
    if (rc) return rc;
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
    JobRec* J = find_job(ctx, job_id);
    if (!J) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    if (comp < 0 || comp >= J->n_comp) return fail(ctx, CSE_EINVAL, "component %d out of range", comp);
    const int n = (int)J->cfg.n_proc;
    if (proc < -1 || proc >= n) return fail(ctx, CSE_EINVAL, "process %d out of range", proc);
    int rc = wait_job(ctx, *J);
    if (rc) return rc;
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

int32_t cse_job_timing(cse_ctx* ctx, int32_t job_id, uint64_t* ticks, uint64_t* tick_hz) {
    if (!ctx) return CSE_EINVAL;
    JobRec* J = find_job(ctx, job_id);
    if (!J) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    int rc = wait_job(ctx, *J);
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

int32_t cse_job_release(cse_ctx* ctx, int32_t job_id) {
    if (!ctx) return CSE_EINVAL;
    auto it = ctx->jobs.find(job_id);
    if (it == ctx->jobs.end()) return fail(ctx, CSE_ENOENT, "unknown job %d", job_id);
    JobRec& J = it->second;
    if (!J.finished) (void)hipEventSynchronize(J.ev_done);
    for (int c = 0; c < J.n_comp; ++c) (void)hipFree(J.cj[c].block);
    (void)hipFree(J.d_t0);
    (void)hipFree(J.d_err);
    (void)hipEventDestroy(J.ev_done);
    ctx->jobs.erase(it);
    return CSE_OK;
}

}  // extern "C"
