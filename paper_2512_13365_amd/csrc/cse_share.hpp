// cse_share.hpp -- solution sharing between the units of one pool
// (Sec. 3.5.2, periodic variant): after every round of at most share_every
// steps, the first ceil(N src_pm / 1000) units by (current cost, process)
// become sources; every active non-source unit becomes a target with
// probability dst_pm / 1000 and restarts from the first k substitutions of
// a source it picks, k uniform in [1, max(1, floor(3 L / 4))].
//
// Ranking needs no sort: a unit's rank is the number of units whose
// (cost, process) key is smaller, and a unit is not a source once it has
// seen n_src smaller keys.  Keys are compared tile by tile from LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cse_kernels.hpp"

namespace csek {

struct ShareScratch {
    int32_t* is_src;    // n
    int32_t* src_list;  // n_src, in rank order
};

// Scratch of one pool: 2 n int32, rounded to 256 bytes.
inline size_t share_scratch_bytes(uint32_t n) { return (((size_t)n * 8) + 255) & ~size_t(255); }

inline ShareScratch share_scratch(int32_t* base, uint32_t n) {
    ShareScratch s;
    s.is_src = base;
    s.src_list = base + n;
    return s;
}

__global__ void fill_i32_kernel(int32_t* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One pool (the units of one component of one job) for the round kernels,
// which cover every pool of a batch in one launch each (grid y = pool).
struct PoolDev {
    UnitState S;
    ShareScratch sc;
    uint64_t seed;
    uint32_t n, n_src, comp, dst_pm, max_rounds, shares;
    int32_t n_fmax;
    uint32_t first_of_job;  // advances the job's round counter
    uint32_t iteration;     // the job's outer iteration (keys the draws)
};

// Active units per pool (counts[p] starts at 0).
__global__ void pools_count_kernel(const PoolDev* __restrict__ pools, int32_t* counts) {
    const PoolDev& P = pools[blockIdx.y];
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    const bool a = u < P.n && P.S.active[u] != 0;
    const int c = __popcll(__ballot(a));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&counts[blockIdx.y], c);
}

// Sources of every sharing pool below its round limit: rank by (cost,
// process), mark the first n_src and list them in rank order.  A block of
// kRankBlock units counts the smaller keys tile by tile, each tile of keys
// staged in LDS, and stops once every one of its units has seen n_src of
// them (such a unit is not a source; the others end with exact ranks).
constexpr int kRankBlock = 256;
__global__ __launch_bounds__(kRankBlock) void pools_rank_kernel(const PoolDev* __restrict__ pools) {
    __shared__ unsigned long long tile[kRankBlock];
    const PoolDev& P = pools[blockIdx.y];
    if (!P.shares || (uint32_t)*P.S.round >= P.max_rounds || blockIdx.x * kRankBlock >= P.n) return;
    const uint32_t u = blockIdx.x * kRankBlock + threadIdx.x;
    const int32_t* cost = P.S.cost;
    const bool in = u < P.n;
    const unsigned long long mine = in ? ((unsigned long long)(uint32_t)cost[u] << 32) | u : ~0ull;
    uint32_t below = 0;
    for (uint32_t t0 = 0; t0 < P.n; t0 += kRankBlock) {
        const uint32_t v = t0 + threadIdx.x;
        tile[threadIdx.x] = v < P.n ? ((unsigned long long)(uint32_t)cost[v] << 32) | v : ~0ull;
        __syncthreads();
        const int cnt = P.n - t0 < (uint32_t)kRankBlock ? (int)(P.n - t0) : kRankBlock;
        for (int i = 0; i < cnt; ++i) below += tile[i] < mine ? 1u : 0u;
        // Also the barrier before the next tile overwrites this one.
        if (__syncthreads_and(!in || below >= P.n_src)) break;
    }
    if (!in) return;
    const bool src = below < P.n_src;
    P.sc.is_src[u] = src ? 1 : 0;
    if (src) P.sc.src_list[below] = (int32_t)u;
}

// Targets of every sharing pool copy a prefix of their source's program
// (the step kernel replays it at its next launch).  Sources are never
// targets of the same event, so every copy reads a program nobody writes.
__global__ void pools_target_kernel(const PoolDev* __restrict__ pools) {
    const PoolDev& P = pools[blockIdx.y];
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (!P.shares || u >= P.n) return;
    const uint32_t round = (uint32_t)*P.S.round;
    if (round >= P.max_rounds) return;
    const UnitState& S = P.S;
    if (!S.active[u] || P.sc.is_src[u]) return;
    const U4 r = philox10(u, domain(TAG_SHARE, P.comp, P.iteration, 0), round, 0u, (uint32_t)P.seed,
                          (uint32_t)(P.seed >> 32));
    if (scale_u32(r.x, 1000u) >= P.dst_pm) return;
    const int src = P.sc.src_list[scale_u32(r.y, P.n_src)];
    const int L = S.t[src];
    if (L == 0) return;
    int kmax = (3 * L) / 4;
    if (kmax < 1) kmax = 1;
    const int k = 1 + (int)scale_u32(r.z, (uint32_t)kmax);
    const size_t nf = (size_t)(P.n_fmax > 0 ? P.n_fmax : 1);
    const uint32_t* from = S.prog + (size_t)src * nf;
    uint32_t* to = S.prog + (size_t)u * nf;
    for (int i = 0; i < k; ++i) to[i] = from[i];
    S.t[u] = k;
    S.epoch[u] += 1;
    S.k0[u] = k;
}

// Outer iterations (Sec. 3.5.1, 3.5.2).  *key becomes the minimum over the
// units of cost << 32 | process: the pool's best unit, ties to the lowest
// process (*key starts at all ones).
__global__ void driver_argmin_kernel(const int32_t* __restrict__ cost, uint32_t n, unsigned long long* key) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long k = u < n ? ((unsigned long long)(uint32_t)cost[u] << 32) | u : ~0ull;
    const unsigned long long m = ~wave_max_u64(~k);
    if ((threadIdx.x & 63) == 0) atomicMin(key, m);
}

// Restart of every unit before iteration `iteration` >= 1: Philox block
// (process, REINIT|comp|iteration|0, 0, 0); with probability reinit_pm/1000
// (word 0) the unit starts from the first k = 1 + floor(u1 max(1, floor(3 L
// / 4)) / 2^32) substitutions of the component's best program (word 1; L its
// length, L = 0: no copy), otherwise from the input.  Its epoch advances, so
// its step and coin draws are new; the step kernel replays the prefix.
__global__ void driver_reinit_kernel(UnitState S, uint32_t n, uint64_t seed, uint32_t comp, uint32_t iteration,
                                     uint32_t reinit_pm, const uint32_t* __restrict__ best, int L, int stride) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const U4 r = philox10(u, domain(TAG_REINIT, comp, iteration, 0), 0u, 0u, (uint32_t)seed,
                          (uint32_t)(seed >> 32));
    int k = 0;
    if (L > 0 && scale_u32(r.x, 1000u) < reinit_pm) {
        int kmax = (3 * L) / 4;
        if (kmax < 1) kmax = 1;
        k = 1 + (int)scale_u32(r.y, (uint32_t)kmax);
        uint32_t* to = S.prog + (size_t)u * stride;
        for (int i = 0; i < k; ++i) to[i] = best[i];
    }
    S.t[u] = k;
    S.k0[u] = k;
    S.epoch[u] += 1;
    S.active[u] = 1;
}

// End of a round: every job's round counter advances once.
__global__ void pools_round_kernel(const PoolDev* __restrict__ pools, int n_pools) {
    for (int p = threadIdx.x; p < n_pools; p += blockDim.x)
        if (pools[p].first_of_job) *pools[p].S.round += 1;
}

}  // namespace csek
