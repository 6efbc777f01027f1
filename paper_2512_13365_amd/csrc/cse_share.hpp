// cse_share.hpp -- solution sharing between the units of one pool
// (Sec. 3.5.2, periodic variant): after every round of at most share_every
// steps, the first ceil(N src_pm / 1000) units by (current cost, process)
// become sources; every active non-source unit becomes a target with
// probability dst_pm / 1000 and restarts from the first k substitutions of
// a source it picks, k uniform in [1, max(1, floor(3 L / 4))].
//
// Ranking needs no sort: a unit's rank is the number of units whose
// (cost, process) key is smaller, and a unit can stop counting as soon as it
// has seen n_src smaller keys, since it is then not a source.  Only the few
// best units scan the whole pool.
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

// Number of active units of a pool, added to *out.
__global__ void count_active_kernel(UnitState S, uint32_t n, int32_t* out) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    const bool a = u < n && S.active[u] != 0;
    const int c = __popcll(__ballot(a));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// Rank every unit by (cost, process); mark the first n_src and list them in
// rank order.
__global__ void share_rank_kernel(UnitState S, uint32_t n, uint32_t n_src, ShareScratch sc) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const unsigned long long mine = ((unsigned long long)(uint32_t)S.cost[u] << 32) | u;
    uint32_t below = 0;
    for (uint32_t v = 0; v < n && below < n_src; ++v) {
        const unsigned long long kv = ((unsigned long long)(uint32_t)S.cost[v] << 32) | v;
        below += kv < mine ? 1u : 0u;
    }
    const bool src = below < n_src;
    sc.is_src[u] = src ? 1 : 0;
    if (src) sc.src_list[below] = (int32_t)u;
}

// Targets copy a prefix of their source's program; the step kernel replays
// it at its next launch.  Sources are never targets of the same event, so
// every copy reads a program that no thread writes concurrently.
__global__ void share_target_kernel(UnitState S, uint32_t n, uint32_t n_src, int n_fmax, uint32_t comp,
                                    uint64_t seed, uint32_t dst_pm, uint32_t round, ShareScratch sc) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n || !S.active[u] || sc.is_src[u]) return;
    const U4 r = philox10(u, domain(TAG_SHARE, comp, 0, 0), round, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    if (scale_u32(r.x, 1000u) >= dst_pm) return;
    const int src = sc.src_list[scale_u32(r.y, n_src)];
    const int L = S.t[src];
    if (L == 0) return;
    int kmax = (3 * L) / 4;
    if (kmax < 1) kmax = 1;
    const int k = 1 + (int)scale_u32(r.z, (uint32_t)kmax);
    const size_t nf = (size_t)(n_fmax > 0 ? n_fmax : 1);
    const uint32_t* from = S.prog + (size_t)src * nf;
    uint32_t* to = S.prog + (size_t)u * nf;
    for (int i = 0; i < k; ++i) to[i] = from[i];
    S.t[u] = k;
    S.epoch[u] += 1;
    S.k0[u] = k;
}

}  // namespace csek
