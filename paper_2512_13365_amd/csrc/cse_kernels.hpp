// cse_kernels.hpp -- gfx950 device code for randomized CSE processes
// (Perminov, arXiv 2512.13365, Algorithm 1 and Sec. 3.4-3.5).
//
// Execution model: one 64-lane wavefront (one workgroup) per unit, i.e. one
// component reduced by one process.  The unit's state lives in LDS:
//   colP[v][w], colN[v][w]  pos / neg bitsets of variable v over the rows,
//                           W 64-bit words per column (rows <= 64 W);
//   live[]                  ids of the variables with a nonzero column,
//                           ascending (fresh ids are always the largest);
//   cand[]                  the pairs occurring at least twice, in canonical
//                           order, one 64-bit entry each: key | c << 32 with
//                           key = a << 16 | b << 1 | (s < 0).
// The pair count of (a, b, +) is popc(Pa & Pb) + popc(Na & Nb) and of
// (a, b, -) popc(Pa & Nb) + popc(Na & Pb), summed over the row words.
// Every random draw is a Philox4x32-10 block of a counter that names the
// process, the component, the epoch and the step, so a unit's result does
// not depend on where or when it runs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csek {

constexpr int kWave = 64;
enum { S_G = 0, S_GA = 1, S_WR = 2, S_GR = 3, S_GI = 4, S_MIX = 5, S_GP = 6, N_STRAT = 7 };
enum { TAG_PROC = 1, TAG_STEP = 2, TAG_COIN = 3, TAG_SHARE = 4 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011).  Ten rounds; each multiplies words
// 0 and 2 by the round constants, mixes the high halves with words 1, 3 and
// the key, and the key advances by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// Counter word 1: tag[31:28] component[27:26] epoch[25:16] step[15:0].
__device__ __forceinline__ uint32_t domain(uint32_t tag, uint32_t comp, uint32_t epoch, uint32_t step) {
    return (tag << 28) | ((comp & 3u) << 26) | ((epoch & 0x3FFu) << 16) | (step & 0xFFFFu);
}

// floor(u * n / 2^32)
__device__ __forceinline__ uint32_t scale_u32(uint32_t u, uint32_t n) {
    return (uint32_t)(((uint64_t)u * n) >> 32);
}

// ---------------------------------------------------------------------------
// Wavefront helpers (64 lanes, one wave per workgroup).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int ctz64(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}
// Inclusive prefix sum across the wave.
__device__ __forceinline__ uint32_t wave_scan(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t w = __shfl_up(v, o);
        if (l >= o) v += w;
    }
    return v;
}

__device__ __forceinline__ uint32_t pair_key(int a, int b, int neg) {
    return ((uint32_t)a << 16) | ((uint32_t)b << 1) | (uint32_t)neg;
}
__device__ __forceinline__ int key_a(uint32_t k) { return (int)(k >> 16); }
__device__ __forceinline__ int key_b(uint32_t k) { return (int)((k >> 1) & 0x7FFFu); }

// ---------------------------------------------------------------------------
// Kernel arguments.
// ---------------------------------------------------------------------------
struct CompArgs {
    const uint64_t* P0;   // n_x columns of W words: positive coefficients
    const uint64_t* N0;   // negative coefficients
    int32_t n_e, n_x, n_fmax, m_cap;
    int32_t naive0;
    uint32_t comp;
    int32_t prog_stride;  // max(1, n_fmax): program entries per unit
};

struct RunArgs {
    uint64_t seed;
    uint32_t weights[N_STRAT];
    uint32_t mix_weights[4];
    uint32_t proc0_greedy, gr_p_q16, step_cap, iteration;
    int32_t budget;        // selection steps per launch; < 0 = until the unit finishes
    uint32_t n_units;
};

struct UnitState {         // per process arrays of one component
    uint32_t* prog;        // n_units x max(1, n_fmax) keys
    int32_t* t;
    int32_t* cost;
    int32_t* executed;
    int32_t* epoch;
    int32_t* k0;
    int32_t* active;
    int32_t* strat;
    unsigned long long* ops;
    unsigned long long* finish;
    const unsigned long long* t0;
};

__device__ __forceinline__ int weighted_pick(const uint32_t* w, int n, uint32_t u) {
    uint64_t total = 0;
    for (int i = 0; i < n; ++i) total += w[i];
    const uint64_t x = ((uint64_t)u * total) >> 32;
    uint64_t run = 0;
    for (int i = 0; i < n; ++i) {
        run += w[i];
        if (run > x) return i;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Substitution x_k = x_a + s x_b on the column bitsets (Algorithm 1): the
// affected rows are R = (Pa & Pb) | (Na & Nb) for s = +1 and
// (Pa & Nb) | (Na & Pb) for s = -1; x_k takes x_a's sign on R and both
// x_a and x_b leave R.  Lanes 0..W-1 handle one row word each.  Returns c
// and sets bit 0 / bit 1 of *dead when column a / b became empty.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ int substitute(uint64_t* colP, uint64_t* colN, uint32_t key, int vk, int* dead) {
    const int l = lane_id();
    const int va = key_a(key) - 1, vb = key_b(key) - 1;
    const bool neg = key & 1u;
    int c = 0;
    bool alive_a = false, alive_b = false;
    if (l < W) {
        const uint64_t Pa = colP[va * W + l], Na = colN[va * W + l];
        const uint64_t Pb = colP[vb * W + l], Nb = colN[vb * W + l];
        const uint64_t R = neg ? ((Pa & Nb) | (Na & Pb)) : ((Pa & Pb) | (Na & Nb));
        colP[vk * W + l] = Pa & R;
        colN[vk * W + l] = Na & R;
        colP[va * W + l] = Pa & ~R;
        colN[va * W + l] = Na & ~R;
        colP[vb * W + l] = Pb & ~R;
        colN[vb * W + l] = Nb & ~R;
        c = popc64(R);
        alive_a = ((Pa | Na) & ~R) != 0;
        alive_b = ((Pb | Nb) & ~R) != 0;
    }
    c = wave_sum(c);
    *dead = (ballot(alive_a) == 0 ? 1 : 0) | (ballot(alive_b) == 0 ? 2 : 0);
    __syncthreads();
    return c;
}

// Remove the variables that died and append the fresh one (the largest id),
// keeping the list ascending.  Returns the new length.
__device__ __forceinline__ int update_live(uint32_t* live, int n_live, int a, int b, int dead, int k) {
    const int l = lane_id();
    int n = n_live;
    if (dead) {
        int out = 0;
        for (int base = 0; base < n_live; base += kWave) {
            const int i = base + l;
            const uint32_t x = i < n_live ? live[i] : 0u;
            const bool keep = i < n_live && !((dead & 1) && (int)x == a) && !((dead & 2) && (int)x == b);
            const uint64_t m = ballot(keep);
            __syncthreads();
            if (keep) live[out + lanes_below(m)] = x;
            out += popc64(m);
            __syncthreads();
        }
        n = out;
    }
    if (l == 0) live[n] = (uint32_t)k;
    __syncthreads();
    return n + 1;
}

// Analysis (Algorithm 1): count every canonical pair of live variables from
// the bitsets and keep those with c >= 2, in canonical order.  Pairs are
// enumerated by (first, second) position in the ascending live list, which
// is the canonical (a, b) order; within a pair '+' precedes '-'.
template <int W>
__device__ __forceinline__ int analyse_full(const uint64_t* colP, const uint64_t* colN, const uint32_t* live,
                                            int n_live, uint64_t* cand, int m_cap, int* overflow) {
    const int l = lane_id();
    int m = 0;
    for (int i = 0; i + 1 < n_live; ++i) {
        const int a = (int)live[i];
        uint64_t Pa[W], Na[W];
#pragma unroll
        for (int w = 0; w < W; ++w) { Pa[w] = colP[(a - 1) * W + w]; Na[w] = colN[(a - 1) * W + w]; }
        for (int jb = i + 1; jb < n_live; jb += kWave) {
            const int j = jb + l;
            const bool valid = j < n_live;
            const int b = valid ? (int)live[j] : 1;
            int cp = 0, cm = 0;
            if (valid) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint64_t Pb = colP[(b - 1) * W + w], Nb = colN[(b - 1) * W + w];
                    cp += popc64(Pa[w] & Pb) + popc64(Na[w] & Nb);
                    cm += popc64(Pa[w] & Nb) + popc64(Na[w] & Pb);
                }
            }
            const bool hp = valid && cp >= 2, hm = valid && cm >= 2;
            const uint64_t bp = ballot(hp), bm = ballot(hm);
            const int pos = m + lanes_below(bp) + lanes_below(bm);
            if (hp) {
                if (pos < m_cap) cand[pos] = pair_key(a, b, 0) | ((uint64_t)cp << 32);
                else *overflow = 1;
            }
            if (hm) {
                const int q = pos + (hp ? 1 : 0);
                if (q < m_cap) cand[q] = pair_key(a, b, 1) | ((uint64_t)cm << 32);
                else *overflow = 1;
            }
            m += popc64(bp) + popc64(bm);
        }
    }
    __syncthreads();
    return m < m_cap ? m : m_cap;
}

// Greedy (Sec. 3.4.1): highest c, first in canonical order.
__device__ __forceinline__ int select_g(const uint64_t* cand, int m) {
    const int l = lane_id();
    unsigned long long best = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        if (q < m) {
            const unsigned long long key = ((cand[q] >> 32) << 32) | (0xFFFFFFFFull - (unsigned)q);
            best = key > best ? key : best;
        }
    }
    best = wave_max_u64(best);
    return (int)(0xFFFFFFFFull - (best & 0xFFFFFFFFull));
}

// Greedy-Alternative (Sec. 3.4.1): uniform among the ties of maximal c,
// numbered in canonical order; tie floor(u n_ties / 2^32) is taken.
__device__ __forceinline__ int select_ga(const uint64_t* cand, int m, uint32_t u) {
    const int l = lane_id();
    int cmax = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        if (q < m) { const int c = (int)(cand[q] >> 32); cmax = c > cmax ? c : cmax; }
    }
    cmax = wave_max(cmax);
    int ties = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        ties += popc64(ballot(q < m && (int)(cand[q] >> 32) == cmax));
    }
    uint32_t want = scale_u32(u, (uint32_t)ties);
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        const bool tie = q < m && (int)(cand[q] >> 32) == cmax;
        const uint64_t bt = ballot(tie);
        const uint32_t cnt = (uint32_t)popc64(bt);
        if (want < cnt) {
            const uint64_t hit = ballot(tie && (uint32_t)lanes_below(bt) == want);
            return base + ctz64(hit);
        }
        want -= cnt;
    }
    return -1;
}

// Weighted-Random (Sec. 3.4.1): probability proportional to c - 1; the first
// candidate whose running sum of c - 1 exceeds floor(u T / 2^32).
__device__ __forceinline__ int select_wr(const uint64_t* cand, int m, uint32_t u) {
    const int l = lane_id();
    int tot = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        tot += q < m ? (int)(cand[q] >> 32) - 1 : 0;
    }
    tot = wave_sum(tot);
    const uint32_t x = scale_u32(u, (uint32_t)tot);
    uint32_t run = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        const uint32_t w = q < m ? (uint32_t)(cand[q] >> 32) - 1u : 0u;
        const uint32_t incl = wave_scan(w);
        const uint64_t hit = ballot(q < m && run + incl > x);
        if (hit) return base + ctz64(hit);
        run += __shfl(incl, kWave - 1);
    }
    return -1;
}

// Greedy-Intersections (Sec. 3.4.2).  Lane p scores candidate p:
//   2^32 H = (c_p - 1) 2^32 + alpha_q (D_p 2^16 + beta_q X_p)
// with D_p the profit of the disjoint candidates and X_p that of the
// intersecting candidates whose coin is 1.  The j-th intersecting candidate
// of p in canonical order uses bit j mod 128 of Philox block
// (proc, COIN|comp|epoch|step, key(p), j div 128).  Every q is visited in
// canonical order (the O(m^2) form).  Ties go to the lower index.
__device__ __forceinline__ int select_gi_dense(const uint64_t* cand, int m, uint32_t aq, uint32_t bq,
                                               uint32_t k0, uint32_t k1, uint32_t proc, uint32_t dw,
                                               long long* n_int, long long* n_blk) {
    const int l = lane_id();
    long long best_h = -1;
    int best_p = 0x7FFFFFFF;
    long long my_int = 0, my_blk = 0;
    for (int base = 0; base < m; base += kWave) {
        const int p = base + l;
        const bool valid = p < m;
        const uint64_t ep = valid ? cand[p] : 0ull;
        const uint32_t kp = (uint32_t)ep;
        const int ap = key_a(kp), bp = key_b(kp);
        U4 blk = philox10(proc, dw, kp, 0u, k0, k1);
        int D = 0, X = 0, j = 0;
        for (int q = 0; q < m; ++q) {
            const uint64_t eq = cand[q];
            const uint32_t kq = (uint32_t)eq;
            const int qa = key_a(kq), qb = key_b(kq);
            const int wq = (int)(eq >> 32) - 1;
            const bool inter = (qa == ap) | (qa == bp) | (qb == ap) | (qb == bp);
            if (!inter) {
                D += wq;
            } else if (q != p) {
                if (j != 0 && (j & 127) == 0) blk = philox10(proc, dw, kp, (uint32_t)(j >> 7), k0, k1);
                const int r = j & 127;
                const uint32_t word = r < 32 ? blk.x : r < 64 ? blk.y : r < 96 ? blk.z : blk.w;
                if ((word >> (r & 31)) & 1u) X += wq;
                ++j;
            }
        }
        if (valid) {
            const long long wp = (long long)(ep >> 32) - 1;
            const long long h = (wp << 32) + (long long)aq * (((long long)D << 16) + (long long)bq * X);
            if (h > best_h) { best_h = h; best_p = p; }
            my_int += j;
            my_blk += (j + 127) >> 7;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const long long oh = __shfl_xor(best_h, o);
        const int op = __shfl_xor(best_p, o);
        if (oh > best_h || (oh == best_h && op < best_p)) { best_h = oh; best_p = op; }
    }
    *n_int = wave_sum64(my_int);
    *n_blk = wave_sum64(my_blk);
    return best_p;
}

// Algorithmic work of a step in 32-bit integer lane operations (the same
// cost model the oracle tallies): 98 per Philox block of the step draw;
// selection 2 n_int + 98 n_blk + 10 m for gi, 2 m otherwise; 10 w for the
// substitution and 24 w (n_live - 1) for recounting the three changed
// columns, w = ceil(n_e / 32).
__device__ __forceinline__ unsigned long long step_ops(int strat, int m, long long n_int, long long n_blk,
                                                       int n_e, int n_live) {
    const long long w = (n_e + 31) / 32;
    const long long sel = strat == S_GI ? (2 * n_int + 98 * n_blk + 10 * (long long)m) : 2 * (long long)m;
    return (unsigned long long)(98 + sel + 10 * w + 24 * w * (long long)(n_live - 1));
}

// ---------------------------------------------------------------------------
// The step kernel: one workgroup (one wave) per unit.  Restores the unit by
// replaying its program from the input system, then runs up to `budget`
// selection steps (Analysis -> Selection -> Substitution) or until no pair
// occurs twice / the program reaches step_cap.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kWave) void step_kernel(CompArgs C, RunArgs R, UnitState S, int* err) {
    extern __shared__ uint64_t smem[];
    const int l = lane_id();
    const uint32_t proc = blockIdx.x;
    if (proc >= R.n_units || S.active[proc] == 0) return;

    const int n_vmax = C.n_x + C.n_fmax;
    uint64_t* colP = smem;
    uint64_t* colN = colP + (size_t)n_vmax * W;
    uint64_t* cand = colN + (size_t)n_vmax * W;
    uint32_t* live = (uint32_t*)(cand + C.m_cap);

    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);

    // Process draws (Sec. 3.5.1): strategy, alpha, beta.
    const U4 pu = philox10(proc, domain(TAG_PROC, 0, R.iteration, 0), 0u, 0u, k0, k1);
    int strat;
    if (R.proc0_greedy && proc == 0 && R.iteration == 0) strat = S_G;
    else strat = weighted_pick(R.weights, N_STRAT, pu.x);
    const uint32_t alpha_q = pu.y >> 17;
    const uint32_t beta_q = 32768u + (pu.z >> 17);

    for (int i = l; i < n_vmax * W; i += kWave) {
        const bool in = i < C.n_x * W;
        colP[i] = in ? C.P0[i] : 0ull;
        colN[i] = in ? C.N0[i] : 0ull;
    }
    __syncthreads();

    int t = S.t[proc];
    const int epoch = S.epoch[proc];
    int executed = S.executed[proc];
    unsigned long long ops = S.ops[proc];
    int cost = C.naive0;
    uint32_t* prog = S.prog + (size_t)proc * C.prog_stride;

    // Replay the unit's program (a shared prefix or an earlier round).
    for (int i = 0; i < t; ++i) {
        int dead;
        const int c = substitute<W>(colP, colN, prog[i], C.n_x + i, &dead);
        cost -= c - 1;
    }

    // Live list: variables with a nonzero column, ascending.
    int n_live = 0;
    {
        const int n_v = C.n_x + t;
        for (int base = 0; base < n_v; base += kWave) {
            const int v = base + l;
            bool nz = false;
            if (v < n_v) {
#pragma unroll
                for (int w = 0; w < W; ++w) nz |= (colP[v * W + w] | colN[v * W + w]) != 0;
            }
            const uint64_t mk = ballot(nz);
            if (nz) live[n_live + lanes_below(mk)] = (uint32_t)(v + 1);
            n_live += popc64(mk);
        }
        __syncthreads();
    }

    int active = 1;
    int overflow = 0;
    for (int done = 0;; ++done) {
        const int m = analyse_full<W>(colP, colN, live, n_live, cand, C.m_cap, &overflow);
        if (m == 0 || (R.step_cap && (uint32_t)t >= R.step_cap) || t >= C.n_fmax) { active = 0; break; }
        if (R.budget >= 0 && done >= R.budget) break;

        const U4 su = philox10(proc, domain(TAG_STEP, C.comp, (uint32_t)epoch, (uint32_t)t), 0u, 0u, k0, k1);
        int s = strat;
        if (s == S_MIX) {
            const int mi = weighted_pick(R.mix_weights, 4, su.x);
            s = mi == 0 ? S_GI : mi == 1 ? S_GA : mi == 2 ? S_GR : S_WR;
        }
        if (s == S_GR) s = ((su.y >> 16) < R.gr_p_q16) ? S_GA : S_WR;

        long long n_int = 0, n_blk = 0;
        int pick;
        if (s == S_G) pick = select_g(cand, m);
        else if (s == S_GA) pick = select_ga(cand, m, su.z);
        else if (s == S_WR) pick = select_wr(cand, m, su.z);
        else pick = select_gi_dense(cand, m, alpha_q, beta_q, k0, k1, proc,
                                    domain(TAG_COIN, C.comp, (uint32_t)epoch, (uint32_t)t), &n_int, &n_blk);
        if (pick < 0 || pick >= m) { if (l == 0) atomicOr(err, 2); active = 0; break; }

        const uint64_t e = cand[pick];
        const uint32_t key = (uint32_t)e;
        const int csel = (int)(e >> 32);
        __syncthreads();
        int dead;
        const int c = substitute<W>(colP, colN, key, C.n_x + t, &dead);
        if (c != csel && l == 0) atomicOr(err, 4);
        n_live = update_live(live, n_live, key_a(key), key_b(key), dead, C.n_x + t + 1);
        if (l == 0) prog[t] = key;
        ++t;
        cost -= c - 1;
        ++executed;
        ops += step_ops(s, m, n_int, n_blk, C.n_e, n_live);
    }
    if (overflow && l == 0) atomicOr(err, 1);

    if (l == 0) {
        S.t[proc] = t;
        S.cost[proc] = cost;
        S.executed[proc] = executed;
        S.ops[proc] = ops;
        S.strat[proc] = strat;
        S.active[proc] = active;
        if (!active) S.finish[proc] = wall_clock64() - *S.t0;
    }
}

// Job start stamp and per-unit state initialisation.
__global__ void init_units_kernel(UnitState S, uint32_t n_units, int stamp) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (stamp && i == 0) *(unsigned long long*)S.t0 = wall_clock64();
    if (i >= n_units) return;
    S.t[i] = 0;
    S.cost[i] = 0;
    S.executed[i] = 0;
    S.epoch[i] = 0;
    S.k0[i] = 0;
    S.active[i] = 1;
    S.strat[i] = -1;
    S.ops[i] = 0;
    S.finish[i] = 0;
}

}  // namespace csek
