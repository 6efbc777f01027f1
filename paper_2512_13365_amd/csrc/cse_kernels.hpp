// cse_kernels.hpp -- gfx950 device code for randomized CSE processes
// (Perminov, arXiv 2512.13365, Algorithm 1 and Sec. 3.4-3.5).
//
// Execution model: one workgroup per unit, i.e. one component reduced by one
// process: one 64-lane wavefront, or two or four for units whose gi walks
// ranges (the *_grp functions).  A launch covers a table of segments;
// a segment is a contiguous range of units that share one system and one run
// configuration, so one launch can hold the three components of a scheme or
// the components of many schemes.  The step kernel is specialised on the row
// words W, on where the unit's state lives, on the form of gi and on the
// waves per unit.  A unit's state:
//   colP[v][w], colN[v][w]  pos / neg bitsets of variable v over the rows,
//                           W 64-bit words per column (rows <= 64 W);
//   live[], vpos[]          ids of the variables with a nonzero column,
//                           ascending (fresh ids are always the largest), and
//                           the position of each live variable in that list;
//   cand[]                  the pairs occurring at least twice, in canonical
//                           order, one 64-bit entry each: key | c << 32 with
//                           key = a << 16 | b << 1 | (s < 0); units of
//                           several waves keep 32-bit entries
//                           a << 21 | b << 10 | (s < 0) << 9 | (c - 1);
//   newc[]                  the pairs of the fresh variable (update scratch);
//   M[], wt[]               per-variable candidate masks and weights (the
//                           mask form of gi; they share newc's region);
//   cand2[], tl[], tinv[], pl[], rng[], ssum[], remap[], kpre[]
//                           for large candidate sets (the range form of gi):
//                           a second candidate buffer, the second ordering
//                           (by second variable) and each candidate's place
//                           in it, weight bit-planes, per-variable ranges
//                           and profit sums, and the index map of the update.
// The lists live in LDS; the rest lives in LDS too, or, for systems whose
// state would leave fewer than four units per CU, in a per-unit slot in HBM
// (optionally with tinv, pl, rng and ssum in LDS).  A slot also records which state
// it holds, so a unit that was not restarted resumes from it at its next
// launch instead of replaying its program.
// The pair count of (a, b, +) is popc(Pa & Pb) + popc(Na & Nb) and of
// (a, b, -) popc(Pa & Nb) + popc(Na & Pb), summed over the row words.
// Every random draw is a Philox4x32-10 block of a counter that names the
// process, the component, the epoch and the step, so a unit's result does
// not depend on where or when it runs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

// Wavefront reductions and scans of the ROCm device library (DPP based).
extern "C" __device__ int __ockl_wfscan_add_i32(int, bool);
extern "C" __device__ __attribute__((const)) long long __ockl_wfred_add_i64(long long);
extern "C" __device__ __attribute__((const)) long long __ockl_wfred_max_i64(long long);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

namespace csek {

constexpr int kWave = 64;
enum { S_G = 0, S_GA = 1, S_WR = 2, S_GR = 3, S_GI = 4, S_MIX = 5, S_GP = 6, N_STRAT = 7 };
enum { TAG_PROC = 1, TAG_STEP = 2, TAG_COIN = 3, TAG_SHARE = 4, TAG_REINIT = 5 };

// Device consistency flags (host reports them as an error).
enum { ERR_CAND_OVERFLOW = 1, ERR_BAD_PICK = 2, ERR_COUNT_MISMATCH = 4, ERR_NEW_OVERFLOW = 8 };

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
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;  // one 32x32->64 multiply each
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// Counter word 1: tag[31:28] component[27:26] epoch[25:16] step[15:0].
__device__ __forceinline__ uint32_t domain(uint32_t tag, uint32_t comp, uint32_t epoch, uint32_t step) {
    return (tag << 28) | ((comp & 3u) << 26) | ((epoch & 0x3FFu) << 16) | (step & 0xFFFFu);
}
// A unit's epoch may pass the 10 bits of word 1 (restarts from sharing
// events and outer iterations add up): its higher bits go to the upper half
// of counter word 3 of the step and coin draws, whose lower half is 0 or a
// coin stream's block index (< 2^11: at most 4 x 32767 coins), so no key is
// reused.
__device__ __forceinline__ uint32_t epoch_high(uint32_t epoch) { return (epoch >> 10) << 16; }

// floor(u * n / 2^32)
__device__ __forceinline__ uint32_t scale_u32(uint32_t u, uint32_t n) {
    return (uint32_t)(((uint64_t)u * n) >> 32);
}

// ---------------------------------------------------------------------------
// Wavefront helpers (64 lanes, one wave per workgroup).  Reductions and scans
// use the device library's DPP sequences; call them in uniform control flow.
// ---------------------------------------------------------------------------
// The lane index, opaque to the compiler: otherwise it computes every
// lane-dependent constant of the step loop (masks, loop bounds, addresses)
// once before the loop and holds them all in vector registers (about 15
// per lane, which cost the one-wave kernels a wave per SIMD); recomputed
// where used, they cost an instruction or two each.
__device__ __forceinline__ int lane_id() {
    int l = (int)threadIdx.x;
    asm volatile("" : "+v"(l));
    return l;
}
// c + a * b on 24-bit operands in one instruction (the compiler turns a
// multiply by a 0/1 value into a compare and a select).
__device__ __forceinline__ int mad_u24(uint32_t a, uint32_t b, int c) {
    int r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
// A pointer known to address global memory (HBM): its accesses compile to
// global loads and stores, counted by the vector-memory counter alone,
// instead of generic ones that also wait on the LDS counter.

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int ctz64(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }
__device__ __forceinline__ int wave_sum(int v) { return __ockl_wfred_add_i32(v); }
__device__ __forceinline__ long long wave_sum64(long long v) { return __ockl_wfred_add_i64(v); }
__device__ __forceinline__ int wave_max(int v) { return __ockl_wfred_max_i32(v); }
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ long long wave_max64(long long v) { return __ockl_wfred_max_i64(v); }
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    return __ockl_wfred_max_u64(v);
}
// Inclusive prefix sum across the wave.
__device__ __forceinline__ int wave_scan(int v) { return __ockl_wfscan_add_i32(v, true); }

__device__ __forceinline__ uint32_t pair_key(int a, int b, int neg) {
    return ((uint32_t)a << 16) | ((uint32_t)b << 1) | (uint32_t)neg;
}
__device__ __forceinline__ int key_a(uint32_t k) { return (int)(k >> 16); }
__device__ __forceinline__ int key_b(uint32_t k) { return (int)((k >> 1) & 0x7FFFu); }
__device__ __forceinline__ int entry_c(uint64_t e) { return (int)((e >> 32) & 0x3FFu); }

// ---------------------------------------------------------------------------
// Kernel arguments.
// ---------------------------------------------------------------------------
struct CompArgs {
    const uint64_t* P0;    // n_x columns of W words: positive coefficients
    const uint64_t* N0;    // negative coefficients
    const uint64_t* cand0; // candidates of the input system, canonical order
    const uint32_t* tl0;   // the same ordered by (second, first, sign): indices into cand0
    int32_t n_e, n_x, n_fmax, m_cap;
    int32_t naive0, m0;    // naive count and number of candidates of the input
    uint32_t comp;
    int32_t prog_stride;   // max(1, n_fmax): program entries per unit
    int32_t newc_cap;      // capacity of the fresh-variable pair list
    int32_t m_words;       // capacity of the gi masks (64-bit words)
    int32_t adj;           // 1: gi walks per-variable ranges (large candidate sets)
    int32_t kbits;         // bit-planes per ordering: bit length of the largest c - 1
};

struct RunArgs {
    uint64_t seed;
    uint32_t weights[N_STRAT];
    uint32_t mix_weights[4];
    uint32_t proc0_greedy, gr_p_q16, step_cap, iteration;
    int32_t budget;        // selection steps per launch; < 0 = until the unit finishes
    uint32_t n_units;
    const int32_t* cancel; // host-visible flag: nonzero stops the job's units (or null)
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
    int32_t* round;        // the job's sharing-round counter (shared by its components)
    char* gs_base;         // HBM-resident unit state (large systems), else null
    unsigned long long gs_stride;  // bytes of HBM state per unit
};

// A contiguous range of grid units sharing one system and one configuration.
struct Segment {
    CompArgs C;
    RunArgs R;
    UnitState S;
    uint32_t unit_begin;   // first grid unit of the segment
    uint32_t pad;
};

// Layout of a unit's state (the host sizes launches with the same formulas).
// The bulk (bitsets, candidates, scratch) lives in LDS, or for systems too
// large for LDS in a per-unit HBM slot; live/vpos always live in LDS.
// Systems with large candidate sets (adj) keep a second candidate buffer,
// the candidates ordered by (second, first, sign), an index remap,
// per-variable ranges, the second ordering packed with weights and the
// weight bit-planes of both orderings instead of the gi masks.  m_words is
// the mask capacity in 64-bit words.
struct BulkLayout {
    size_t colP, colN, cand, cand2, newc, M, wt, tl, remap, kpre, rng, ssum, tinv, pl, bytes;
};
// Words of one bit-plane (one bit per candidate, 64-candidate granules).
__host__ __device__ inline int plane_words(int m_cap) { return 2 * ((m_cap + 63) / 64); }
// The weight bit-planes of one ordering are stored word-interleaved: the k
// planes' words for candidates 32 w .. 32 w + 31 sit together at
// pl[w * ks .. w * ks + ks - 1], ks = plane_stride(k) a multiple of four
// (the planes beyond k zero), so one 16-byte load fetches four planes.
__host__ __device__ inline int plane_stride(int k) { return (k + 3) & ~3; }
// Bit-planes needed for the weights c - 1 <= n_e - 1.
__host__ __device__ inline int weight_bits(int n_e) {
    int k = 1;
    while (k < 31 && (1 << k) <= n_e - 1) ++k;
    return k;
}
// esz: bytes per candidate entry (8, or 4 for units of several waves).
__host__ __device__ inline BulkLayout bulk_layout(int n_vmax, int W, int m_cap, int newc_cap, int m_words,
                                                  int adj, int kbits, int esz = 8) {
    BulkLayout L;
    size_t o = 0;
    L.colP = o;  o += (size_t)n_vmax * W * 8;
    L.colN = o;  o += (size_t)n_vmax * W * 8;
    L.cand = o;  o += (((size_t)m_cap * esz + 7) & ~size_t(7));
    if (!adj) {
        // The fresh-variable pairs (update) and the gi masks and weights
        // (selection) are never live at the same time: one region.
        const size_t gi = (size_t)m_words * 8 + (((size_t)m_cap * 2 + 7) & ~size_t(7));
        const size_t up = (size_t)newc_cap * 8 + (size_t)((n_vmax + 63) / 64) * 24;
        L.newc = o;
        L.M = o;
        L.wt = o + (size_t)m_words * 8;
        o += gi > up ? gi : up;
        L.cand2 = L.tl = L.remap = L.kpre = L.rng = L.ssum = L.tinv = L.pl = o;
        L.bytes = (o + 255) & ~size_t(255);
        return L;
    }
    L.M = L.wt = o;
    L.cand2 = o; o += (((size_t)m_cap * esz + 7) & ~size_t(7));
    L.newc = o;  o += (size_t)newc_cap * 8;
    L.tl = o;    o += (size_t)m_cap * 4;
    L.remap = o; o += (size_t)m_cap * 4;
    L.kpre = o;  o += ((size_t)m_cap * 4 + 8) & ~size_t(7);
    o = (o + 15) & ~size_t(15);
    L.rng = o;   o += (size_t)n_vmax * 16;
    L.ssum = o;  o += ((size_t)n_vmax * 4 + 15) & ~size_t(15);
    L.tinv = o;  o += ((size_t)m_cap * 4 + 7) & ~size_t(7);
    o = (o + 15) & ~size_t(15);
    L.pl = o;    o += (size_t)2 * plane_stride(kbits) * plane_words(m_cap) * 4;
    L.bytes = (o + 255) & ~size_t(255);
    return L;
}
// live and vpos: n_vmax int32 each.
__host__ __device__ inline size_t list_bytes(int n_vmax) { return ((size_t)n_vmax * 8 + 15) & ~size_t(15); }
// Units of several waves (HBM state, gi over ranges) keep the new-pair table
// of the candidate update after the lists: per 64 live positions, the
// ballots of the fresh variable's '+' and '-' pairs (u64 each) and the number
// of new pairs before them (i32).
__host__ __device__ inline size_t newpair_table_bytes(int n_vmax) {
    return ((size_t)((n_vmax + 63) / 64) * 24 + 15) & ~size_t(15);
}
// After that table they keep a fixed LDS budget for gi's per-step tables
// (ranges, per-variable profit sums and weight planes), used at every step
// whose tables fit it; steps whose tables do not fit use the copies in the
// HBM slot.
constexpr int kGsTableBudget = 11 * 1024;

// Units with state in HBM slots may keep the per-step tables of the range
// form of gi (ranges, places in the second ordering, weight bit-planes) in
// LDS after their lists instead of in the slot: offsets in LDS, and bytes
// of LDS in all.
struct TableLayout {
    size_t rng, ssum, tinv, pl, bytes;
};
__host__ __device__ inline TableLayout table_layout(int n_vmax, int m_cap, int kbits) {
    TableLayout T;
    size_t o = list_bytes(n_vmax) + newpair_table_bytes(n_vmax);  // HBM state with ranges: several waves
    T.rng = o;  o += (size_t)n_vmax * 16;
    T.ssum = o; o += ((size_t)n_vmax * 4 + 15) & ~size_t(15);
    T.tinv = o; o += ((size_t)m_cap * 4 + 7) & ~size_t(7);
    o = (o + 15) & ~size_t(15);
    T.pl = o;   o += (size_t)2 * plane_stride(kbits) * plane_words(m_cap) * 4;
    T.bytes = (o + 15) & ~size_t(15);
    return T;
}

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

// Pair counts of two columns: .x = c(+), .y = c(-).
template <int W>
__device__ __forceinline__ int2 pair_counts(const uint64_t* colP, const uint64_t* colN, int va, int vb) {
    int cp = 0, cm = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t Pa = colP[va * W + w], Na = colN[va * W + w];
        const uint64_t Pb = colP[vb * W + w], Nb = colN[vb * W + w];
        cp += popc64(Pa & Pb) + popc64(Na & Nb);
        cm += popc64(Pa & Nb) + popc64(Na & Pb);
    }
    return make_int2(cp, cm);
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
// keeping the list ascending and vpos in step.  Returns the new length.
__device__ __forceinline__ int update_live(uint32_t* live, int32_t* vpos, int n_live, int a, int b, int dead,
                                           int k) {
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
            if (keep) {
                const int p = out + lanes_below(m);
                live[p] = x;
                vpos[x - 1] = p;
            }
            out += popc64(m);
            __syncthreads();
        }
        n = out;
    }
    if (l == 0) {
        live[n] = (uint32_t)k;
        vpos[k - 1] = n;
    }
    __syncthreads();
    return n + 1;
}

// Full Analysis (Algorithm 1): count every canonical pair of live variables
// from the bitsets and keep those with c >= 2, in canonical order.  Pairs are
// enumerated by (first, second) position in the ascending live list, which
// is the canonical (a, b) order; within a pair '+' precedes '-'.  Used once
// per launch; later steps update the list incrementally.
template <int W>
__device__ int analyse_full(const uint64_t* colP, const uint64_t* colN, const uint32_t* live, int n_live,
                            uint64_t* cand, int m_cap, int* err_flags) {
    const int l = lane_id();
    int m = 0;
    for (int i = 0; i + 1 < n_live; ++i) {
        const int a = (int)live[i];
        for (int jb = i + 1; jb < n_live; jb += kWave) {
            const int j = jb + l;
            const bool valid = j < n_live;
            const int b = valid ? (int)live[j] : a;
            const int2 c = valid ? pair_counts<W>(colP, colN, a - 1, b - 1) : make_int2(0, 0);
            const bool hp = c.x >= 2, hm = c.y >= 2;
            const uint64_t bp = ballot(hp), bm = ballot(hm);
            const int pos = m + lanes_below(bp) + lanes_below(bm);
            if (hp) {
                if (pos < m_cap) cand[pos] = pair_key(a, b, 0) | ((uint64_t)c.x << 32);
                else *err_flags |= ERR_CAND_OVERFLOW;
            }
            if (hm) {
                const int q = pos + (hp ? 1 : 0);
                if (q < m_cap) cand[q] = pair_key(a, b, 1) | ((uint64_t)c.y << 32);
                else *err_flags |= ERR_CAND_OVERFLOW;
            }
            m += popc64(bp) + popc64(bm);
        }
    }
    __syncthreads();
    return m < m_cap ? m : m_cap;
}

// Incremental Analysis after substituting (a, b) -> k.  Only pairs touching a,
// b or k change: counts touching a or b can only fall (they are recounted
// and dropped below 2); pairs with k are new.  Pairs (x, k) sort after every
// old pair whose first variable is <= x (k is the largest id), so the new
// list is an ordered merge of the filtered old list and the new pairs.
template <int W>
__device__ int update_candidates(const uint64_t* colP, const uint64_t* colN, const uint32_t* live,
                                 const int32_t* vpos, int n_live, uint64_t* cand, int m, uint64_t* newc,
                                 int newc_cap, int m_cap, int a, int b, int k, int* err_flags) {
    const int l = lane_id();
    // Per 64 live positions: which have a new '+' / '-' pair with k, and the
    // number of new pairs before them (stored after the new pairs).
    uint64_t* nmask = newc + newc_cap;
    int32_t* nbefore = (int32_t*)(nmask + 2 * ((n_live + kWave - 1) / kWave));
    // 1. Recount the pairs touching a or b; compact in place.
    int mf = 0;
    for (int base = 0; base < m; base += kWave) {
        const int i = base + l;
        const bool valid = i < m;
        uint64_t e = valid ? cand[i] : 0ull;
        const uint32_t key = (uint32_t)e;
        const int qa = key_a(key), qb = key_b(key);
        const bool touch = valid && (qa == a || qa == b || qb == a || qb == b);
        int c = entry_c(e);
        if (touch) {
            const int2 cc = pair_counts<W>(colP, colN, qa - 1, qb - 1);
            c = (key & 1u) ? cc.y : cc.x;
            e = (uint64_t)key | ((uint64_t)c << 32);
        }
        const bool keep = valid && c >= 2;
        const uint64_t bk = ballot(keep);
        __syncthreads();
        if (keep) cand[mf + lanes_below(bk)] = e;
        mf += popc64(bk);
    }
    __syncthreads();
    // 2. Pairs of the fresh variable k (the last live entry) with every other.
    int n_new = 0;
    for (int base = 0; base < n_live - 1; base += kWave) {
        const int i = base + l;
        const bool valid = i < n_live - 1;
        const int x = valid ? (int)live[i] : k;
        const int2 c = valid ? pair_counts<W>(colP, colN, x - 1, k - 1) : make_int2(0, 0);
        const bool hp = c.x >= 2, hm = c.y >= 2;
        const uint64_t bp = ballot(hp), bm = ballot(hm);
        if (l == 0) {
            nmask[2 * (base / kWave)] = bp;
            nmask[2 * (base / kWave) + 1] = bm;
            nbefore[base / kWave] = n_new;
        }
        const int pos = n_new + lanes_below(bp) + lanes_below(bm);
        if (hp) {
            if (pos < newc_cap) newc[pos] = pair_key(x, k, 0) | ((uint64_t)c.x << 32);
            else *err_flags |= ERR_NEW_OVERFLOW;
        }
        if (hm) {
            const int q = pos + (hp ? 1 : 0);
            if (q < newc_cap) newc[q] = pair_key(x, k, 1) | ((uint64_t)c.y << 32);
            else *err_flags |= ERR_NEW_OVERFLOW;
        }
        n_new += popc64(bp) + popc64(bm);
    }
    if (n_new > newc_cap) n_new = newc_cap;
    if (mf + n_new > m_cap) { *err_flags |= ERR_CAND_OVERFLOW; n_new = m_cap - mf; }
    __syncthreads();
    if (n_new == 0) return mf;
    // 3a. Destination of each new pair: its index plus the number of old
    // pairs whose first variable is <= x (binary search).  Kept in bits 42+.
    for (int base = 0; base < n_new; base += kWave) {
        const int e = base + l;
        if (e < n_new) {
            const uint64_t v = newc[e];
            const int x = key_a((uint32_t)v);
            int lo = 0, hi = mf;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key_a((uint32_t)cand[mid]) <= x) lo = mid + 1; else hi = mid;
            }
            newc[e] = v | ((uint64_t)(e + lo) << 42);
        }
    }
    __syncthreads();
    // 3b. Move old pairs up by the number of new pairs with a smaller first
    // variable, last chunk first (destinations are increasing in the index).
    // New pairs (x, k) come from the live positions below the old pair's
    // first variable: a prefix of the step-2 ballots.
    for (int base = ((mf - 1) / kWave) * kWave; base >= 0; base -= kWave) {
        const int i = base + l;
        const bool valid = i < mf;
        const uint64_t v = valid ? cand[i] : 0ull;
        int shift = 0;
        if (valid) {
            const int pv = vpos[key_a((uint32_t)v) - 1];
            const int cw = pv / kWave;
            const uint64_t below = (1ull << (pv % kWave)) - 1ull;
            shift = nbefore[cw] + popc64(nmask[2 * cw] & below) + popc64(nmask[2 * cw + 1] & below);
        }
        __syncthreads();
        if (valid) cand[i + shift] = v;
        __syncthreads();
    }
    // 3c. Place the new pairs.
    for (int base = 0; base < n_new; base += kWave) {
        const int e = base + l;
        if (e < n_new) {
            const uint64_t v = newc[e];
            cand[(int)(v >> 42)] = v & ((1ull << 42) - 1);
        }
    }
    __syncthreads();
    return mf + n_new;
}

// Greedy (Sec. 3.4.1): highest c, first in canonical order.
__device__ __forceinline__ int select_g(const uint64_t* cand, int m) {
    const int l = lane_id();
    unsigned long long best = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        if (q < m) {
            const unsigned long long key = ((unsigned long long)entry_c(cand[q]) << 32) |
                                           (0xFFFFFFFFull - (unsigned)q);
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
        if (q < m) { const int c = entry_c(cand[q]); cmax = c > cmax ? c : cmax; }
    }
    cmax = wave_max(cmax);
    int ties = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        ties += popc64(ballot(q < m && entry_c(cand[q]) == cmax));
    }
    uint32_t want = scale_u32(u, (uint32_t)ties);
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        const bool tie = q < m && entry_c(cand[q]) == cmax;
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

// Sum of c - 1 over the candidates.
__device__ __forceinline__ int total_profit(const uint64_t* cand, int m) {
    const int l = lane_id();
    int tot = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        tot += q < m ? entry_c(cand[q]) - 1 : 0;
    }
    return wave_sum(tot);
}

// Weighted-Random (Sec. 3.4.1): probability proportional to c - 1; the first
// candidate whose running sum of c - 1 exceeds floor(u T / 2^32).
__device__ __forceinline__ int select_wr(const uint64_t* cand, int m, uint32_t u) {
    const int l = lane_id();
    const int tot = total_profit(cand, m);
    const uint32_t x = scale_u32(u, (uint32_t)tot);
    uint32_t run = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        const int w = q < m ? entry_c(cand[q]) - 1 : 0;
        const uint32_t incl = (uint32_t)wave_scan(w);
        const uint64_t hit = ballot(q < m && run + incl > x);
        if (hit) return base + ctz64(hit);
        run += (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    }
    return -1;
}

// Greedy-Intersections argmax over per-lane (score, index) with ties to the
// lower index.
__device__ __forceinline__ int gi_argmax(long long best_h, int best_p) {
    const long long hmax = wave_max64(best_h);
    return wave_min(best_h == hmax ? best_p : 0x7FFFFFFF);
}

// Incremental Analysis for large candidate sets, double-buffered: the same
// update as update_candidates, written from src into dst in one pass.  Each
// kept pair lands at (kept pairs before it) + (new pairs with a smaller first
// variable); each new pair (x, k) at its index + (kept pairs with first
// variable <= x).  remap[i] receives the new index of old pair i (-1 when
// dropped) and the new pairs' indices are kept in bits 42+ of newc, for the
// maintenance of the second ordering.  Returns the new count; *n_new_out
// receives the number of new pairs.
template <int W>
__device__ int update_candidates_db(const uint64_t* colP, const uint64_t* colN, const uint32_t* live, int n_live,
                                    const uint64_t* src, int m, uint64_t* dst, uint64_t* newc, int newc_cap,
                                    int m_cap, int32_t* remap, int32_t* kpre, int a, int b, int k, int* n_new_out,
                                    int* err_flags) {
    const int l = lane_id();
    // 1. Pairs of the fresh variable k (the last live entry), by first variable.
    int n_new = 0;
    for (int base = 0; base < n_live - 1; base += kWave) {
        const int i = base + l;
        const bool valid = i < n_live - 1;
        const int x = valid ? (int)live[i] : k;
        const int2 c = valid ? pair_counts<W>(colP, colN, x - 1, k - 1) : make_int2(0, 0);
        const bool hp = c.x >= 2, hm = c.y >= 2;
        const uint64_t bp = ballot(hp), bm = ballot(hm);
        const int pos = n_new + lanes_below(bp) + lanes_below(bm);
        if (hp) {
            if (pos < newc_cap) newc[pos] = pair_key(x, k, 0) | ((uint64_t)c.x << 32);
            else *err_flags |= ERR_NEW_OVERFLOW;
        }
        if (hm) {
            const int q = pos + (hp ? 1 : 0);
            if (q < newc_cap) newc[q] = pair_key(x, k, 1) | ((uint64_t)c.y << 32);
            else *err_flags |= ERR_NEW_OVERFLOW;
        }
        n_new += popc64(bp) + popc64(bm);
    }
    if (n_new > newc_cap) n_new = newc_cap;
    __syncthreads();
    // 2. Old pairs: recount those touching a or b, keep c >= 2, place.
    int mf = 0;
    for (int base = 0; base < m; base += kWave) {
        const int i = base + l;
        const bool valid = i < m;
        uint64_t e = valid ? src[i] : 0ull;
        const uint32_t key = (uint32_t)e;
        const int qa = key_a(key), qb = key_b(key);
        int c = entry_c(e);
        if (valid && (qa == a || qa == b || qb == a || qb == b)) {
            const int2 cc = pair_counts<W>(colP, colN, qa - 1, qb - 1);
            c = (key & 1u) ? cc.y : cc.x;
            e = (uint64_t)key | ((uint64_t)c << 32);
        }
        const bool keep = valid && c >= 2;
        const uint64_t bk = ballot(keep);
        const int kept = mf + lanes_below(bk);
        if (valid) {
            int lo = 0, hi = n_new;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key_a((uint32_t)newc[mid]) < qa) lo = mid + 1; else hi = mid;
            }
            const int dest = kept + lo;
            kpre[i] = kept;
            if (keep) {
                if (dest < m_cap) dst[dest] = e;
                else *err_flags |= ERR_CAND_OVERFLOW;
            }
            remap[i] = keep ? dest : -1;
        }
        mf += popc64(bk);
    }
    if (l == 0) kpre[m] = mf;
    if (mf + n_new > m_cap) { *err_flags |= ERR_CAND_OVERFLOW; n_new = m_cap > mf ? m_cap - mf : 0; }
    __syncthreads();
    // 3. New pairs.
    for (int base = 0; base < n_new; base += kWave) {
        const int e = base + l;
        if (e < n_new) {
            const uint64_t v = newc[e] & ((1ull << 42) - 1);
            const int x = key_a((uint32_t)v);
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key_a((uint32_t)src[mid]) <= x) lo = mid + 1; else hi = mid;
            }
            const int dest = e + kpre[lo];
            dst[dest] = v;
            newc[e] = v | ((uint64_t)dest << 42);
        }
    }
    __syncthreads();
    *n_new_out = n_new;
    return mf + n_new;
}

// The candidates ordered by (second, first, sign), as indices into the
// canonical list, after an update: kept entries keep their relative order
// (their keys did not change) and take their new indices; the new pairs
// (x, k) all have the largest second variable k and come last, by x.
__device__ void update_tl(uint32_t* tl, int m_old, const int32_t* remap, const uint64_t* newc, int n_new) {
    const int l = lane_id();
    int mt = 0;
    for (int base = 0; base < m_old; base += kWave) {
        const int i = base + l;
        const int v = i < m_old ? remap[tl[i]] : -1;
        const bool keep = v >= 0;
        const uint64_t bk = ballot(keep);
        __syncthreads();
        if (keep) tl[mt + lanes_below(bk)] = (uint32_t)v;
        mt += popc64(bk);
    }
    __syncthreads();
    for (int base = 0; base < n_new; base += kWave) {
        const int e = base + l;
        if (e < n_new) tl[mt + e] = (uint32_t)(newc[e] >> 42);
    }
    __syncthreads();
}

// Second ordering from scratch after a full Analysis: enumerate pairs by
// (second, first) position in the live list, count them again, and look up
// each kept pair's index in the canonical list.
template <int W>
__device__ void build_tl(const uint64_t* colP, const uint64_t* colN, const uint32_t* live, int n_live,
                         const uint64_t* cand, int m, uint32_t* tl) {
    const int l = lane_id();
    int mt = 0;
    for (int j = 1; j < n_live; ++j) {
        const int b = (int)live[j];
        for (int ib = 0; ib < j; ib += kWave) {
            const int i = ib + l;
            const bool valid = i < j;
            const int a = valid ? (int)live[i] : b;
            const int2 c = valid ? pair_counts<W>(colP, colN, a - 1, b - 1) : make_int2(0, 0);
            const bool hp = c.x >= 2, hm = c.y >= 2;
            const uint64_t bp = ballot(hp), bm = ballot(hm);
            const int pos = mt + lanes_below(bp) + lanes_below(bm);
            for (int sgn = 0; sgn < 2; ++sgn) {
                const bool has = sgn ? hm : hp;
                if (!has) continue;
                const uint32_t key = pair_key(a, b, sgn);
                int lo = 0, hi = m;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if ((uint32_t)cand[mid] < key) lo = mid + 1; else hi = mid;
                }
                const int q = pos + (sgn && hp ? 1 : 0);
                if (q < m) tl[q] = (uint32_t)lo;
            }
            mt += popc64(bp) + popc64(bm);
        }
    }
    __syncthreads();
}

// Per-step tables of the range form of gi, indexed by live position v:
// rng[v] = (first, end) of the canonical-list range of the pairs whose first
// variable is v, then (first, end) of the range of the second ordering
// holding the pairs whose second variable is v.  tinv[q] is the place of
// candidate q in the second ordering.  pl holds the kbits bit-planes of the
// weights c - 1 in canonical order, then those of the second ordering at
// pl + plane_stride(kbits) pw, each word-interleaved (bit i of plane k's
// word w, pl[w ks + k], is candidate 32 w + i).  Returns the number of
// planes in use: the bit length of the largest weight.
__device__ int gi_prepare(const uint64_t* cand, const uint32_t* tl, int m, const int32_t* vpos, int n_live,
                          int32_t* rng, int32_t* tinv, uint32_t* pl, int pw, int kbits) {
    const int l = lane_id();
    for (int i = l; i < 4 * n_live; i += kWave) rng[i] = 0;
    __syncthreads();
    int wmax = 0;
    for (int base = 0; base < m; base += kWave) {
        const int i = base + l;
        const bool valid = i < m;
        const uint64_t e = valid ? cand[i] : 0ull;
        const uint32_t q = valid ? tl[i] : 0u;
        const uint64_t eq = valid ? cand[q] : 0ull;
        const int w = valid ? entry_c(e) - 1 : 0;
        const int wq = valid ? entry_c(eq) - 1 : 0;
        const int a = key_a((uint32_t)e), b = key_b((uint32_t)eq);
        // Neighbours in each ordering: other lanes of the chunk, or memory at its edges.
        int pa = __shfl_up(a, 1), na = __shfl_down(a, 1);
        int pb = __shfl_up(b, 1), nb = __shfl_down(b, 1);
        if (l == 0) {
            pa = i > 0 && valid ? key_a((uint32_t)cand[i - 1]) : -1;
            pb = i > 0 && valid ? key_b((uint32_t)cand[tl[i - 1]]) : -1;
        }
        if (l == kWave - 1 || i + 1 >= m) {
            na = i + 1 < m ? key_a((uint32_t)cand[i + 1]) : -1;
            nb = i + 1 < m ? key_b((uint32_t)cand[tl[i + 1]]) : -1;
        }
        if (valid) {
            const int va = vpos[a - 1], vb = vpos[b - 1];
            if (a != pa) rng[4 * va + 0] = i;
            if (a != na) rng[4 * va + 1] = i + 1;
            if (b != pb) rng[4 * vb + 2] = i;
            if (b != nb) rng[4 * vb + 3] = i + 1;
            tinv[q] = i;
        }
        wmax = w > wmax ? w : wmax;
        const int word = 2 * (base / kWave);
        const int ks = plane_stride(kbits);
        for (int k = 0; k < ks; ++k) {
            const uint64_t bc = ballot((w >> k) & 1), bt = ballot((wq >> k) & 1);
            if (l < 2) {
                pl[(word + l) * ks + k] = (uint32_t)(l ? bc >> 32 : bc);
                pl[ks * pw + (word + l) * ks + k] = (uint32_t)(l ? bt >> 32 : bt);
            }
        }
    }
    __syncthreads();
    wmax = wave_max(wmax);
    int K = 0;
    while (K < kbits && (wmax >> K) != 0) ++K;
    return K;
}

// The coin stream of candidate p: bit j is coin j, taken from Philox block
// (proc, dw, key(p), j div 128 | eh), bit j mod 32 of its word
// (j mod 128) / 32, eh the high epoch bits.  Holds the current block and,
// once needed, the next.
struct CoinStream {
    uint32_t proc, dw, kp, eh, k0, k1;
    int cb;
    bool has_nb;
    uint32_t a0, a1, a2, a3, b0, b1, b2, b3;

    // No block is drawn until a coin is needed.
    __device__ void init(uint32_t proc_, uint32_t dw_, uint32_t kp_, uint32_t eh_, uint32_t k0_, uint32_t k1_) {
        proc = proc_; dw = dw_; kp = kp_; eh = eh_; k0 = k0_; k1 = k1_;
        cb = -1;
        has_nb = false;
        a0 = a1 = a2 = a3 = 0u;
        b0 = b1 = b2 = b3 = 0u;
    }
    __device__ void next_block() {
        if (!has_nb) {
            const U4 x = philox10(proc, dw, kp, (uint32_t)(cb + 1) | eh, k0, k1);
            b0 = x.x; b1 = x.y; b2 = x.z; b3 = x.w;
            has_nb = true;
        }
    }
    // Make block blk the held one (blk never below the held block).
    __device__ __forceinline__ void hold(int blk) {
        if (blk == cb + 1) {
            next_block();
            a0 = b0; a1 = b1; a2 = b2; a3 = b3;
        } else {
            const U4 x = philox10(proc, dw, kp, (uint32_t)blk | eh, k0, k1);
            a0 = x.x; a1 = x.y; a2 = x.z; a3 = x.w;
        }
        cb = blk;
        has_nb = false;
    }
    // Block 0 drawn now, by every lane at once (a stream's first block is
    // nearly always needed; drawn lazily it would run once per lane group
    // that reaches it).
    __device__ void first_block() {
        const U4 x = philox10(proc, dw, kp, eh, k0, k1);
        a0 = x.x; a1 = x.y; a2 = x.z; a3 = x.w;
        cb = 0;
        has_nb = false;
    }
    // Coins j .. j + n - 1 in bits 0 .. n - 1 (1 <= n <= 32; higher bits
    // unspecified).  A block is drawn only if one of these coins is in it.
    // The words are picked by selects, not branches: only a block draw
    // branches.
    __device__ uint32_t bits(int j, int n) {
        const int u = j >> 5, sh = j & 31, s = u & 3;
        if ((u >> 2) != cb) hold(u >> 2);
        if (s == 3 && sh + n > 32) next_block();
        const bool odd = (s & 1) != 0, high = (s & 2) != 0;
        const uint32_t x0 = a0, x1 = a1, x2 = a2, x3 = a3, x4 = b0;
        const uint32_t lo0 = odd ? x1 : x0, hi0 = odd ? x3 : x2, lo1 = odd ? x2 : x1, hi1 = odd ? x4 : x3;
        const uint32_t w0 = high ? hi0 : lo0, w1 = high ? hi1 : lo1;
        return __builtin_amdgcn_alignbit(w1, w0, (uint32_t)sh);
    }
};

// Bits sh .. sh + n - 1 of a word (0 <= sh <= 31, 1 <= n <= 32 - sh).
__device__ __forceinline__ uint32_t window_bits(int sh, int n) {
    return (0xFFFFFFFFu << sh) & (0xFFFFFFFFu >> (32 - sh - n));
}

// Weighted coin sum over a contiguous range [pos, end) of one ordering whose
// candidates take the consecutive coins j, j + 1, ...: I += sum of c - 1,
// X += sum of c - 1 over coin 1, 32 candidates per plane word; the planes
// are word-interleaved with stride ks, and the first ku (a multiple of
// four) are summed, four per 16-byte load.
__device__ __forceinline__ void plane_window(const uint32_t* pl, int ks, int ku, int pos, int end, int& j,
                                             CoinStream& co, int& I, int& X) {
    while (pos < end) {
        const int sh = pos & 31;
        const int n = min(32 - sh, end - pos);
        const uint32_t msk = window_bits(sh, n);
        const uint32_t cw = co.bits(j, n) << sh;
        const uint4* q = (const uint4*)(pl + (pos >> 5) * ks);
        for (int g = 0; g < ku; g += 4) {
            const uint4 v = q[g >> 2];
            const uint32_t x0 = v.x & msk, x1 = v.y & msk, x2 = v.z & msk, x3 = v.w & msk;
            I += (__popc(x0) + (__popc(x1) << 1) + (__popc(x2) << 2) + (__popc(x3) << 3)) << g;
            X += (__popc(x0 & cw) + (__popc(x1 & cw) << 1) + (__popc(x2 & cw) << 2) + (__popc(x3 & cw) << 3)) << g;
        }
        pos += n;
        j += n;
    }
}

// As plane_window, the coin-weighted sum X only.
__device__ __forceinline__ void plane_window_x(const uint32_t* pl, int ks, int pos, int end, int& j,
                                               CoinStream& co, int& X) {
    while (pos < end) {
        const int sh = pos & 31;
        const int n = min(32 - sh, end - pos);
        const uint32_t msk = window_bits(sh, n);
        const uint32_t mc = (co.bits(j, n) << sh) & msk;
        const uint4* q = (const uint4*)(pl + (pos >> 5) * ks);
        for (int g = 0; g < ks; g += 4) {
            const uint4 v = q[g >> 2];
            X += (__popc(v.x & mc) + (__popc(v.y & mc) << 1) + (__popc(v.z & mc) << 2) + (__popc(v.w & mc) << 3))
                 << g;
        }
        pos += n;
        j += n;
    }
}


// The window [pos, end) of one ordering less the gap [s0, s0 + ns) inside it
// (the scored candidate, or the pair's one or two entries): the coins run on
// over the gap, so the plane word that holds it is read once, its coin word
// spread around the gap (coins after it move up by the gap's width in that
// word), rather than as two windows with a partial word each.  Per word:
// the window's bits less the gap (msk) and its coin mask (mc).
struct GapWord {
    uint32_t msk, mc;
    int n;   // positions of the window in this word
    int nc;  // coins taken: n less the gap's positions in this word
};
__device__ __forceinline__ GapWord gap_word(int pos, int end, int s0, int ns, int j, CoinStream& co) {
    GapWord g;
    const int sh = pos & 31;
    g.n = min(32 - sh, end - pos);
    const int wb = pos - sh;  // the position of the word's bit 0
    const int gl = min(max(s0 - wb, sh), sh + g.n), gh = min(max(s0 + ns - wb, sh), sh + g.n);
    const int e = gh - gl;
    g.nc = g.n - e;
    // gl is 32 only with an empty gap (e = 0), where the shifts below (taken
    // mod 32) give no gap bits and the same coin word on both sides.
    const int gs = gl & 31;
    g.msk = window_bits(sh, g.n) & ~(((1u << e) - 1u) << gs);
    const uint32_t cc = (g.nc > 0 ? co.bits(j, g.nc) : 0u) << sh;
    const uint32_t below = (1u << gs) - 1u;
    g.mc = ((cc & below) | ((cc << e) & ~below)) & g.msk;
    return g;
}

// plane_window over [pos, end) less the gap [s0, s0 + ns).
__device__ __forceinline__ void plane_window_gap(const uint32_t* pl, int ks, int ku, int pos, int end, int s0,
                                                 int ns, int& j, CoinStream& co, int& I, int& X) {
    while (pos < end) {
        const GapWord g = gap_word(pos, end, s0, ns, j, co);
        const uint4* q = (const uint4*)(pl + (pos >> 5) * ks);
        for (int k = 0; k < ku; k += 4) {
            const uint4 v = q[k >> 2];
            const uint32_t x0 = v.x & g.msk, x1 = v.y & g.msk, x2 = v.z & g.msk, x3 = v.w & g.msk;
            I += (__popc(x0) + (__popc(x1) << 1) + (__popc(x2) << 2) + (__popc(x3) << 3)) << k;
            X += (__popc(x0 & g.mc) + (__popc(x1 & g.mc) << 1) + (__popc(x2 & g.mc) << 2) + (__popc(x3 & g.mc) << 3))
                 << k;
        }
        j += g.nc;
        pos += g.n;
    }
}

// plane_window_x over [pos, end) less the gap [s0, s0 + ns).
__device__ __forceinline__ void plane_window_x_gap(const uint32_t* pl, int ks, int pos, int end, int s0, int ns,
                                                   int& j, CoinStream& co, int& X) {
    while (pos < end) {
        const GapWord g = gap_word(pos, end, s0, ns, j, co);
        const uint4* q = (const uint4*)(pl + (pos >> 5) * ks);
        for (int k = 0; k < ks; k += 4) {
            const uint4 v = q[k >> 2];
            X += (__popc(v.x & g.mc) + (__popc(v.y & g.mc) << 1) + (__popc(v.z & g.mc) << 2) +
                  (__popc(v.w & g.mc) << 3))
                 << k;
        }
        j += g.nc;
        pos += g.n;
    }
}

// Sum of c - 1 over the candidates [pos, end) of one ordering, from its planes.
__device__ __forceinline__ int plane_sum(const uint32_t* pl, int ks, int pos, int end) {
    int I = 0;
    while (pos < end) {
        const int sh = pos & 31;
        const int n = min(32 - sh, end - pos);
        const uint32_t msk = window_bits(sh, n);
        const uint4* q = (const uint4*)(pl + (pos >> 5) * ks);
        for (int g = 0; g < ks; g += 4) {
            const uint4 v = q[g >> 2];
            I += (__popc(v.x & msk) + (__popc(v.y & msk) << 1) + (__popc(v.z & msk) << 2) +
                  (__popc(v.w & msk) << 3))
                 << g;
        }
        pos += n;
    }
    return I;
}

// Greedy-Intersections over per-variable ranges (any number of candidates).
// The intersecting candidates of p = (a, b), a < b, in coin order:
//   A_p (coins 0 .. |A_p| - 1): the candidates holding a, in canonical
//       order: the pairs (x, a), x < a (a's range of the second ordering),
//       then the pairs (a, y) (a's canonical range, which holds p and its
//       twin; p skipped);
//   B_p (the next |B_p| coins): the candidates holding b but not a: the
//       pairs (x, b), x < b, without (a, b, +-) (b's range of the second
//       ordering, where those entries sit together at tinv of the first),
//       then the pairs (b, y) (b's canonical range).
// Every part is a contiguous range (p's canonical range less p, b's range of
// the second ordering less the pair's entries) whose members take
// consecutive coins, so lane p sums them 32 candidates at a time through the
// weight bit-planes.
__device__ int select_gi_planes(const uint64_t* cand, int m, const int32_t* vpos, const int32_t* rng,
                                const int32_t* tinv, const uint32_t* pl, int pw, int kbits, int K, uint32_t aq,
                                uint32_t bq, uint32_t k0, uint32_t k1, uint32_t proc, uint32_t dw, uint32_t eh,
                                long long* n_int, long long* n_blk) {
    const int l = lane_id();
    const int T = total_profit(cand, m);
    const int ks = plane_stride(kbits), ku = plane_stride(K);
    const uint32_t* plc = pl;            // canonical order
    const uint32_t* plt = pl + ks * pw;  // second ordering
    long long best_h = -1;
    int best_p = 0x7FFFFFFF;
    int my_int = 0, my_blk = 0;
    for (int base = 0; base < m; base += kWave) {
        const int p = base + l;
        if (p < m) {
            const uint64_t ep = cand[p];
            const uint32_t kp = (uint32_t)ep;
            const int va = vpos[key_a(kp) - 1], vb = vpos[key_b(kp) - 1];
            const int4 ra = *(const int4*)(rng + 4 * va);
            const int4 rb = *(const int4*)(rng + 4 * vb);
            // The twin (a, b, other sign) is adjacent in both orderings.
            const bool tprev = p > 0 && ((uint32_t)cand[p - 1] >> 1) == (kp >> 1);
            const bool tnext = p + 1 < m && ((uint32_t)cand[p + 1] >> 1) == (kp >> 1);
            const int q_lo = tprev ? p - 1 : p;
            const int n_ab = (tprev || tnext) ? 2 : 1;
            const int t_ab = tinv[q_lo];
            int I = 0, X = 0, j = 0;
            CoinStream co;
            co.init(proc, dw, kp, eh, k0, k1);
            co.first_block();
            if ((ra.w - ra.z) + (ra.y - ra.x - 1) + (rb.w - rb.z - n_ab) + (rb.y - rb.x) > 128) co.next_block();
            plane_window(plt, ks, ku, ra.z, ra.w, j, co, I, X);
            plane_window_gap(plc, ks, ku, ra.x, ra.y, p, 1, j, co, I, X);
            plane_window_gap(plt, ks, ku, rb.z, rb.w, t_ab, n_ab, j, co, I, X);
            plane_window(plc, ks, ku, rb.x, rb.y, j, co, I, X);
            const long long wp = (long long)entry_c(ep) - 1;
            const long long D = (long long)T - wp - I;
            const long long hsc = (wp << 32) + (long long)aq * ((D << 16) + (long long)bq * X);
            if (hsc > best_h) { best_h = hsc; best_p = p; }
            my_int += j;
            my_blk += (j + 127) >> 7;
        }
    }
    *n_int = wave_sum(my_int);
    *n_blk = wave_sum(my_blk);
    return gi_argmax(best_h, best_p);
}

// Greedy-Intersections (Sec. 3.4.2).  Lane p scores candidate p:
//   2^32 H = (c_p - 1) 2^32 + alpha_q (D_p 2^16 + beta_q X_p)
// with D_p the profit of the disjoint candidates and X_p that of the
// intersecting candidates whose coin is 1.  The intersecting candidates of
// p = (a, b) form two lists in canonical order, A_p holding a (p's twin
// included) and B_p holding b but not a; the i-th member of A_p then B_p
// (i = 0 .. |A_p| + |B_p| - 1) uses bit i mod 128 of Philox block
// (proc, COIN|comp|epoch|step, key(p), i div 128 | eh), eh the high epoch
// bits.  This form visits every q (the O(m^2) scan, after a count of A_p);
// it serves when the masks of the sparse form do not fit.
__device__ int select_gi_dense(const uint64_t* cand, int m, uint32_t aq, uint32_t bq, uint32_t k0, uint32_t k1,
                               uint32_t proc, uint32_t dw, uint32_t eh, long long* n_int, long long* n_blk) {
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
        // |A_p| first: B_p's coins follow A_p's in the one stream.
        int na = 0;
        for (int q = 0; q < m; ++q) {
            const uint32_t kq = (uint32_t)cand[q];
            na += q != p && (key_a(kq) == ap || key_b(kq) == ap);
        }
        U4 ba = {0u, 0u, 0u, 0u}, bb = {0u, 0u, 0u, 0u};
        int cur_a = -1, cur_b = -1;  // blocks held for A_p's and B_p's coins
        int D = 0, X = 0, ja = 0, jb = 0;
        for (int q = 0; q < m; ++q) {
            const uint64_t eq = cand[q];
            const uint32_t kq = (uint32_t)eq;
            const int qa = key_a(kq), qb = key_b(kq);
            const int wq = entry_c(eq) - 1;
            const bool sa = (qa == ap) | (qb == ap);
            const bool sb = (qa == bp) | (qb == bp);
            if (!sa && !sb) {
                D += wq;
            } else if (q != p) {
                int j;
                U4 blk;
                if (sa) {
                    j = ja++;
                    if ((j >> 7) != cur_a) {
                        ba = philox10(proc, dw, kp, (uint32_t)(j >> 7) | eh, k0, k1);
                        cur_a = j >> 7;
                    }
                    blk = ba;
                } else {
                    j = na + jb++;
                    if ((j >> 7) != cur_b) {
                        bb = philox10(proc, dw, kp, (uint32_t)(j >> 7) | eh, k0, k1);
                        cur_b = j >> 7;
                    }
                    blk = bb;
                }
                const int r = j & 127;
                const uint32_t word = r < 32 ? blk.x : r < 64 ? blk.y : r < 96 ? blk.z : blk.w;
                if ((word >> (r & 31)) & 1u) X += wq;
            }
        }
        if (valid) {
            const long long wp = (long long)entry_c(ep) - 1;
            const long long h = (wp << 32) + (long long)aq * (((long long)D << 16) + (long long)bq * X);
            if (h > best_h) { best_h = h; best_p = p; }
            my_int += ja + jb;
            my_blk += (ja + jb + 127) >> 7;
        }
    }
    *n_int = wave_sum64(my_int);
    *n_blk = wave_sum64(my_blk);
    return gi_argmax(best_h, best_p);
}

// Greedy-Intersections, sparse form: M[v] marks (bit i of 32-bit word w)
// the candidates 32 w + i that contain the live variable at position v.
// Lane p walks the set bits of M[a] (minus p itself), then those of
// M[b] & ~M[a], in increasing index: the two lists of the other forms
// (candidates holding a, twin included; those holding b only), A_p's
// members taking coins 0 .. |A_p| - 1 and B_p's the next ones, the members
// of a word the next window of coins.
// D_p = T - (c_p - 1) - I_p with I_p the profit of all intersecting
// candidates.  wt[q] = c_q - 1 is filled on the way.
__device__ __forceinline__ void mask_walk(const uint32_t* Ma, const uint32_t* Mb, int nw, int self_w,
                                          uint32_t self_bit, const uint16_t* wt, CoinStream& co, int& I, int& X,
                                          int& j) {
    for (int w = 0; w < nw; ++w) {
        uint32_t u = Ma[w] & (w == self_w ? ~self_bit : 0xFFFFFFFFu);
        if (Mb) u = Mb[w] & ~Ma[w];
        if (u == 0) continue;
        const int nm = __popc(u);
        uint32_t cw = co.bits(j, nm);
        j += nm;
        const uint16_t* wrow = wt + (w << 5);
        // The next member's weight is read before this one is summed, so the
        // LDS latency overlaps the arithmetic (the last read repeats a
        // member's own weight and is unused).
        int bit = __builtin_ctz(u);
        u &= u - 1u;
        uint32_t wq = wrow[bit];
        while (true) {
            const bool more = u != 0u;
            bit = more ? __builtin_ctz(u) : bit;
            const uint32_t wn = wrow[bit];
            u &= u - 1u;
            I += (int)wq;
            X = mad_u24(cw & 1u, wq, X);
            cw >>= 1;
            if (!more) break;
            wq = wn;
        }
    }
}

__device__ int select_gi_sparse(const uint64_t* cand, int m, const int32_t* vpos, int n_live, uint64_t* M64,
                                uint16_t* wt, uint32_t aq, uint32_t bq, uint32_t k0, uint32_t k1, uint32_t proc,
                                uint32_t dw, uint32_t eh, long long* n_int, long long* n_blk) {
    const int l = lane_id();
    const int nw = (m + 31) >> 5;
    uint32_t* M = (uint32_t*)M64;
    for (int i = l; i < n_live * nw; i += kWave) M[i] = 0u;
    __syncthreads();
    int tsum = 0;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        if (q < m) {
            const uint64_t e = cand[q];
            const uint32_t key = (uint32_t)e;
            const int w = entry_c(e) - 1;
            wt[q] = (uint16_t)w;
            tsum += w;
            const uint32_t bit = 1u << (q & 31);
            atomicOr(&M[vpos[key_a(key) - 1] * nw + (q >> 5)], bit);
            atomicOr(&M[vpos[key_b(key) - 1] * nw + (q >> 5)], bit);
        }
    }
    const int T = wave_sum(tsum);
    __syncthreads();
    long long best_h = -1;
    int best_p = 0x7FFFFFFF;
    int my_int = 0, my_blk = 0;
    for (int base = 0; base < m; base += kWave) {
        const int p = base + l;
        const bool valid = p < m;
        const uint64_t ep = valid ? cand[p] : 0ull;
        const uint32_t kp = (uint32_t)ep;
        if (valid) {
            const uint32_t* Ma = M + vpos[key_a(kp) - 1] * nw;
            const uint32_t* Mb = M + vpos[key_b(kp) - 1] * nw;
            const int self_w = p >> 5;
            const uint32_t self_bit = 1u << (p & 31);
            // One coin stream: A_p's members take coins 0 .. |A_p| - 1, B_p's the next ones.
            int I = 0, X = 0, j = 0;
            CoinStream co;
            co.init(proc, dw, kp, eh, k0, k1);
            co.first_block();
            mask_walk(Ma, nullptr, nw, self_w, self_bit, wt, co, I, X, j);
            mask_walk(Ma, Mb, nw, self_w, self_bit, wt, co, I, X, j);
            const long long wp = (long long)entry_c(ep) - 1;
            const long long D = (long long)T - wp - I;
            const long long hsc = (wp << 32) + (long long)aq * ((D << 16) + (long long)bq * X);
            if (hsc > best_h) { best_h = hsc; best_p = p; }
            my_int += j;
            my_blk += (j + 127) >> 7;
        }
    }
    *n_int = wave_sum(my_int);
    *n_blk = wave_sum(my_blk);
    return gi_argmax(best_h, best_p);
}

// Greedy-Potential (Sec. 2 and 3.4, potential as new pairs): for each candidate
// (a, b, s), the column the fresh variable would get (rows of a and b with
// relative sign s, carrying a's sign) is counted against every other live
// column; N_new is the number of its pairs (x, +/-) with count >= 2.  The
// score 2^16 (c - 1) + alpha_q N_new is maximal, ties to the first candidate.
// One lane per candidate holds the trial column in registers; the loop over
// the live list is uniform across the wave, so each column word is one
// broadcast read.  A column's pos and neg sets are disjoint, so each sign
// pair's count is one popcount of a union.  The columns of a and b lose
// exactly the rewritten rows, so they share none with the fresh column and
// are skipped.  *n_cols receives m (n_live - 2), the columns counted.
template <int W>
__device__ int select_gp(const uint64_t* cand, int m, const uint64_t* colP, const uint64_t* colN,
                         const uint32_t* live, int n_live, uint32_t alpha_q, long long* n_cols) {
    const int l = lane_id();
    long long best_h = -1;
    int best_p = 0x7FFFFFFF;
    for (int base = 0; base < m; base += kWave) {
        const int q = base + l;
        const uint64_t e = cand[q < m ? q : 0];
        const uint32_t key = (uint32_t)e;
        const int a = key_a(key), b = key_b(key);
        const bool neg = key & 1u;
        uint64_t Pk[W], Nk[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t Pa = colP[(a - 1) * W + w], Na = colN[(a - 1) * W + w];
            const uint64_t Pb = colP[(b - 1) * W + w], Nb = colN[(b - 1) * W + w];
            const uint64_t R = neg ? ((Pa & Nb) | (Na & Pb)) : ((Pa & Pb) | (Na & Nb));
            Pk[w] = Pa & R;
            Nk[w] = Na & R;
        }
        int n_new = 0;
        for (int i = 0; i < n_live; ++i) {
            const int x = (int)live[i];
            int same = 0, opp = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t Px = colP[(x - 1) * W + w], Nx = colN[(x - 1) * W + w];
                same += popc64((Px & Pk[w]) | (Nx & Nk[w]));
                opp += popc64((Px & Nk[w]) | (Nx & Pk[w]));
            }
            n_new += (x == a || x == b) ? 0 : (same >= 2) + (opp >= 2);
        }
        if (q < m) {
            const long long h = ((long long)(entry_c(e) - 1) << 16) + (long long)alpha_q * n_new;
            if (h > best_h) {
                best_h = h;
                best_p = q;
            }
        }
    }
    *n_cols = (long long)m * (n_live > 2 ? n_live - 2 : 0);
    return gi_argmax(best_h, best_p);
}

// ---------------------------------------------------------------------------
// Units of NW > 1 waves (one workgroup of 64 NW lanes per unit).  Systems
// whose state lives in HBM slots have thousands of candidates; spreading a
// unit's loops over several waves puts that many more independent memory
// accesses in flight per unit (their steps wait on memory) and shortens the
// rounds that only the largest units still run.  Every loop strides over 64
// NW entries; wave results meet in small shared arrays: a wave's ballot count
// becomes its offset among the waves (compaction), wave reductions become
// group reductions.  Values that steer control flow (counts, picks) are the
// same in every wave, so the waves take the same branches and barriers.
// The single-wave kernels keep the functions above.
// ---------------------------------------------------------------------------
// Candidates of units of several waves are 32-bit entries: first variable
// (11 bits), second variable (11), sign (1) and c - 1 (9), so the canonical
// order is the order of the entries' upper 23 bits.  Their systems have at
// most 2047 variables (c <= 512 rows always fits).
constexpr int kCompactMaxVars = 2047;
__device__ __forceinline__ uint32_t ce_make(int a, int b, int neg, int c) {
    return (uint32_t)a << 21 | (uint32_t)b << 10 | (uint32_t)neg << 9 | (uint32_t)(c - 1);
}
__device__ __forceinline__ int ce_a(uint32_t e) { return (int)(e >> 21); }
__device__ __forceinline__ int ce_b(uint32_t e) { return (int)((e >> 10) & 0x7FFu); }
__device__ __forceinline__ int ce_neg(uint32_t e) { return (int)((e >> 9) & 1u); }
__device__ __forceinline__ int ce_w(uint32_t e) { return (int)(e & 0x1FFu); }  // c - 1
__device__ __forceinline__ int ce_c(uint32_t e) { return ce_w(e) + 1; }
__device__ __forceinline__ uint32_t ce_pair(uint32_t e) { return e >> 10; }   // (a, b) without the sign
__device__ __forceinline__ uint32_t ce_order(uint32_t e) { return e >> 9; }   // a << 12 | b << 1 | sign
// The canonical 32-bit key (programs, random draws).
__device__ __forceinline__ uint32_t ce_key(uint32_t e) { return pair_key(ce_a(e), ce_b(e), ce_neg(e)); }
__device__ __forceinline__ uint32_t ce_from64(uint64_t e) {
    const uint32_t k = (uint32_t)e;
    return ce_make(key_a(k), key_b(k), (int)(k & 1u), entry_c(e));
}

// A value every lane of the wave holds, marked so for the compiler (kept in
// a scalar register; loop bounds and branches on it stay scalar).
template <class T>
__device__ __forceinline__ T wave_uniform(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_readfirstlane((uint32_t)v);
    } else {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

__device__ __forceinline__ int grp_tid() { return lane_id(); }
__device__ __forceinline__ int grp_lane() { return lane_id() & 63; }
__device__ __forceinline__ int grp_wave() { return wave_uniform((int)(threadIdx.x >> 6)); }

// Every wave passes one wave-uniform value; all receive the NW values.
template <int NW, class T>
__device__ __forceinline__ void grp_exchange(T v, T (&all)[NW]) {
    __shared__ T slot[NW];
    if (grp_lane() == 0) slot[grp_wave()] = v;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) all[w] = wave_uniform(slot[w]);
    __syncthreads();
}
// Offset of this wave's wave-uniform count among the waves (lower waves
// first); *total receives the sum.
template <int NW>
__device__ __forceinline__ int grp_offset(int count, int* total) {
    int all[NW];
    grp_exchange<NW>(count, all);
    int off = 0, tot = 0;
    const int me = grp_wave();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        off += w < me ? all[w] : 0;
        tot += all[w];
    }
    *total = tot;
    return off;
}
template <int NW>
__device__ __forceinline__ int grp_sum(int v) {
    int all[NW];
    grp_exchange<NW>(wave_sum(v), all);
    int s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += all[w];
    return s;
}
template <int NW>
__device__ __forceinline__ int grp_max(int v) {
    int all[NW];
    grp_exchange<NW>(wave_max(v), all);
    int s = all[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = all[w] > s ? all[w] : s;
    return s;
}
template <int NW>
__device__ __forceinline__ int grp_min(int v) {
    int all[NW];
    grp_exchange<NW>(wave_min(v), all);
    int s = all[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = all[w] < s ? all[w] : s;
    return s;
}
template <int NW>
__device__ __forceinline__ long long grp_max64(long long v) {
    long long all[NW];
    grp_exchange<NW>(wave_max64(v), all);
    long long s = all[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = all[w] > s ? all[w] : s;
    return s;
}
template <int NW>
__device__ __forceinline__ unsigned long long grp_max_u64(unsigned long long v) {
    unsigned long long all[NW];
    grp_exchange<NW>(wave_max_u64(v), all);
    unsigned long long s = all[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = all[w] > s ? all[w] : s;
    return s;
}
template <int NW>
__device__ __forceinline__ unsigned grp_or(unsigned v) {
    unsigned all[NW];
    grp_exchange<NW>(__ockl_wfred_or_u32(v), all);
    unsigned s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s |= all[w];
    return s;
}

// Substitution (as substitute): every wave reads the two columns and
// computes c and the dead flags; after a barrier wave 0 writes.
template <int W, int NW>
__device__ __forceinline__ int substitute_grp(uint64_t* colP, uint64_t* colN, uint32_t key, int vk, int* dead) {
    const int l = grp_lane();
    const int va = key_a(key) - 1, vb = key_b(key) - 1;
    const bool neg = key & 1u;
    int c = 0;
    bool alive_a = false, alive_b = false;
    uint64_t Pa = 0, Na = 0, Pb = 0, Nb = 0, R = 0;
    if (l < W) {
        Pa = colP[va * W + l];
        Na = colN[va * W + l];
        Pb = colP[vb * W + l];
        Nb = colN[vb * W + l];
        R = neg ? ((Pa & Nb) | (Na & Pb)) : ((Pa & Pb) | (Na & Nb));
        c = popc64(R);
        alive_a = ((Pa | Na) & ~R) != 0;
        alive_b = ((Pb | Nb) & ~R) != 0;
    }
    c = wave_sum(c);
    *dead = (ballot(alive_a) == 0 ? 1 : 0) | (ballot(alive_b) == 0 ? 2 : 0);
    __syncthreads();
    if (l < W && grp_wave() == 0) {
        colP[vk * W + l] = Pa & R;
        colN[vk * W + l] = Na & R;
        colP[va * W + l] = Pa & ~R;
        colN[va * W + l] = Na & ~R;
        colP[vb * W + l] = Pb & ~R;
        colN[vb * W + l] = Nb & ~R;
    }
    __syncthreads();
    return c;
}

template <int NW>
__device__ __forceinline__ int update_live_grp(uint32_t* live, int32_t* vpos, int n_live, int a, int b, int dead,
                                               int k) {
    const int t = grp_tid();
    int n = n_live;
    if (dead) {
        int out = 0;
        for (int base = 0; base < n_live; base += kWave * NW) {
            const int i = base + t;
            const uint32_t x = i < n_live ? live[i] : 0u;
            const bool keep = i < n_live && !((dead & 1) && (int)x == a) && !((dead & 2) && (int)x == b);
            const uint64_t m = ballot(keep);
            int tot;
            const int off = grp_offset<NW>(popc64(m), &tot);
            if (keep) {
                const int p = out + off + lanes_below(m);
                live[p] = x;
                vpos[x - 1] = p;
            }
            out += tot;
            __syncthreads();
        }
        n = out;
    }
    if (t == 0) {
        live[n] = (uint32_t)k;
        vpos[k - 1] = n;
    }
    __syncthreads();
    return n + 1;
}

// Live list of the first n_v variables from their columns (ascending).
template <int W, int NW>
__device__ __forceinline__ int build_live_grp(const uint64_t* colP, const uint64_t* colN, int n_v, uint32_t* live,
                                              int32_t* vpos) {
    int n_live = 0;
    for (int b0 = 0; b0 < n_v; b0 += kWave * NW) {
        const int v = b0 + grp_tid();
        bool nz = false;
        if (v < n_v) {
#pragma unroll
            for (int w = 0; w < W; ++w) nz |= (colP[v * W + w] | colN[v * W + w]) != 0;
        }
        const uint64_t mk = ballot(nz);
        int tot;
        const int off = grp_offset<NW>(popc64(mk), &tot);
        if (nz) {
            const int p = n_live + off + lanes_below(mk);
            live[p] = (uint32_t)(v + 1);
            vpos[v] = p;
        }
        n_live += tot;
    }
    __syncthreads();
    return n_live;
}

template <int W, int NW>
__device__ int analyse_full_grp(const uint64_t* colP, const uint64_t* colN, const uint32_t* live, int n_live,
                                uint32_t* cand, int m_cap, int* err_flags) {
    const int t = grp_tid();
    int m = 0;
    for (int i = 0; i + 1 < n_live; ++i) {
        const int a = (int)live[i];
        for (int jb = i + 1; jb < n_live; jb += kWave * NW) {
            const int j = jb + t;
            const bool valid = j < n_live;
            const int b = valid ? (int)live[j] : a;
            const int2 c = valid ? pair_counts<W>(colP, colN, a - 1, b - 1) : make_int2(0, 0);
            const bool hp = c.x >= 2, hm = c.y >= 2;
            const uint64_t bp = ballot(hp), bm = ballot(hm);
            int tot;
            const int off = grp_offset<NW>(popc64(bp) + popc64(bm), &tot);
            const int pos = m + off + lanes_below(bp) + lanes_below(bm);
            if (hp) {
                if (pos < m_cap) cand[pos] = ce_make(a, b, 0, c.x);
                else *err_flags |= ERR_CAND_OVERFLOW;
            }
            if (hm) {
                const int q = pos + (hp ? 1 : 0);
                if (q < m_cap) cand[q] = ce_make(a, b, 1, c.y);
                else *err_flags |= ERR_CAND_OVERFLOW;
            }
            m += tot;
        }
    }
    __syncthreads();
    return m < m_cap ? m : m_cap;
}

template <int W, int NW>
__device__ int update_candidates_db_grp(const uint64_t* colP, const uint64_t* colN, const uint32_t* live, int n_live,
                                        const uint32_t* src, int m, uint32_t* dst, uint64_t* newc, int newc_cap,
                                        int m_cap, int32_t* remap, int32_t* kpre, const int32_t* vpos,
                                        uint64_t* npm, int32_t* npb, int a, int b, int k, int* n_new_out,
                                        int* err_flags) {
    const int t = grp_tid();
    int n_new = 0;
    for (int base = 0; base < n_live - 1; base += kWave * NW) {
        const int i = base + t;
        const bool valid = i < n_live - 1;
        const int x = valid ? (int)live[i] : k;
        const int2 c = valid ? pair_counts<W>(colP, colN, x - 1, k - 1) : make_int2(0, 0);
        const bool hp = c.x >= 2, hm = c.y >= 2;
        const uint64_t bp = ballot(hp), bm = ballot(hm);
        int tot;
        const int off = grp_offset<NW>(popc64(bp) + popc64(bm), &tot);
        const int pos = n_new + off + lanes_below(bp) + lanes_below(bm);
        if (hp) {
            if (pos < newc_cap) newc[pos] = pair_key(x, k, 0) | ((uint64_t)c.x << 32);
            else *err_flags |= ERR_NEW_OVERFLOW;
        }
        if (hm) {
            const int q = pos + (hp ? 1 : 0);
            if (q < newc_cap) newc[q] = pair_key(x, k, 1) | ((uint64_t)c.y << 32);
            else *err_flags |= ERR_NEW_OVERFLOW;
        }
        // This wave's 64 live positions: which have new pairs, and how many
        // new pairs come before them.
        const int cb = base + kWave * grp_wave();
        if (grp_lane() == 0 && cb < n_live - 1) {
            npm[2 * (cb / kWave)] = bp;
            npm[2 * (cb / kWave) + 1] = bm;
            npb[cb / kWave] = n_new + off;
        }
        n_new += tot;
    }
    if (n_new > newc_cap) n_new = newc_cap;
    __syncthreads();
    int mf = 0;
    for (int base = 0; base < m; base += kWave * NW) {
        const int i = base + t;
        const bool valid = i < m;
        uint32_t e = valid ? src[i] : 0u;
        const int qa = ce_a(e), qb = ce_b(e);
        int c = valid ? ce_c(e) : 0;
        if (valid && (qa == a || qa == b || qb == a || qb == b)) {
            const int2 cc = pair_counts<W>(colP, colN, qa - 1, qb - 1);
            c = ce_neg(e) ? cc.y : cc.x;
            if (c >= 2) e = ce_make(qa, qb, ce_neg(e), c);
        }
        const bool keep = valid && c >= 2;
        const uint64_t bk = ballot(keep);
        int tot;
        const int off = grp_offset<NW>(popc64(bk), &tot);
        const int kept = mf + off + lanes_below(bk);
        if (valid) {
            // New pairs (x, k) with x < qa: those from the live positions
            // below qa's (a kept pair's first variable is live).
            int lo = 0;
            if (keep) {
                const int pv = vpos[qa - 1];
                const int cw = pv / kWave;
                const uint64_t below = (1ull << (pv % kWave)) - 1ull;
                lo = npb[cw] + popc64(npm[2 * cw] & below) + popc64(npm[2 * cw + 1] & below);
            }
            const int dest = kept + lo;
            kpre[i] = kept;
            if (keep) {
                if (dest < m_cap) dst[dest] = e;
                else *err_flags |= ERR_CAND_OVERFLOW;
            }
            remap[i] = keep ? dest : -1;
        }
        mf += tot;
    }
    if (t == 0) kpre[m] = mf;
    if (mf + n_new > m_cap) { *err_flags |= ERR_CAND_OVERFLOW; n_new = m_cap > mf ? m_cap - mf : 0; }
    __syncthreads();
    for (int base = 0; base < n_new; base += kWave * NW) {
        const int e = base + t;
        if (e < n_new) {
            const uint64_t v = newc[e] & ((1ull << 42) - 1);
            const int x = key_a((uint32_t)v);
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ce_a(src[mid]) <= x) lo = mid + 1; else hi = mid;
            }
            const int dest = e + kpre[lo];
            dst[dest] = ce_from64(v);
            newc[e] = v | ((uint64_t)dest << 42);
        }
    }
    __syncthreads();
    *n_new_out = n_new;
    return mf + n_new;
}

template <int NW>
__device__ void update_tl_grp(uint32_t* tl, int m_old, const int32_t* remap, const uint64_t* newc, int n_new) {
    const int t = grp_tid();
    int mt = 0;
    for (int base = 0; base < m_old; base += kWave * NW) {
        const int i = base + t;
        const int v = i < m_old ? remap[tl[i]] : -1;
        const bool keep = v >= 0;
        const uint64_t bk = ballot(keep);
        int tot;
        const int off = grp_offset<NW>(popc64(bk), &tot);
        if (keep) tl[mt + off + lanes_below(bk)] = (uint32_t)v;
        mt += tot;
    }
    __syncthreads();
    for (int base = 0; base < n_new; base += kWave * NW) {
        const int e = base + t;
        if (e < n_new) tl[mt + e] = (uint32_t)(newc[e] >> 42);
    }
    __syncthreads();
}

template <int W, int NW>
__device__ __forceinline__ void build_tl_grp(const uint64_t* colP, const uint64_t* colN, const uint32_t* live, int n_live,
                             const uint32_t* cand, int m, uint32_t* tl) {
    const int t = grp_tid();
    int mt = 0;
    for (int j = 1; j < n_live; ++j) {
        const int b = (int)live[j];
        for (int ib = 0; ib < j; ib += kWave * NW) {
            const int i = ib + t;
            const bool valid = i < j;
            const int a = valid ? (int)live[i] : b;
            const int2 c = valid ? pair_counts<W>(colP, colN, a - 1, b - 1) : make_int2(0, 0);
            const bool hp = c.x >= 2, hm = c.y >= 2;
            const uint64_t bp = ballot(hp), bm = ballot(hm);
            int tot;
            const int off = grp_offset<NW>(popc64(bp) + popc64(bm), &tot);
            const int pos = mt + off + lanes_below(bp) + lanes_below(bm);
            for (int sgn = 0; sgn < 2; ++sgn) {
                const bool has = sgn ? hm : hp;
                if (!has) continue;
                const uint32_t key = (uint32_t)a << 12 | (uint32_t)b << 1 | (uint32_t)sgn;
                int lo = 0, hi = m;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (ce_order(cand[mid]) < key) lo = mid + 1; else hi = mid;
                }
                const int q = pos + (sgn && hp ? 1 : 0);
                if (q < m) tl[q] = (uint32_t)lo;
            }
            mt += tot;
        }
    }
    __syncthreads();
}

// Total profit T = sum (c - 1) over the candidates and the number K of
// weight bit-planes (bit length of the largest c - 1, at most kbits).
template <int NW>
__device__ __forceinline__ void gi_totals_grp(const uint32_t* cand, int m, int kbits, int* T, int* K) {
    int tot = 0, wmax = 0;
    for (int q = grp_tid(); q < m; q += kWave * NW) {
        const int w = ce_w(cand[q]);
        tot += w;
        wmax = w > wmax ? w : wmax;
    }
    *T = grp_sum<NW>(tot);
    wmax = grp_max<NW>(wmax);
    int k = 0;
    while (k < kbits && (wmax >> k) != 0) ++k;
    *K = k;
}

// As gi_prepare, with the K planes of each ordering, word-interleaved with
// stride plane_stride(K) (the canonical ordering's at pl, the second
// ordering's at pl + plane_stride(K) pw), and tinv[q] the place in the
// second ordering of the first entry of q's pair (a, b), bit 31 set when
// the pair is there with both signs: all the twin test of the scoring
// loop needs.
template <int NW>
__device__ __forceinline__ void gi_prepare_grp(const uint32_t* cand, const uint32_t* tl, int m,
                                               const int32_t* vpos, int n_live, int32_t* rng, int32_t* ssum,
                                               int32_t* tinv, uint32_t* pl, int pw, int K) {
    const int l = grp_lane();
    for (int i = grp_tid(); i < 4 * n_live; i += kWave * NW) rng[i] = 0;
    __syncthreads();
    const int ks = plane_stride(K);
    // One chunk of 64 candidates of the canonical list (e) and the second
    // ordering (q, its candidate eq) at positions cb + lane; lanes 0 and 63
    // also hold the entries just outside the chunk in both orderings (ex,
    // exq), at x = cb - 1 and cb + 64 when those exist.
    auto chunk = [&](const int cb, const uint32_t e, const uint32_t q, const uint32_t eq, const int x,
                     const uint32_t ex, const uint32_t exq) {
        const int i = cb + l;
        const bool valid = i < m;
        const int w = valid ? ce_w(e) : 0;
        const int wq = valid ? ce_w(eq) : 0;
        const int a = ce_a(e), b = ce_b(eq);
        // Neighbours in each ordering (other lanes of the chunk, or the
        // entries at its edges): first variables of the canonical list,
        // pairs of the second ordering (for b's range and the twin test).
        const uint32_t pq = valid ? ce_pair(eq) : 0u;
        int pa = __shfl_up(a, 1), na = __shfl_down(a, 1);
        uint32_t pp = __shfl_up(pq, 1), pn = __shfl_down(pq, 1);
        if (l == 0) {
            pa = x >= 0 && valid ? ce_a(ex) : -1;
            pp = x >= 0 && valid ? ce_pair(exq) : 0u;
        }
        if (l == kWave - 1 || i + 1 >= m) {
            na = x >= 0 && l == kWave - 1 ? ce_a(ex) : -1;
            pn = x >= 0 && l == kWave - 1 ? ce_pair(exq) : 0u;
        }
        if (valid) {
            const int va = vpos[a - 1], vb = vpos[b - 1];
            if (a != pa) rng[4 * va + 0] = i;
            if (a != na) rng[4 * va + 1] = i + 1;
            if ((pp & 0x7FFu) != (uint32_t)b) rng[4 * vb + 2] = i;
            if ((pn & 0x7FFu) != (uint32_t)b) rng[4 * vb + 3] = i + 1;
            // The place of q's pair in the second ordering: the first of
            // its entries (the twins of the two signs sit together there),
            // and bit 31 set when there are two.
            const bool twin_prev = pp == pq, twin_next = pn == pq;
            tinv[q] = (twin_prev ? i - 1 : i) | (twin_prev || twin_next ? (int)0x80000000u : 0);
        }
        const int word = 2 * (cb / kWave);
        // Lanes 0 and 1 store the low and high halves of four planes' ballots
        // at a time (one 16-byte store per ordering).
        for (int k = 0; k < ks; k += 4) {
            uint32_t c4[4], t4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t bc = ballot((w >> (k + u)) & 1), bt = ballot((wq >> (k + u)) & 1);
                c4[u] = (uint32_t)(l ? bc >> 32 : bc);
                t4[u] = (uint32_t)(l ? bt >> 32 : bt);
            }
            if (l < 2) {
                *(uint4*)(pl + (word + l) * ks + k) = make_uint4(c4[0], c4[1], c4[2], c4[3]);
                *(uint4*)(pl + ks * pw + (word + l) * ks + k) = make_uint4(t4[0], t4[1], t4[2], t4[3]);
            }
        }
    };
    // Two chunks per wave and iteration: their loads (the candidates, the
    // second ordering and its candidates, a dependent gather, the same for
    // the entries at the chunks' edges) are all in flight before either
    // chunk is processed.
    auto edge = [&](const int i) {  // cb - 1 for lane 0, cb + 64 for lane 63
        const int x = l == 0 ? i - 1 : l == kWave - 1 ? i + 1 : -1;
        return x >= 0 && x < m ? x : -1;
    };
    for (int base = 0; base < m; base += 2 * kWave * NW) {
        const int cb0 = base + kWave * grp_wave(), cb1 = cb0 + kWave * NW;
        const int i0 = cb0 + l, i1 = cb1 + l;
        const bool v0 = i0 < m, v1 = i1 < m;
        const int x0 = edge(i0), x1 = edge(i1);
        const uint32_t e0 = v0 ? cand[i0] : 0u, q0 = v0 ? tl[i0] : 0u;
        const uint32_t e1 = v1 ? cand[i1] : 0u, q1 = v1 ? tl[i1] : 0u;
        const uint32_t ex0 = x0 >= 0 ? cand[x0] : 0u, tx0 = x0 >= 0 ? tl[x0] : 0u;
        const uint32_t ex1 = x1 >= 0 ? cand[x1] : 0u, tx1 = x1 >= 0 ? tl[x1] : 0u;
        const uint32_t eq0 = v0 ? cand[q0] : 0u, eq1 = v1 ? cand[q1] : 0u;
        const uint32_t exq0 = x0 >= 0 ? cand[tx0] : 0u, exq1 = x1 >= 0 ? cand[tx1] : 0u;
        if (cb0 < m) chunk(cb0, e0, q0, eq0, x0, ex0, exq0);
        if (cb1 < m) chunk(cb1, e1, q1, eq1, x1, ex1, exq1);
    }
    __syncthreads();
    // S_v: the profit of the candidates holding live variable v, its pairs
    // (v, y) (canonical range) and (x, v) (range of the second ordering).
    for (int v = grp_tid(); v < n_live; v += kWave * NW) {
        const int4 r = *(const int4*)(rng + 4 * v);
        ssum[v] = plane_sum(pl, ks, r.x, r.y) + plane_sum(pl + ks * pw, ks, r.z, r.w);
    }
    __syncthreads();
}

template <int NW>
__device__ __forceinline__ int total_profit_grp(const uint32_t* cand, int m) {
    int tot = 0;
    for (int q = grp_tid(); q < m; q += kWave * NW) tot += ce_w(cand[q]);
    return grp_sum<NW>(tot);
}

template <int NW>
__device__ __forceinline__ int gi_argmax_grp(long long best_h, int best_p) {
    const long long hmax = grp_max64<NW>(best_h);
    return grp_min<NW>(best_h == hmax ? best_p : 0x7FFFFFFF);
}

// As select_gi_planes over the tables of gi_prepare_grp.
template <int NW>
__device__ __forceinline__ int select_gi_planes_grp(const uint32_t* cand, int m, int T, const int32_t* vpos,
                                                    const int32_t* rng, const int32_t* ssum,
                                                    const int32_t* tinv, const uint32_t* pl,
                                                    int pw, int K, uint32_t aq, uint32_t bq, uint32_t k0,
                                                    uint32_t k1, uint32_t proc, uint32_t dw, uint32_t eh,
                                                    long long* n_int, long long* n_blk) {
    const int ks = plane_stride(K);
    const uint32_t* plc = pl;
    const uint32_t* plt = pl + ks * pw;
    long long best_h = -1;
    int best_p = 0x7FFFFFFF;
    int my_int = 0, my_blk = 0;
    for (int p = grp_tid(); p < m; p += kWave * NW) {
        const uint32_t ep = cand[p];
        const uint32_t kp = ce_key(ep);
        const int va = vpos[ce_a(ep) - 1], vb = vpos[ce_b(ep) - 1];
        const int4 ra = *(const int4*)(rng + 4 * va);
        const int4 rb = *(const int4*)(rng + 4 * vb);
        const int tv = tinv[p];
        const int n_ab = tv < 0 ? 2 : 1;
        const int t_ab = tv & 0x7FFFFFFF;
        // I_p: the candidates holding a or b, less p (counted in both) and
        // its twin of the other sign (in both; next to p in canonical order).
        const int wp = ce_w(ep);
        const int w_twin = tv < 0 ? ce_w(cand[ce_neg(ep) ? p - 1 : p + 1]) : 0;
        const int I = ssum[va] + ssum[vb] - 2 * wp - w_twin;
        int X = 0, j = 0;
        CoinStream co;
        co.init(proc, dw, kp, eh, k0, k1);
        // The blocks of the first 256 coins are drawn by all lanes at once
        // (lazily, lanes reaching a block at different points would each
        // draw it in their own pass of the loop).
        co.first_block();
        if ((ra.w - ra.z) + (ra.y - ra.x - 1) + (rb.w - rb.z - n_ab) + (rb.y - rb.x) > 128) co.next_block();
        plane_window_x(plt, ks, ra.z, ra.w, j, co, X);
        plane_window_x_gap(plc, ks, ra.x, ra.y, p, 1, j, co, X);
        plane_window_x_gap(plt, ks, rb.z, rb.w, t_ab, n_ab, j, co, X);
        plane_window_x(plc, ks, rb.x, rb.y, j, co, X);
        const long long D = (long long)T - wp - I;
        const long long hsc = ((long long)wp << 32) + (long long)aq * ((D << 16) + (long long)bq * X);
        if (hsc > best_h) { best_h = hsc; best_p = p; }
        my_int += j;
        my_blk += (j + 127) >> 7;
    }
    *n_int = grp_sum<NW>(my_int);
    *n_blk = grp_sum<NW>(my_blk);
    return gi_argmax_grp<NW>(best_h, best_p);
}

template <int NW>
__device__ __forceinline__ int select_g_grp(const uint32_t* cand, int m) {
    unsigned long long best = 0;
    for (int q = grp_tid(); q < m; q += kWave * NW) {
        const unsigned long long key = ((unsigned long long)ce_c(cand[q]) << 32) | (0xFFFFFFFFull - (unsigned)q);
        best = key > best ? key : best;
    }
    best = grp_max_u64<NW>(best);
    return (int)(0xFFFFFFFFull - (best & 0xFFFFFFFFull));
}

template <int NW>
__device__ __forceinline__ int select_ga_grp(const uint32_t* cand, int m, uint32_t u) {
    const int t = grp_tid();
    int cmax = 0;
    for (int q = t; q < m; q += kWave * NW) {
        const int c = ce_c(cand[q]);
        cmax = c > cmax ? c : cmax;
    }
    cmax = grp_max<NW>(cmax);
    int mine = 0;
    for (int q = t; q < m; q += kWave * NW) mine += ce_c(cand[q]) == cmax;
    const int ties = grp_sum<NW>(mine);
    uint32_t want = scale_u32(u, (uint32_t)ties);
    for (int base = 0; base < m; base += kWave * NW) {
        const int q = base + t;
        const bool tie = q < m && ce_c(cand[q]) == cmax;
        const uint64_t bt = ballot(tie);
        const int cnt = popc64(bt);
        int tot;
        const int off = grp_offset<NW>(cnt, &tot);
        if (want < (uint32_t)tot) {
            int found = -1;
            const uint32_t rel = want - (uint32_t)off;
            if (want >= (uint32_t)off && rel < (uint32_t)cnt) {
                const uint64_t hit = ballot(tie && (uint32_t)lanes_below(bt) == rel);
                found = base + kWave * grp_wave() + ctz64(hit);
            }
            return grp_max<NW>(found);
        }
        want -= (uint32_t)tot;
    }
    return -1;
}

template <int NW>
__device__ __forceinline__ int select_wr_grp(const uint32_t* cand, int m, uint32_t u) {
    const int t = grp_tid();
    const int tot = total_profit_grp<NW>(cand, m);
    const uint32_t x = scale_u32(u, (uint32_t)tot);
    uint32_t run = 0;
    for (int base = 0; base < m; base += kWave * NW) {
        const int q = base + t;
        const int w = q < m ? ce_w(cand[q]) : 0;
        const uint32_t incl = (uint32_t)wave_scan(w);
        const int wtot = __builtin_amdgcn_readlane((int)incl, kWave - 1);
        int gtot;
        const int off = grp_offset<NW>(wtot, &gtot);
        const uint64_t hit = ballot(q < m && run + (uint32_t)off + incl > x);
        const int found = grp_min<NW>(hit ? base + kWave * grp_wave() + ctz64(hit) : 0x7FFFFFFF);
        if (found != 0x7FFFFFFF) return found;
        run += (uint32_t)gtot;
    }
    return -1;
}

template <int W, int NW>
__device__ int select_gp_grp(const uint32_t* cand, int m, const uint64_t* colP, const uint64_t* colN,
                             const uint32_t* live, int n_live, uint32_t alpha_q, long long* n_cols) {
    long long best_h = -1;
    int best_p = 0x7FFFFFFF;
    for (int base = 0; base < m; base += kWave * NW) {
        const int q = base + grp_tid();
        const uint32_t e = cand[q < m ? q : 0];
        const int a = ce_a(e), b = ce_b(e);
        const bool neg = ce_neg(e);
        uint64_t Pk[W], Nk[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t Pa = colP[(a - 1) * W + w], Na = colN[(a - 1) * W + w];
            const uint64_t Pb = colP[(b - 1) * W + w], Nb = colN[(b - 1) * W + w];
            const uint64_t R = neg ? ((Pa & Nb) | (Na & Pb)) : ((Pa & Pb) | (Na & Nb));
            Pk[w] = Pa & R;
            Nk[w] = Na & R;
        }
        int n_new = 0;
        for (int i = 0; i < n_live; ++i) {
            const int x = (int)live[i];
            int same = 0, opp = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t Px = colP[(x - 1) * W + w], Nx = colN[(x - 1) * W + w];
                same += popc64((Px & Pk[w]) | (Nx & Nk[w]));
                opp += popc64((Px & Nk[w]) | (Nx & Pk[w]));
            }
            n_new += (x == a || x == b) ? 0 : (same >= 2) + (opp >= 2);
        }
        if (q < m) {
            const long long h = ((long long)ce_w(e) << 16) + (long long)alpha_q * n_new;
            if (h > best_h) {
                best_h = h;
                best_p = q;
            }
        }
    }
    *n_cols = (long long)m * (n_live > 2 ? n_live - 2 : 0);
    return gi_argmax_grp<NW>(best_h, best_p);
}

// Algorithmic work of a step in 32-bit integer lane operations (the same
// cost model the oracle tallies): 98 per Philox block of the step draw;
// selection 2 n_int + 98 n_blk + 10 m for gi, 10 w m + 8 w n_cols + 2 m for
// gp (trial columns, their counts against n_cols columns, argmax), 2 m
// otherwise; 10 w for the substitution and 24 w (n_live - 1) for recounting
// the three changed columns, w = ceil(n_e / 32).
template <bool GP>
__device__ __forceinline__ unsigned long long step_ops(int strat, int m, long long n_int, long long n_blk,
                                                       int n_e, int n_live) {
    const long long w = (n_e + 31) / 32;
    const long long sel = GP               ? (10 * w * m + 8 * w * n_int + 2 * (long long)m)
                          : strat == S_GI ? (2 * n_int + 98 * n_blk + 10 * (long long)m)
                                          : 2 * (long long)m;
    return (unsigned long long)(98 + sel + 10 * w + 24 * w * (long long)(n_live - 1));
}

// Process draws (Sec. 3.5.1): one Philox block (process, PROC|0|iteration|0)
// gives the strategy by the integer weights (word 0; process 0 of iteration
// 0 runs g when proc0_greedy), alpha_q = u1 >> 17 in [0, 2^15) and
// beta_q = 2^15 + (u2 >> 17) in [2^15, 2^16), shared by U, V and W^T.
struct ProcDraw {
    int strat;
    uint32_t alpha_q, beta_q;
};
__device__ __forceinline__ ProcDraw process_draw(const RunArgs& R, uint32_t proc) {
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
    const U4 pu = philox10(proc, domain(TAG_PROC, 0, R.iteration, 0), 0u, 0u, k0, k1);
    ProcDraw d;
    d.strat = (R.proc0_greedy && proc == 0 && R.iteration == 0) ? (int)S_G : weighted_pick(R.weights, N_STRAT, pu.x);
    d.alpha_q = pu.y >> 17;
    d.beta_q = 32768u + (pu.z >> 17);
    return d;
}

#ifndef CSE_STEP_TU
// Strategy of every process of a run (the host orders the dispatch of units
// by expected work with it).
__global__ void proc_strategy_kernel(RunArgs R, uint32_t n, int32_t* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = process_draw(R, i).strat;
}
#endif  // CSE_STEP_TU

// A copy of a unit's segment with every word made wave-uniform.  The
// segment is read with vector loads, whose results the compiler keeps in
// vector registers and, with them, everything computed from them (the
// Philox key schedule, every state pointer): about 50 registers per lane
// held across the step loop.  Uniform copies live in scalar registers.
__device__ __forceinline__ Segment uniform_segment(const Segment& src) {
    constexpr int n = (int)(sizeof(Segment) / 4);
    uint32_t w[n];
    __builtin_memcpy(w, &src, sizeof(Segment));
#pragma unroll
    for (int i = 0; i < n; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    Segment s;
    __builtin_memcpy(&s, w, sizeof(Segment));
    return s;
}

__device__ __forceinline__ int find_segment(const Segment* segs, int n_segs, uint32_t g) {
    int lo = 0, hi = n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].unit_begin <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// The step kernel: one workgroup (one wave) per unit.  Restores the unit by
// replaying its program from the input system, counts all pairs once, then
// runs up to `budget` selection steps (Selection -> Substitution ->
// incremental Analysis) or until no pair occurs twice / the program reaches
// step_cap.  Grid unit g maps to segment s and process g - unit_begin; block
// b runs grid unit order[b].
// ---------------------------------------------------------------------------
// W: row words; GS: bulk state in HBM slots; ADJ: gi over per-variable
// ranges (large candidate sets) instead of masks; TL (with GS and ADJ): the
// range tables in LDS; GP: the body of the Greedy-Potential units (every
// other unit runs in the body without it); NW: waves per unit (one
// workgroup of 64 NW lanes; more than one only with ADJ).  Each
// (W, GS, ADJ, TL, NW) is its own kernel, so a launch carries only the code
// its units run and every pointer's memory is known.
template <int W, bool GS, bool ADJ, bool TL, bool GP, int NW>
__device__ __forceinline__ void step_body(const Segment* __restrict__ segs, int n_segs,
                                          const uint32_t* __restrict__ order, uint32_t n_grid, int* err) {
    extern __shared__ __attribute__((aligned(16))) uint64_t smem[];
    static_assert(NW == 1 || ADJ, "units of several waves walk ranges in gi");
    constexpr int NT = kWave * NW;  // lanes of the unit
    const int l = lane_id();
    if (blockIdx.x >= n_grid) return;
    // Dispatch order: the host lists grid units longest expected work first.
    const uint32_t g = order ? order[blockIdx.x] : blockIdx.x;
    const Segment sg = uniform_segment(segs[find_segment(segs, n_segs, g)]);
    const CompArgs& C = sg.C;
    const RunArgs& R = sg.R;
    const UnitState& S = sg.S;
    const uint32_t proc = g - sg.unit_begin;
    if (proc >= R.n_units || S.active[proc] == 0) return;

    const int n_vmax = C.n_x + C.n_fmax;
    // Candidate entries: 64-bit, or 32-bit for units of several waves.
    using Ent = typename std::conditional<(NW > 1), uint32_t, uint64_t>::type;
    const BulkLayout BL =
        bulk_layout(n_vmax, W, C.m_cap, C.newc_cap, C.m_words, ADJ ? 1 : 0, C.kbits, (int)sizeof(Ent));
    // HBM slots are addressed from a kernel argument (which the compiler
    // knows to be global memory) plus a byte offset, so every access to them
    // compiles to global rather than generic loads and stores.
    char* const garg = (char*)segs;
    char* bulk = GS ? garg + ((uintptr_t)(S.gs_base + (size_t)proc * S.gs_stride) - (uintptr_t)garg)
                    : (char*)smem;
    char* lists = GS ? (char*)smem : (char*)smem + BL.bytes;
    uint64_t* colP = (uint64_t*)(bulk + BL.colP);
    uint64_t* colN = (uint64_t*)(bulk + BL.colN);
    Ent* cand = (Ent*)(bulk + BL.cand);
    Ent* cand2 = (Ent*)(bulk + BL.cand2);
    uint64_t* newc = (uint64_t*)(bulk + BL.newc);
    uint64_t* M = (uint64_t*)(bulk + BL.M);
    uint16_t* wt = (uint16_t*)(bulk + BL.wt);
    uint32_t* tl = (uint32_t*)(bulk + BL.tl);
    int32_t* remap = (int32_t*)(bulk + BL.remap);
    int32_t* kpre = (int32_t*)(bulk + BL.kpre);
    const TableLayout TB = table_layout(n_vmax, C.m_cap, C.kbits);
    int32_t* rng = TL ? (int32_t*)((char*)smem + TB.rng) : (int32_t*)(bulk + BL.rng);
    int32_t* ssum = TL ? (int32_t*)((char*)smem + TB.ssum) : (int32_t*)(bulk + BL.ssum);
    int32_t* tinv = TL ? (int32_t*)((char*)smem + TB.tinv) : (int32_t*)(bulk + BL.tinv);
    uint32_t* pl = TL ? (uint32_t*)((char*)smem + TB.pl) : (uint32_t*)(bulk + BL.pl);
    const int pw = plane_words(C.m_cap);
    uint32_t* live = (uint32_t*)lists;
    int32_t* vpos = (int32_t*)(lists + (size_t)n_vmax * 4);
    // New-pair table and gi table budget of units of several waves (after the lists).
    uint64_t* npm = (uint64_t*)(lists + list_bytes(n_vmax));
    int32_t* npb = (int32_t*)(npm + 2 * ((n_vmax + 63) / 64));
    char* gtab = lists + list_bytes(n_vmax) + newpair_table_bytes(n_vmax);

    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);

    // Process draws (Sec. 3.5.1): strategy, alpha, beta.
    const ProcDraw pd = process_draw(R, proc);
    const int strat = pd.strat;
    const uint32_t alpha_q = pd.alpha_q;
    const uint32_t beta_q = pd.beta_q;
    // Each unit runs in exactly one of the two kernels of its class.
    if ((strat == S_GP) != GP) return;
    // The second candidate ordering is kept only where gi walks ranges.
    const bool need_tl = ADJ && (strat == S_GI || strat == S_MIX);

    if constexpr (!GS) {
        for (int i = l; i < n_vmax * W; i += NT) {
            const bool in = i < C.n_x * W;
            colP[i] = in ? C.P0[i] : 0ull;
            colN[i] = in ? C.N0[i] : 0ull;
        }
        __syncthreads();
    }

    int t = S.t[proc];
    const int epoch = S.epoch[proc];
    int executed = S.executed[proc];
    unsigned long long ops = S.ops[proc];
    int cost = C.naive0;
    uint32_t* prog = S.prog + (size_t)proc * C.prog_stride;

    // A unit whose state lives in an HBM slot resumes from it when the slot
    // holds the state after its current program (same length and epoch: no
    // restart since its last launch); the state is the one a replay would
    // rebuild.  Otherwise the unit replays its program (a shared prefix or an
    // earlier round) from the input.  The last 16 bytes of a slot record
    // (t, epoch, m, current candidate buffer) of the state it holds; t = -1:
    // none.
    bool resumed = false;
    int4 rs = make_int4(-1, 0, 0, 0);
    int4* rec = nullptr;
    if constexpr (GS) {
        rec = (int4*)(bulk + S.gs_stride - 16);
        rs = *rec;
        resumed = t > 0 && rs.x == t && rs.y == epoch;
        if (resumed) {
            cost = S.cost[proc];
            if constexpr (ADJ) {
                if (rs.w) {
                    Ent* sw = cand;
                    cand = cand2;
                    cand2 = sw;
                }
            }
        } else {
            for (int i = l; i < n_vmax * W; i += NT) {
                const bool in = i < C.n_x * W;
                colP[i] = in ? C.P0[i] : 0ull;
                colN[i] = in ? C.N0[i] : 0ull;
            }
            __syncthreads();
        }
    }

    // Replay the unit's program (a shared prefix or an earlier round).
    if (!resumed) {
        for (int i = 0; i < t; ++i) {
            int dead;
            int c;
            if constexpr (NW > 1) c = substitute_grp<W, NW>(colP, colN, prog[i], C.n_x + i, &dead);
            else c = substitute<W>(colP, colN, prog[i], C.n_x + i, &dead);
            cost -= c - 1;
        }
    }

    // Live list: variables with a nonzero column, ascending.
    int n_live = 0;
    if constexpr (NW > 1) {
        n_live = build_live_grp<W, NW>(colP, colN, C.n_x + t, live, vpos);
    } else {
        const int n_v = C.n_x + t;
        for (int b0 = 0; b0 < n_v; b0 += kWave) {
            const int v = b0 + l;
            bool nz = false;
            if (v < n_v) {
#pragma unroll
                for (int w = 0; w < W; ++w) nz |= (colP[v * W + w] | colN[v * W + w]) != 0;
            }
            const uint64_t mk = ballot(nz);
            if (nz) {
                const int p = n_live + lanes_below(mk);
                live[p] = (uint32_t)(v + 1);
                vpos[v] = p;
            }
            n_live += popc64(mk);
        }
        __syncthreads();
    }

    int err_flags = 0;
    int m;
    if (resumed) {
        m = rs.z;
    } else if (t == 0) {
        // Every unit of a component starts from the same input: its
        // candidates (and second ordering) were counted once, on load.
        m = C.m0;
        if constexpr (NW > 1)
            for (int i = l; i < m; i += NT) cand[i] = ce_from64(C.cand0[i]);
        else
            for (int i = l; i < m; i += NT) cand[i] = C.cand0[i];
        if (need_tl)
            for (int i = l; i < m; i += NT) tl[i] = C.tl0[i];
        __syncthreads();
    } else if constexpr (NW > 1) {
        m = analyse_full_grp<W, NW>(colP, colN, live, n_live, cand, C.m_cap, &err_flags);
        if (need_tl) build_tl_grp<W, NW>(colP, colN, live, n_live, cand, m, tl);
    } else {
        m = analyse_full<W>(colP, colN, live, n_live, cand, C.m_cap, &err_flags);
        if (need_tl) build_tl<W>(colP, colN, live, n_live, cand, m, tl);
    }
    int active = 1;
    for (int done = 0;; ++done) {
        if (m == 0 || (R.step_cap && (uint32_t)t >= R.step_cap) || t >= C.n_fmax) { active = 0; break; }
        if (R.budget >= 0 && done >= R.budget) break;
        // Cancellation is checked every 256 steps (a read of host memory);
        // the unit keeps its prefix.
        if ((done & 255) == 255 && R.cancel) {
            int flag;
            if constexpr (NW > 1) {
                // One read for the whole unit, so every wave leaves together.
                __shared__ int cflag;
                if (l == 0) cflag = __hip_atomic_load(R.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __syncthreads();
                flag = cflag;
                __syncthreads();
            } else {
                flag = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(R.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
            }
            if (flag) break;
        }

        // The step draw is consumed by ga, wr, gr and mix only.
        U4 su = {0u, 0u, 0u, 0u};
        if (!GP && strat != S_G && strat != S_GI)
            su = philox10(proc, domain(TAG_STEP, C.comp, (uint32_t)epoch, (uint32_t)t), 0u, epoch_high(epoch), k0,
                          k1);
        int s = strat;
        if (s == S_MIX) {
            const int mi = weighted_pick(R.mix_weights, 4, su.x);
            s = mi == 0 ? S_GI : mi == 1 ? S_GA : mi == 2 ? S_GR : S_WR;
        }
        if (s == S_GR) s = ((su.y >> 16) < R.gr_p_q16) ? S_GA : S_WR;

        long long n_int = 0, n_blk = 0;
        int pick;
        if constexpr (GP && NW > 1) {
            pick = select_gp_grp<W, NW>(cand, m, colP, colN, live, n_live, alpha_q, &n_int);
        } else if constexpr (GP) {
            pick = select_gp<W>(cand, m, colP, colN, live, n_live, alpha_q, &n_int);
        } else if (s == S_G) {
            if constexpr (NW > 1) pick = select_g_grp<NW>(cand, m);
            else pick = select_g(cand, m);
        } else if (s == S_GA) {
            if constexpr (NW > 1) pick = select_ga_grp<NW>(cand, m, su.z);
            else pick = select_ga(cand, m, su.z);
        } else if (s == S_WR) {
            if constexpr (NW > 1) pick = select_wr_grp<NW>(cand, m, su.z);
            else pick = select_wr(cand, m, su.z);
        } else {
            const uint32_t dw = domain(TAG_COIN, C.comp, (uint32_t)epoch, (uint32_t)t);
            const uint32_t eh = epoch_high((uint32_t)epoch);
            if constexpr (ADJ && NW > 1) {
                int T, K;
                gi_totals_grp<NW>(cand, m, C.kbits, &T, &K);
                // The ranges, profit sums and planes go to the unit's LDS
                // budget when they fit it (the range tables of TL units are in
                // LDS anyway).
                const int pw_m = plane_words(m);
                const int ss_b = (4 * n_live + 15) & ~15;
                if (GS && !TL && 16 * n_live + ss_b + 8 * plane_stride(K) * pw_m <= kGsTableBudget) {
                    int32_t* rng_l = (int32_t*)gtab;
                    int32_t* ssum_l = (int32_t*)(gtab + 16 * (size_t)n_live);
                    uint32_t* pl_l = (uint32_t*)(gtab + 16 * (size_t)n_live + ss_b);
                    gi_prepare_grp<NW>(cand, tl, m, vpos, n_live, rng_l, ssum_l, tinv, pl_l, pw_m, K);
                    pick = select_gi_planes_grp<NW>(cand, m, T, vpos, rng_l, ssum_l, tinv, pl_l, pw_m, K, alpha_q,
                                                    beta_q, k0, k1, proc, dw, eh, &n_int, &n_blk);
                } else {
                    gi_prepare_grp<NW>(cand, tl, m, vpos, n_live, rng, ssum, tinv, pl, pw, K);
                    pick = select_gi_planes_grp<NW>(cand, m, T, vpos, rng, ssum, tinv, pl, pw, K, alpha_q, beta_q, k0,
                                                    k1, proc, dw, eh, &n_int, &n_blk);
                }
            } else if constexpr (ADJ) {
                const int K = gi_prepare(cand, tl, m, vpos, n_live, rng, tinv, pl, pw, C.kbits);
                pick = select_gi_planes(cand, m, vpos, rng, tinv, pl, pw, C.kbits, K, alpha_q, beta_q, k0, k1, proc,
                                        dw, eh, &n_int, &n_blk);
            } else if (n_live * ((m + 31) / 32) <= 2 * C.m_words)
                pick = select_gi_sparse(cand, m, vpos, n_live, M, wt, alpha_q, beta_q, k0, k1, proc, dw, eh,
                                        &n_int, &n_blk);
            else
                pick = select_gi_dense(cand, m, alpha_q, beta_q, k0, k1, proc, dw, eh, &n_int, &n_blk);
        }
        if (pick < 0 || pick >= m) { err_flags |= ERR_BAD_PICK; active = 0; break; }

        uint32_t key;
        int csel;
        if constexpr (NW > 1) {
            key = ce_key(cand[pick]);
            csel = ce_c(cand[pick]);
        } else {
            const uint64_t e = cand[pick];
            key = (uint32_t)e;
            csel = entry_c(e);
        }
        __syncthreads();
        int dead;
        const int k = C.n_x + t + 1;
        int c;
        if constexpr (NW > 1) {
            c = substitute_grp<W, NW>(colP, colN, key, k - 1, &dead);
            n_live = update_live_grp<NW>(live, vpos, n_live, key_a(key), key_b(key), dead, k);
        } else {
            c = substitute<W>(colP, colN, key, k - 1, &dead);
            n_live = update_live(live, vpos, n_live, key_a(key), key_b(key), dead, k);
        }
        if (c != csel) err_flags |= ERR_COUNT_MISMATCH;
        if (l == 0) prog[t] = key;
        ++t;
        cost -= c - 1;
        ++executed;
        ops += step_ops<GP>(s, m, n_int, n_blk, C.n_e, n_live);
        if constexpr (ADJ) {
            int n_new = 0;
            const int m_old = m;
            if constexpr (NW > 1)
                m = update_candidates_db_grp<W, NW>(colP, colN, live, n_live, cand, m, cand2, newc, C.newc_cap,
                                                    C.m_cap, remap, kpre, vpos, npm, npb, key_a(key), key_b(key), k,
                                                    &n_new, &err_flags);
            else
                m = update_candidates_db<W>(colP, colN, live, n_live, cand, m, cand2, newc, C.newc_cap, C.m_cap,
                                            remap, kpre, key_a(key), key_b(key), k, &n_new, &err_flags);
            Ent* sw = cand;
            cand = cand2;
            cand2 = sw;
            if (need_tl) {
                if constexpr (NW > 1) update_tl_grp<NW>(tl, m_old, remap, newc, n_new);
                else update_tl(tl, m_old, remap, newc, n_new);
            }
        } else {
            m = update_candidates<W>(colP, colN, live, vpos, n_live, cand, m, newc, C.newc_cap, C.m_cap, key_a(key),
                                     key_b(key), k, &err_flags);
        }
    }
    unsigned any_err;
    if constexpr (NW > 1) any_err = grp_or<NW>((unsigned)err_flags);
    else any_err = __ockl_wfred_or_u32((unsigned)err_flags);
    if (any_err && l == 0) atomicOr(err, (int)any_err);

    if (l == 0) {
        if constexpr (GS) {
            const int cur = (ADJ && cand != (Ent*)(bulk + BL.cand)) ? 1 : 0;
            *rec = make_int4(t, epoch, m, cur);
        }
        S.t[proc] = t;
        S.cost[proc] = cost;
        S.executed[proc] = executed;
        S.ops[proc] = ops;
        S.strat[proc] = strat;
        S.active[proc] = active;
        if (!active) S.finish[proc] = wall_clock64() - *S.t0;
    }
}

// Each unit runs in the body of its strategy; the other body returns after
// the process draw.  gp units (any_gp: some job of the launch weights gp)
// thus share the launch with the others, while each body is compiled on its
// own.
// Units of several waves are held to 72 registers (seven waves per SIMD), a
// few spills below their natural need: the extra wave hides more memory
// latency than the spills cost (batch pass 1.217 s at seven, 1.254 s at
// six, 1.338 s at eight; the 6x6x6 job 66.0, 68.6 and 83.9 ms), while at 64
// registers (eight) the spills dominate.
template <int W, bool GS, bool ADJ, bool TL, int NW>
__global__ __launch_bounds__((kWave * NW), (NW > 1 ? 7 : 1)) void step_kernel(
    const Segment* __restrict__ segs, int n_segs, const uint32_t* __restrict__ order, uint32_t n_grid, int* err,
    int any_gp) {
    step_body<W, GS, ADJ, TL, false, NW>(segs, n_segs, order, n_grid, err);
    if (any_gp) step_body<W, GS, ADJ, TL, true, NW>(segs, n_segs, order, n_grid, err);
}

#ifndef CSE_STEP_TU
// Lowest cost over a component's units (out starts at INT_MAX).
__global__ void best_cost_kernel(const int32_t* cost, uint32_t n, int32_t* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMin(out, cost[i]);
}

// Job start stamp and per-unit state initialisation.
__global__ void init_units_kernel(UnitState S, uint32_t n_units, int stamp) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (stamp && i == 0) {
        *(unsigned long long*)S.t0 = wall_clock64();
        *S.round = 0;
    }
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
    if (S.gs_base) *(int4*)(S.gs_base + (size_t)i * S.gs_stride + S.gs_stride - 16) = make_int4(-1, 0, 0, 0);
}
#endif  // CSE_STEP_TU

}  // namespace csek
