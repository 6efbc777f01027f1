/*
 * cse_oracle.c -- plain CPU oracle for the randomized common-subexpression
 * elimination (CSE) processes of A. I. Perminov, "Parallel Heuristic
 * Exploration for Additive Complexity Reduction in Fast Matrix
 * Multiplication" (arXiv 2512.13365).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, no
 * header and no table with the HIP library; the product path never calls it.
 *
 * It is written to be checked by eye against the paper, not to be fast:
 *   - one unit = one linear-form system (E_U, E_V or E_W^T, Sec. 3.2) reduced
 *     by one process; its state is a dense int8 matrix rows x variables that
 *     gains one column per substitution;
 *   - every step recounts all canonical pairs from scratch (Algorithm 1,
 *     Analysis) by listing every pair occurrence of every row, sorting the
 *     list and counting equal runs;
 *   - selection follows Sec. 3.4 (g, ga, wr, gr, gi, mix) literally, the
 *     Greedy-Intersections score (Sec. 3.4.2, H and I) summed over every
 *     other candidate with an explicit intersection test (the O(m^2) form);
 *     Greedy-Potential (Sec. 2 and 3.4, described only in words there) does
 *     each candidate's trial substitution on a copy of the system and counts
 *     the fresh variable's pairs row by row;
 *   - substitution rewrites every row holding the pair or its negation
 *     (Algorithm 1, Substitution; Sec. 3.2.1).
 *
 * Points the paper leaves open (random generator, tie-breaks, fixed-point
 * score, coin indexing, sharing schedule) are fixed by explicit readings;
 * each is stated where it is used below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OC_OK 0
#define OC_EINVAL (-1)
#define OC_ENOMEM (-2)
#define OC_ERANGE (-3)

/* Strategy ids (Sec. 3.4.1, 3.4.2, 3.4.3; gp of Sec. 2 and 3.4, read as below). */
enum { S_G = 0, S_GA = 1, S_WR = 2, S_GR = 3, S_GI = 4, S_MIX = 5, S_GP = 6, N_STRAT = 7 };

/* Random-stream tags placed in the top nibble of counter word 1 (REINIT is
 * drawn by the outer-iteration driver, which composes pool runs). */
enum { TAG_PROC = 1, TAG_STEP = 2, TAG_COIN = 3, TAG_SHARE = 4, TAG_REINIT = 5, TAG_FLIP = 6 };

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplications
 * with a Weyl-sequence key schedule.  The paper does not name a generator;
 * a counter-based one makes every draw a pure function of its counter.
 * ---------------------------------------------------------------------- */
void oc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter word 1: tag[31:28] component[27:26] epoch[25:16] step[15:0]. */
uint32_t oc_domain_word(uint32_t tag, uint32_t comp, uint32_t epoch, uint32_t step)
{
    return (tag << 28) | ((comp & 3u) << 26) | ((epoch & 0x3FFu) << 16) | (step & 0xFFFFu);
}

/* A unit's epoch counts its restarts and can pass the 10 bits of word 1
 * (sharing events and outer iterations add up).  So that no step or coin key
 * is ever reused, the epoch's bits above the tenth go to the upper half of
 * counter word 3 of those draws (whose lower half is 0 for a step draw, and
 * a coin stream's block index, < 2^15, plus its side bit 2^15 for a coin
 * draw); epochs below 1024 leave word 3 as it was. */
uint32_t oc_epoch_high(uint32_t epoch) { return (epoch >> 10) << 16; }

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = { c0, c1, c2, c3 };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    oc_philox4x32_10(ctr, key, out);
}

/* An index in [0, n) from a 32-bit word: floor(u * n / 2^32). */
static uint32_t scale_index(uint32_t u, uint64_t n) { return (uint32_t)(((uint64_t)u * n) >> 32); }

/* Pick i with probability w[i] / sum(w): the first i whose running sum
 * exceeds floor(u * sum / 2^32). */
static int weighted_pick(const uint32_t* w, int n, uint32_t u)
{
    uint64_t total = 0;
    for (int i = 0; i < n; i++) total += w[i];
    uint64_t x = ((uint64_t)u * total) >> 32;
    uint64_t run = 0;
    for (int i = 0; i < n; i++) {
        run += w[i];
        if (run > x) return i;
    }
    return -1;
}

/* ------------------------------------------------------------------------
 * Canonical pairs (Sec. 3.3.1): x_a + s x_b with a < b (1-based ids) and the
 * sign normalised so that x_a has coefficient +1; s is the product of the two
 * coefficients.  key = a<<16 | b<<1 | (s<0) orders pairs by (a, b, sign) with
 * + before -; this order is the canonical order used for every tie-break.
 * ---------------------------------------------------------------------- */
static uint32_t pair_key(int a, int b, int s) { return ((uint32_t)a << 16) | ((uint32_t)b << 1) | (uint32_t)(s < 0); }
static int key_a(uint32_t k) { return (int)(k >> 16); }
static int key_b(uint32_t k) { return (int)((k >> 1) & 0x7FFFu); }
static int key_s(uint32_t k) { return (k & 1u) ? -1 : 1; }

typedef struct { uint32_t key; int32_t c; } oc_cand;

/* Naive additions of a system (Sec. 3.2.1): sum over rows of (nnz - 1). */
int64_t oc_naive(const int8_t* A, int n_e, int n_v, int stride)
{
    int64_t total = 0;
    for (int i = 0; i < n_e; i++) {
        int nnz = 0;
        for (int j = 0; j < n_v; j++) nnz += (A[(size_t)i * stride + j] != 0);
        total += nnz - 1;
    }
    return total;
}

/* Upper bound on pair occurrences: sum over rows of C(nnz, 2).  Rows only
 * lose nonzeros over time, so the initial value bounds every later one. */
int64_t oc_pair_occurrences(const int8_t* A, int n_e, int n_v, int stride)
{
    int64_t total = 0;
    for (int i = 0; i < n_e; i++) {
        int64_t nnz = 0;
        for (int j = 0; j < n_v; j++) nnz += (A[(size_t)i * stride + j] != 0);
        total += nnz * (nnz - 1) / 2;
    }
    return total;
}

static int cmp_u32(const void* x, const void* y)
{
    uint32_t a = *(const uint32_t*)x, b = *(const uint32_t*)y;
    return (a > b) - (a < b);
}

/* Algorithm 1, Analysis: list every canonical pair of every row, sort, and
 * keep the pairs that occur at least twice, in canonical order.  occ must
 * hold oc_pair_occurrences() entries.  Returns the number of candidates. */
int oc_analyse(const int8_t* A, int n_e, int n_v, int stride, uint32_t* occ, oc_cand* out)
{
    int n_occ = 0;
    for (int i = 0; i < n_e; i++) {
        const int8_t* row = A + (size_t)i * stride;
        for (int x = 0; x < n_v; x++) {
            if (!row[x]) continue;
            for (int y = x + 1; y < n_v; y++) {
                if (!row[y]) continue;
                occ[n_occ++] = pair_key(x + 1, y + 1, row[x] * row[y]);
            }
        }
    }
    qsort(occ, (size_t)n_occ, sizeof(uint32_t), cmp_u32);
    int m = 0;
    for (int i = 0; i < n_occ;) {
        int j = i;
        while (j < n_occ && occ[j] == occ[i]) j++;
        if (j - i >= 2) { out[m].key = occ[i]; out[m].c = j - i; m++; }
        i = j;
    }
    return m;
}

/* ------------------------------------------------------------------------
 * Selection strategies (Sec. 3.4).  Each returns an index into the
 * candidate list, which is in canonical order.
 * ---------------------------------------------------------------------- */

/* Greedy (g): highest frequency c; ties go to the first in canonical order. */
int oc_select_g(const oc_cand* C, int m)
{
    int best = 0;
    for (int q = 1; q < m; q++)
        if (C[q].c > C[best].c) best = q;
    return best;
}

/* Greedy-Alternative (ga): uniform among the pairs of maximal frequency; the
 * ties are numbered in canonical order and index floor(u * n_ties / 2^32) is
 * taken. */
int oc_select_ga(const oc_cand* C, int m, uint32_t u)
{
    int cmax = 0, n_ties = 0;
    for (int q = 0; q < m; q++) if (C[q].c > cmax) cmax = C[q].c;
    for (int q = 0; q < m; q++) n_ties += (C[q].c == cmax);
    int want = (int)scale_index(u, (uint64_t)n_ties);
    for (int q = 0; q < m; q++) {
        if (C[q].c != cmax) continue;
        if (want == 0) return q;
        want--;
    }
    return -1;
}

/* Weighted-Random (wr): probability proportional to the profit c - 1, drawn
 * by running sums in canonical order. */
int oc_select_wr(const oc_cand* C, int m, uint32_t u)
{
    uint64_t total = 0;
    for (int q = 0; q < m; q++) total += (uint64_t)(C[q].c - 1);
    uint64_t x = ((uint64_t)u * total) >> 32;
    uint64_t run = 0;
    for (int q = 0; q < m; q++) {
        run += (uint64_t)(C[q].c - 1);
        if (run > x) return q;
    }
    return -1;
}

/* Greedy-Intersections (gi), Sec. 3.4.2, scores
 *     H(p) = (c_p - 1) + alpha * sum_{q != p} I(p, q)
 *     I(p, q) = c_q - 1                          if p and q are disjoint,
 *               0 or beta (c_q - 1), prob 1/2    if they intersect.
 * alpha = alpha_q / 2^16 in [0, 0.5), beta = beta_q / 2^16 in [0.5, 1).
 * 2^32 H is evaluated exactly in 64-bit integers:
 *     (c_p - 1) 2^32 + alpha_q (D_p 2^16 + beta_q X_p),
 * D_p = sum of c_q - 1 over disjoint q, X_p = the same over intersecting q
 * whose coin is 1.  Ties go to the first in canonical order.
 *
 * Two candidates intersect when they share a variable index (the sign is
 * ignored: a substitution removes both variables from the affected rows).
 * Coins: every intersecting q of p = (a, b) gets one fair coin of its own.
 * The intersecting candidates are split by the variable they share with p:
 * A_p = the candidates holding a (p's twin of the other sign included),
 * B_p = those holding b but not a, each in canonical order.  The i-th member
 * of the sequence A_p then B_p (i = 0 .. |A_p| + |B_p| - 1) takes bit
 * i mod 128 of the Philox block counter (process, COIN|comp|epoch|step,
 * key(p), i div 128 | high epoch bits), as word (i mod 128) div 32, bit
 * i mod 32.
 *
 * n_int and n_blk (optional) receive sum_p (|A_p| + |B_p|) and the Philox
 * blocks a candidate's coins span, sum_p ceil((|A_p| + |B_p|) / 128), for
 * the algorithmic work tally. */
int oc_select_gi(const oc_cand* C, int m, uint32_t alpha_q, uint32_t beta_q,
                 uint64_t seed, uint32_t proc, uint32_t comp, uint32_t epoch, uint32_t step,
                 int64_t* n_int, int64_t* n_blk)
{
    int best = -1;
    int64_t best_h = 0, tot_int = 0, tot_blk = 0;
    const uint32_t dw = oc_domain_word(TAG_COIN, comp, epoch, step);
    const uint32_t eh = oc_epoch_high(epoch);
    for (int p = 0; p < m; p++) {
        const int pa = key_a(C[p].key), pb = key_b(C[p].key);
        /* |A_p| first: B_p's coins follow A_p's. */
        int64_t na = 0;
        for (int q = 0; q < m; q++)
            if (q != p && (key_a(C[q].key) == pa || key_b(C[q].key) == pa)) na++;
        int64_t D = 0, X = 0;
        int64_t ia = 0, ib = 0;             /* members of A_p and B_p so far */
        /* The block of A_p's current coin and of B_p's (-1: none drawn). */
        int64_t cur_a = -1, cur_b = -1;
        uint32_t blk_a[4] = { 0, 0, 0, 0 }, blk_b[4] = { 0, 0, 0, 0 };
        for (int q = 0; q < m; q++) {
            if (q == p) continue;
            const int64_t wq = C[q].c - 1;
            const int qa = key_a(C[q].key), qb = key_b(C[q].key);
            int64_t i;
            uint32_t* blk;
            int64_t* cur;
            if (qa == pa || qb == pa) {
                i = ia++;
                blk = blk_a;
                cur = &cur_a;
            } else if (qa == pb || qb == pb) {
                i = na + ib++;
                blk = blk_b;
                cur = &cur_b;
            } else {
                D += wq;
                continue;
            }
            if (*cur != i / 128) {
                draw(seed, proc, dw, C[p].key, (uint32_t)(i / 128) | eh, blk);
                *cur = i / 128;
            }
            if ((blk[(i % 128) / 32] >> (i % 32)) & 1u) X += wq;
        }
        tot_int += ia + ib;
        tot_blk += (ia + ib + 127) / 128;
        int64_t h = ((int64_t)(C[p].c - 1) << 32) + (int64_t)alpha_q * ((D << 16) + (int64_t)beta_q * X);
        if (best < 0 || h > best_h) { best = p; best_h = h; }
    }
    if (n_int) *n_int = tot_int;
    if (n_blk) *n_blk = tot_blk;
    return best;
}

int oc_substitute(int8_t* A, int n_e, int stride, int a, int b, int s, int k);

/* Greedy-Potential (gp), Sec. 2 and 3.4: a candidate's potential is the
 * number of new substitution possibilities a trial substitution creates.
 * Counts of old pairs can only fall, so the new possibilities are the pairs
 * (x, k, s) of the fresh variable k that occur at least twice.  Reading:
 *     2^16 H(p) = (c_p - 1) 2^16 + alpha_q N_new(p),
 * alpha_q the process's alpha (alpha = alpha_q / 2^16 in [0, 0.5), as for
 * gi), evaluated exactly; ties go to the first in canonical order.  For each
 * candidate the oracle substitutes on a copy of the n_e x n_v system and
 * counts the fresh variable's pairs row by row.  n_cols (optional) receives
 * the number of (candidate, live column other than a and b) pairs counted,
 * for the algorithmic work tally. */
int oc_select_gp(const int8_t* A, int n_e, int n_v, int stride, const oc_cand* C, int m, uint32_t alpha_q,
                 int64_t* n_cols)
{
    int8_t* T = (int8_t*)malloc((size_t)n_e * stride);
    int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * 2 * ((size_t)n_v + 1));
    if (!T || !cnt) { free(T); free(cnt); return -1; }
    int live = 0;
    for (int j = 0; j < n_v; j++) {
        for (int i = 0; i < n_e; i++)
            if (A[(size_t)i * stride + j]) { live++; break; }
    }
    int best = -1;
    int64_t best_h = 0;
    for (int p = 0; p < m; p++) {
        int a = key_a(C[p].key), b = key_b(C[p].key), s = key_s(C[p].key);
        memcpy(T, A, (size_t)n_e * stride);
        int k = n_v + 1;
        oc_substitute(T, n_e, stride, a, b, s, k);
        memset(cnt, 0, sizeof(int32_t) * 2 * ((size_t)n_v + 1));
        for (int i = 0; i < n_e; i++) {
            int8_t ak = T[(size_t)i * stride + (k - 1)];
            if (!ak) continue;
            for (int x = 1; x <= n_v; x++) {
                int8_t ax = T[(size_t)i * stride + (x - 1)];
                if (ax) cnt[2 * x + (ax * ak < 0)]++;
            }
        }
        int64_t n_new = 0;
        for (int x = 1; x <= n_v; x++) n_new += (cnt[2 * x] >= 2) + (cnt[2 * x + 1] >= 2);
        int64_t h = ((int64_t)(C[p].c - 1) << 16) + (int64_t)alpha_q * n_new;
        if (best < 0 || h > best_h) { best = p; best_h = h; }
    }
    if (n_cols) *n_cols = (int64_t)m * (live > 2 ? live - 2 : 0);
    free(T);
    free(cnt);
    return best;
}

/* ------------------------------------------------------------------------
 * Substitution (Algorithm 1; Sec. 3.2.1): fresh x_k = x_a + s x_b replaces
 * the pair in every row where both occur with relative sign s; the row keeps
 * the coefficient of x_a on x_k (alpha_a x_a + alpha_b x_b = alpha_a x_k when
 * alpha_a alpha_b = s).  Returns the number of rows rewritten, c.
 * ---------------------------------------------------------------------- */
int oc_substitute(int8_t* A, int n_e, int stride, int a, int b, int s, int k)
{
    int c = 0;
    for (int i = 0; i < n_e; i++) {
        int8_t* row = A + (size_t)i * stride;
        int8_t va = row[a - 1], vb = row[b - 1];
        if (va == 0 || vb == 0 || va * vb != s) continue;
        row[k - 1] = va;
        row[a - 1] = 0;
        row[b - 1] = 0;
        c++;
    }
    return c;
}

/* ------------------------------------------------------------------------
 * Configuration and per-process initialisation (Sec. 3.5.1).
 * ---------------------------------------------------------------------- */
typedef struct {
    uint64_t seed;
    uint32_t n_proc;
    uint32_t weights[7];      /* g, ga, wr, gr, gi, mix, gp */
    uint32_t mix_weights[4];  /* gi, ga, gr, wr (Sec. 3.4.3: 8, 4, 2, 1) */
    uint32_t proc0_greedy;    /* process 0 of iteration 0 runs g (Sec. 3.5.1) */
    uint32_t gr_p_q16;        /* Greedy-Random: probability of ga, 2^-16 units */
    uint32_t step_cap;        /* maximum program length; 0 = none */
    uint32_t share_every;     /* steps per sharing round; 0 = no sharing */
    uint32_t share_src_pm;    /* sources: first ceil(N * pm / 1000) by (cost, process) */
    uint32_t share_dst_pm;    /* each active non-source unit is a target with prob pm/1000 */
    uint32_t share_max_rounds;/* sharing events at most */
    uint32_t iteration;       /* outer iteration; keys the per-process draws */
} oc_cfg;

/* Strategy, alpha and beta of process `proc`: one Philox block keyed by
 * (process, PROC|0|iteration|0); word 0 picks the strategy by the integer
 * weights, word 1 gives alpha_q = u >> 17 in [0, 2^15), word 2 gives
 * beta_q = 2^15 + (u >> 17) in [2^15, 2^16).  Shared by U, V and W^T. */
int oc_proc_init(const oc_cfg* cfg, uint32_t proc, uint32_t* alpha_q, uint32_t* beta_q)
{
    uint32_t u[4];
    draw(cfg->seed, proc, oc_domain_word(TAG_PROC, 0, cfg->iteration, 0), 0, 0, u);
    int strat;
    if (cfg->proc0_greedy && proc == 0 && cfg->iteration == 0) strat = S_G;
    else strat = weighted_pick(cfg->weights, N_STRAT, u[0]);
    *alpha_q = u[1] >> 17;
    *beta_q = 32768u + (u[2] >> 17);
    return strat;
}

/* ------------------------------------------------------------------------
 * One unit: one component reduced by one process.
 * ---------------------------------------------------------------------- */
typedef struct {
    int8_t* A;          /* n_e x stride, stride = n_v_max */
    int32_t* prog;      /* 3 * n_f_max: a, b, s per substitution */
    uint32_t* occ;      /* pair-occurrence scratch */
    oc_cand* cand;      /* candidate scratch */
    int t;              /* program length */
    int64_t cost;
    int epoch;          /* reinitialisations so far */
    int k0;             /* program length right after the last reinitialisation */
    int executed;       /* selection steps executed (replays excluded) */
    int active;
    int64_t ops;        /* algorithmic work tally */
    uint32_t proc;
    int strat;
    uint32_t alpha_q, beta_q;
} oc_unit;

typedef struct {
    const int8_t* A0;
    int n_e, n_x, n_vmax, n_fmax;
    int64_t naive0;
    int64_t occ_cap;
    uint32_t comp;
    const oc_cfg* cfg;
} oc_problem;

static int live_columns(const int8_t* A, int n_e, int n_v, int stride)
{
    int live = 0;
    for (int j = 0; j < n_v; j++) {
        for (int i = 0; i < n_e; i++)
            if (A[(size_t)i * stride + j]) { live++; break; }
    }
    return live;
}

/* Algorithmic work of one step, in 32-bit integer lane operations (a cost
 * model, not a count of what any implementation executes):
 *   98                       one Philox4x32-10 block for the step draw
 *   gi:  2 n_int + 98 n_blk + 10 m   coin tests and masked adds, coin blocks,
 *                                    disjoint sums, score and argmax
 *   gp:  10 w m + 8 w n_cols + 2 m   trial substitutions, the fresh column's
 *                                    pair counts against n_cols live columns
 *                                    (four sign pairs: AND + POPC), argmax
 *   other strategies: 2 m             one scan plus one pick pass
 *   10 w                              substitution over w 32-bit row words
 *   24 w (n_live - 1)                 recount of the three changed columns
 *                                    against every other live column
 * with w = ceil(n_e / 32) and n_live counted after the substitution. */
static int64_t step_ops(int strat, int m, int64_t n_int, int64_t n_blk, int n_e, int n_live)
{
    int64_t w = (n_e + 31) / 32;
    int64_t sel = (strat == S_GI) ? (2 * n_int + 98 * n_blk + 10 * (int64_t)m)
                : (strat == S_GP) ? (10 * w * (int64_t)m + 8 * w * n_int + 2 * (int64_t)m) : (2 * (int64_t)m);
    return 98 + sel + 10 * w + 24 * w * (int64_t)(n_live - 1);
}

/* Restart a unit from the input system and replay the first k substitutions
 * of `src` (Sec. 3.5.2: copy the first k substitutions of a solution). */
static int unit_replay(const oc_problem* P, oc_unit* U, const int32_t* src, int k)
{
    memcpy(U->A, P->A0, (size_t)P->n_e * P->n_vmax);
    U->cost = P->naive0;
    U->t = 0;
    for (int i = 0; i < k; i++) {
        int a = src[3 * i], b = src[3 * i + 1], s = src[3 * i + 2];
        int kk = P->n_x + i + 1;
        int c = oc_substitute(U->A, P->n_e, P->n_vmax, a, b, s, kk);
        if (c < 2) return OC_EINVAL;
        U->prog[3 * i] = a; U->prog[3 * i + 1] = b; U->prog[3 * i + 2] = s;
        U->cost -= c - 1;
        U->t++;
    }
    return OC_OK;
}

/* Run a unit for at most `budget` selection steps (budget < 0: unlimited).
 * At the top of every step the pairs are recounted; the unit finishes when
 * no pair occurs twice (Algorithm 1's loop condition) or its program reached
 * step_cap; otherwise, with the budget spent, it stays active. */
static void unit_run(const oc_problem* P, oc_unit* U, int budget)
{
    const oc_cfg* cfg = P->cfg;
    int done = 0;
    while (U->active) {
        int m = oc_analyse(U->A, P->n_e, P->n_x + U->t, P->n_vmax, U->occ, U->cand);
        if (m == 0 || (cfg->step_cap && (uint32_t)U->t >= cfg->step_cap) || U->t >= P->n_fmax) {
            U->active = 0;
            break;
        }
        if (budget >= 0 && done >= budget) break;

        uint32_t u[4];
        draw(cfg->seed, U->proc, oc_domain_word(TAG_STEP, P->comp, (uint32_t)U->epoch, (uint32_t)U->t), 0,
             oc_epoch_high((uint32_t)U->epoch), u);
        int strat = U->strat;
        if (strat == S_MIX) {
            static const int mix_map[4] = { S_GI, S_GA, S_GR, S_WR };
            strat = mix_map[weighted_pick(cfg->mix_weights, 4, u[0])];
        }
        if (strat == S_GR)
            strat = ((u[1] >> 16) < cfg->gr_p_q16) ? S_GA : S_WR;

        int64_t n_int = 0, n_blk = 0;
        int pick;
        switch (strat) {
        case S_G:  pick = oc_select_g(U->cand, m); break;
        case S_GA: pick = oc_select_ga(U->cand, m, u[2]); break;
        case S_WR: pick = oc_select_wr(U->cand, m, u[2]); break;
        case S_GI: pick = oc_select_gi(U->cand, m, U->alpha_q, U->beta_q, cfg->seed, U->proc, P->comp,
                                       (uint32_t)U->epoch, (uint32_t)U->t, &n_int, &n_blk); break;
        case S_GP: pick = oc_select_gp(U->A, P->n_e, P->n_x + U->t, P->n_vmax, U->cand, m, U->alpha_q, &n_int);
                   break;
        default:   pick = -1; break;
        }
        if (pick < 0) { U->active = 0; break; }

        uint32_t key = U->cand[pick].key;
        int a = key_a(key), b = key_b(key), s = key_s(key);
        int k = P->n_x + U->t + 1;
        int c = oc_substitute(U->A, P->n_e, P->n_vmax, a, b, s, k);
        U->prog[3 * U->t] = a; U->prog[3 * U->t + 1] = b; U->prog[3 * U->t + 2] = s;
        U->t++;
        U->cost -= c - 1;
        U->executed++;
        int n_live = live_columns(U->A, P->n_e, P->n_x + U->t, P->n_vmax);
        U->ops += step_ops(strat, m, n_int, n_blk, P->n_e, n_live);
        done++;
    }
}

/* ------------------------------------------------------------------------
 * Pool driver: every unit of one component, with optional sharing rounds.
 * ---------------------------------------------------------------------- */
typedef struct {
    const oc_problem* P;
    oc_unit* units;
    int n_units;
    int budget;
    int tid, n_threads;
} oc_job;

static void* run_slice(void* arg)
{
    oc_job* J = (oc_job*)arg;
    for (int i = J->tid; i < J->n_units; i += J->n_threads)
        if (J->units[i].active) unit_run(J->P, &J->units[i], J->budget);
    return NULL;
}

static void run_all(const oc_problem* P, oc_unit* units, int n_units, int budget, int n_threads)
{
    if (n_threads <= 1) {
        oc_job J = { P, units, n_units, budget, 0, 1 };
        run_slice(&J);
        return;
    }
    pthread_t th[256];
    oc_job J[256];
    if (n_threads > 256) n_threads = 256;
    for (int t = 0; t < n_threads; t++) {
        J[t] = (oc_job){ P, units, n_units, budget, t, n_threads };
        pthread_create(&th[t], NULL, run_slice, &J[t]);
    }
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
}

static const oc_unit* g_sort_units;
static int cmp_rank(const void* x, const void* y)
{
    const oc_unit* a = &g_sort_units[*(const int*)x];
    const oc_unit* b = &g_sort_units[*(const int*)y];
    if (a->cost != b->cost) return (a->cost > b->cost) - (a->cost < b->cost);
    return (a->proc > b->proc) - (a->proc < b->proc);
}

/* One sharing event (Sec. 3.5.2, periodic variant): rank all units of the
 * pool by (current cost, process); the first ceil(N src_pm / 1000) are the
 * sources.  Each active non-source unit draws one Philox block keyed by
 * (process, SHARE|comp|iteration|0, round, 0): word 0 makes it a target with
 * probability dst_pm / 1000, word 1 picks its source among the sources in
 * rank order, word 2 picks k uniformly in [1, max(1, floor(3 L / 4))] with L
 * the source's program length.  A target restarts from the first k
 * substitutions of its source, keeps its own strategy, alpha and beta, and
 * increments its epoch.  Sources of this event are never targets, so every
 * copy reads a source's state from before the event. */
static int share_round(const oc_problem* P, oc_unit* units, int n_units, uint32_t round, int32_t* snap)
{
    const oc_cfg* cfg = P->cfg;
    int* order = (int*)malloc(sizeof(int) * (size_t)n_units);
    char* is_src = (char*)calloc((size_t)n_units, 1);
    if (!order || !is_src) { free(order); free(is_src); return OC_ENOMEM; }
    for (int i = 0; i < n_units; i++) order[i] = i;
    g_sort_units = units;
    qsort(order, (size_t)n_units, sizeof(int), cmp_rank);
    int n_src = (int)(((int64_t)n_units * cfg->share_src_pm + 999) / 1000);
    if (n_src < 1) n_src = 1;
    if (n_src > n_units) n_src = n_units;
    for (int i = 0; i < n_src; i++) is_src[order[i]] = 1;
    /* Sources are not modified during the event; their programs are read
     * directly, the snapshot only guards the in-place rewrite below. */
    int rc = OC_OK;
    for (int i = 0; i < n_units && rc == OC_OK; i++) {
        oc_unit* U = &units[i];
        if (!U->active || is_src[i]) continue;
        uint32_t u[4];
        draw(cfg->seed, U->proc, oc_domain_word(TAG_SHARE, P->comp, cfg->iteration, 0), round, 0, u);
        if (scale_index(u[0], 1000) >= cfg->share_dst_pm) continue;
        const oc_unit* S = &units[order[scale_index(u[1], (uint64_t)n_src)]];
        int L = S->t;
        if (L == 0) continue;
        int kmax = (3 * L) / 4;
        if (kmax < 1) kmax = 1;
        int k = 1 + (int)scale_index(u[2], (uint64_t)kmax);
        memcpy(snap, S->prog, sizeof(int32_t) * 3 * (size_t)k);
        rc = unit_replay(P, U, snap, k);
        U->epoch++;
        U->k0 = k;
    }
    free(order);
    free(is_src);
    return rc;
}

/* Run units of one component.
 *   A0            n_e x n_x input system, row-major int8 in {-1, 0, 1}
 *   comp          component id 0..3 (keys the random streams)
 *   procs         process index of each unit; NULL = 0 .. n_units-1
 *                 (sharing needs the whole pool: NULL and n_units = n_proc)
 *   init_prog/init_len/init_epoch   optional per-unit starting prefix
 *                 (n_units x prog_cap x 3) and epoch, for continuing a unit
 *                 from a known prefix; NULL = start from the input system
 *   outputs       per unit; prog is n_units x prog_cap x 3 (a, b, s)
 * Returns OC_OK or a negative error. */
int oc_run_pool(const int8_t* A0, int n_e, int n_x, int comp, const oc_cfg* cfg,
                int n_units, const int32_t* procs,
                const int32_t* init_prog, const int32_t* init_len, const int32_t* init_epoch,
                int64_t* cost, int32_t* steps, int32_t* executed, int32_t* epoch, int32_t* k0,
                int64_t* ops, int32_t* strat, int32_t* prog, int prog_cap, int n_threads)
{
    if (n_e < 1 || n_x < 1 || n_units < 0 || comp < 0 || comp > 3 || !cfg) return OC_EINVAL;
    for (int64_t i = 0; i < (int64_t)n_e * n_x; i++) if (A0[i] < -1 || A0[i] > 1) return OC_EINVAL;
    for (int i = 0; i < n_e; i++) {
        int nnz = 0;
        for (int j = 0; j < n_x; j++) nnz += A0[(size_t)i * n_x + j] != 0;
        if (nnz == 0) return OC_EINVAL;
    }
    if (cfg->share_every && procs) return OC_EINVAL;

    oc_problem P;
    int64_t nnz0 = 0;
    for (int64_t i = 0; i < (int64_t)n_e * n_x; i++) nnz0 += A0[i] != 0;
    P.n_e = n_e; P.n_x = n_x; P.comp = (uint32_t)comp; P.cfg = cfg;
    /* Each substitution removes c >= 2 nonzeros and rows never empty, so at
     * most floor((nnz - n_e) / 2) fresh variables are ever created. */
    P.n_fmax = (int)((nnz0 - n_e) / 2);
    P.n_vmax = n_x + P.n_fmax;
    if (P.n_vmax >= 32768 || prog_cap < P.n_fmax) return OC_ERANGE;
    int8_t* A0w = (int8_t*)calloc((size_t)n_e * P.n_vmax, 1);
    if (!A0w) return OC_ENOMEM;
    for (int i = 0; i < n_e; i++) memcpy(A0w + (size_t)i * P.n_vmax, A0 + (size_t)i * n_x, (size_t)n_x);
    P.A0 = A0w;
    P.naive0 = oc_naive(A0w, n_e, n_x, P.n_vmax);
    P.occ_cap = oc_pair_occurrences(A0w, n_e, n_x, P.n_vmax);

    oc_unit* units = (oc_unit*)calloc((size_t)n_units + 1, sizeof(oc_unit));
    int32_t* snap = (int32_t*)malloc(sizeof(int32_t) * 3 * ((size_t)P.n_fmax + 1));
    int rc = (units && snap) ? OC_OK : OC_ENOMEM;
    for (int i = 0; i < n_units && rc == OC_OK; i++) {
        oc_unit* U = &units[i];
        U->A = (int8_t*)malloc((size_t)n_e * P.n_vmax);
        U->prog = (int32_t*)malloc(sizeof(int32_t) * 3 * ((size_t)P.n_fmax + 1));
        U->occ = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)P.occ_cap + 1));
        U->cand = (oc_cand*)malloc(sizeof(oc_cand) * ((size_t)P.occ_cap + 1));
        if (!U->A || !U->prog || !U->occ || !U->cand) { rc = OC_ENOMEM; break; }
        U->proc = procs ? (uint32_t)procs[i] : (uint32_t)i;
        U->strat = oc_proc_init(cfg, U->proc, &U->alpha_q, &U->beta_q);
        U->active = 1;
        int k = init_len ? init_len[i] : 0;
        if (k < 0 || k > P.n_fmax) { rc = OC_EINVAL; break; }
        rc = unit_replay(&P, U, init_prog ? init_prog + (size_t)i * prog_cap * 3 : NULL, k);
        U->epoch = init_epoch ? init_epoch[i] : 0;
        U->k0 = k;
    }

    if (rc == OC_OK) {
        if (!cfg->share_every) {
            run_all(&P, units, n_units, -1, n_threads);
        } else {
            for (uint32_t r = 0;; r++) {
                run_all(&P, units, n_units, (int)cfg->share_every, n_threads);
                int any = 0;
                for (int i = 0; i < n_units; i++) any |= units[i].active;
                if (!any) break;
                if (r < cfg->share_max_rounds && cfg->share_src_pm > 0) {
                    rc = share_round(&P, units, n_units, r, snap);
                    if (rc != OC_OK) break;
                }
            }
        }
    }

    if (rc == OC_OK) {
        for (int i = 0; i < n_units; i++) {
            oc_unit* U = &units[i];
            if (cost) cost[i] = U->cost;
            if (steps) steps[i] = U->t;
            if (executed) executed[i] = U->executed;
            if (epoch) epoch[i] = U->epoch;
            if (k0) k0[i] = U->k0;
            if (ops) ops[i] = U->ops;
            if (strat) strat[i] = U->strat;
            if (prog) {
                int32_t* dst = prog + (size_t)i * prog_cap * 3;
                memset(dst, 0, sizeof(int32_t) * 3 * (size_t)prog_cap);
                memcpy(dst, U->prog, sizeof(int32_t) * 3 * (size_t)U->t);
            }
        }
    }
    for (int i = 0; units && i < n_units; i++) {
        free(units[i].A); free(units[i].prog); free(units[i].occ); free(units[i].cand);
    }
    free(units);
    free(snap);
    free(A0w);
    return rc;
}

/* Size helpers for callers: the fresh-variable bound and the candidate bound
 * (every candidate accounts for at least two pair occurrences). */
int oc_bounds(const int8_t* A0, int n_e, int n_x, int32_t* n_fmax, int64_t* occ_cap)
{
    int64_t nnz0 = 0;
    for (int64_t i = 0; i < (int64_t)n_e * n_x; i++) nnz0 += A0[i] != 0;
    if (n_fmax) *n_fmax = (int32_t)((nnz0 - n_e) / 2);
    if (occ_cap) *occ_cap = oc_pair_occurrences(A0, n_e, n_x, n_x);
    return OC_OK;
}

/* ------------------------------------------------------------------------
 * Random flips of a scheme (Sec. 3.5.3).  A scheme of format (n, m, p : r)
 * is r products t, each the tensor product U_t (x) V_t (x) W_t of three
 * ternary vectors: U_t over the entries of A (n x m, row-major), V_t over B
 * (m x p), W_t over C (n x p); the system E_W of Sec. 3.2 is W transposed.
 * The paper takes its flips from the ternary flip graph of another work;
 * reading used here: when two products i != j share a factor up to sign,
 * X_j = s X_i (s = +1 or -1, X one of U, V, W, X_i nonzero), then
 *     X_i (x) Y_i (x) Z_i + X_j (x) Y_j (x) Z_j
 *   = X_i (x) (Y_i + s Y_j) (x) Z_i + X_j (x) Y_j (x) (Z_j - Z_i)     (h = 0)
 *   = X_i (x) Y_i (x) (Z_i + s Z_j) + X_j (x) (Y_j - Y_i) (x) Z_j     (h = 1)
 * with (Y, Z) = (V, W) for X = U, (U, W) for X = V and (U, V) for X = W.
 * Both sides are the same tensor, so the scheme stays a valid algorithm of
 * the same rank.  A flip is valid when the two changed vectors stay ternary
 * and nonzero.  Valid flips are numbered in the order (X, i, j, h).
 *
 * Variant v at iteration `iteration`: variant 0 is the scheme itself; any
 * other draws F = 1 + floor(u F_max / 2^32) from the Philox block
 * (v, FLIP|0|iteration|0, 0, 0) and applies F flips in turn, flip f being
 * valid flip number floor(u' n_valid / 2^32) of the current scheme, u' word
 * 0 of (v, FLIP|0|iteration|f+1, 0, 0); it stops early when no flip is
 * valid.  *n_done receives the flips applied.
 * ---------------------------------------------------------------------- */
static int8_t* flip_row(int8_t* M, int len, int t) { return M + (size_t)t * len; }

/* 1 if Y_a + s Y_b and the other update stay ternary and nonzero. */
static int row_sum_ok(const int8_t* a, const int8_t* b, int s, int len)
{
    int nz = 0;
    for (int k = 0; k < len; k++) {
        int v = a[k] + s * b[k];
        if (v < -1 || v > 1) return 0;
        nz |= v != 0;
    }
    return nz;
}

/* Sign s with X_j = s X_i (X_i nonzero), or 0. */
static int factor_sign(const int8_t* xi, const int8_t* xj, int len)
{
    int sp = 1, sm = 1, nz = 0;
    for (int k = 0; k < len; k++) {
        sp &= xj[k] == xi[k];
        sm &= xj[k] == -xi[k];
        nz |= xi[k] != 0;
    }
    if (!nz) return 0;
    return sp ? 1 : (sm ? -1 : 0);
}

/* Visit the valid flips in order; apply number `want` (>= 0) or count them
 * (want < 0).  Returns the count, or 1 when the flip was applied. */
static int64_t flips_visit(int8_t* M[3], const int len[3], int r, int64_t want)
{
    static const int other[3][2] = { { 1, 2 }, { 0, 2 }, { 0, 1 } };
    int64_t count = 0;
    for (int X = 0; X < 3; X++) {
        const int Y = other[X][0], Z = other[X][1];
        for (int i = 0; i < r; i++) {
            for (int j = 0; j < r; j++) {
                if (i == j) continue;
                const int s = factor_sign(flip_row(M[X], len[X], i), flip_row(M[X], len[X], j), len[X]);
                if (!s) continue;
                for (int h = 0; h < 2; h++) {
                    /* h = 0: Y_i += s Y_j, Z_j -= Z_i;  h = 1: Z_i += s Z_j, Y_j -= Y_i. */
                    const int P = h ? Z : Y, Q = h ? Y : Z;
                    int8_t* Pi = flip_row(M[P], len[P], i);
                    const int8_t* Pj = flip_row(M[P], len[P], j);
                    int8_t* Qj = flip_row(M[Q], len[Q], j);
                    const int8_t* Qi = flip_row(M[Q], len[Q], i);
                    if (!row_sum_ok(Pi, Pj, s, len[P]) || !row_sum_ok(Qj, Qi, -1, len[Q])) continue;
                    if (count == want) {
                        for (int k = 0; k < len[P]; k++) Pi[k] = (int8_t)(Pi[k] + s * Pj[k]);
                        for (int k = 0; k < len[Q]; k++) Qj[k] = (int8_t)(Qj[k] - Qi[k]);
                        return 1;
                    }
                    count++;
                }
            }
        }
    }
    return count;
}

int oc_flip_variant(const int8_t* U, const int8_t* V, const int8_t* W, int n, int m, int p, int r,
                    uint64_t seed, uint32_t variant, uint32_t iteration, uint32_t max_flips,
                    int8_t* outU, int8_t* outV, int8_t* outW, int32_t* n_done)
{
    if (n < 1 || m < 1 || p < 1 || r < 1 || max_flips < 1 || max_flips > 65534) return OC_EINVAL;
    const int len[3] = { n * m, m * p, n * p };
    memcpy(outU, U, (size_t)r * len[0]);
    memcpy(outV, V, (size_t)r * len[1]);
    memcpy(outW, W, (size_t)r * len[2]);
    int8_t* M[3] = { outU, outV, outW };
    int done = 0;
    if (variant != 0) {
        uint32_t u[4];
        draw(seed, variant, oc_domain_word(TAG_FLIP, 0, iteration, 0), 0, 0, u);
        const uint32_t F = 1 + scale_index(u[0], max_flips);
        for (uint32_t f = 0; f < F; f++) {
            const int64_t n_valid = flips_visit(M, len, r, -1);
            if (n_valid == 0) break;
            draw(seed, variant, oc_domain_word(TAG_FLIP, 0, iteration, f + 1), 0, 0, u);
            flips_visit(M, len, r, (int64_t)scale_index(u[0], (uint64_t)n_valid));
            done++;
        }
    }
    if (n_done) *n_done = done;
    return OC_OK;
}
