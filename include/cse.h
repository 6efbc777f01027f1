/*
 * cse.h -- C ABI of libcse, an MI355X (gfx950) engine that runs many
 * independent randomized common-subexpression-elimination (CSE) processes
 * over the ternary linear forms of fast matrix-multiplication schemes, after
 * A. I. Perminov, "Parallel Heuristic Exploration for Additive Complexity
 * Reduction in Fast Matrix Multiplication" (arXiv 2512.13365).
 *
 * Terms.
 *   system     n_e linear forms over n_x variables with coefficients in
 *              {-1, 0, 1} (Sec. 3.2.1), given as an int8 row-major matrix,
 *              rows = forms, columns = variables.  No row may be all zero.
 *   scheme     the three systems of a scheme (Sec. 3.2): U (forms over the
 *              entries of A), V (over the entries of B) and W^T (one form per
 *              entry of C over the products).  Components 0, 1, 2.
 *   process    one reduction process of Sec. 3.5.1: a strategy, alpha and
 *              beta, applied to each component independently.
 *   unit       one component reduced by one process.  Unit results are a
 *              pure function of (system, run configuration, process index):
 *              they do not depend on batching or on other jobs.
 *   program    the substitutions of a unit in order, as int32 triples
 *              (a, b, s): 1-based variable ids a < b, s = +1 or -1.  The t-th
 *              triple (t = 0, 1, ...) defines fresh variable n_x + t + 1 as
 *              x_a + s x_b (Sec. 3.2.1, 3.6).
 *   cost       additions of a unit: n_f + naive(final forms) (Sec. 3.2.1).
 *
 * Conventions.  Every function returns a status (0 = CSE_OK, < 0 = error)
 * and never aborts or throws across the ABI.  Input arrays are copied; the
 * caller keeps ownership.  Output arrays are caller-allocated host memory.
 * A context serves one host thread at a time (no internal locking).
 * `stream` arguments are hipStream_t values passed as void* (NULL = the
 * default stream).  Device work is asynchronous until cse_wait or any
 * cse_get_* call, which block until the job is done.
 */
#ifndef CSE_H_
#define CSE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSE_OK         0
#define CSE_EINVAL    (-1)  /* bad shape, entry outside {-1,0,1}, zero row, bad configuration */
#define CSE_ENOMEM    (-2)  /* device memory or LDS footprint exceeds capacity */
#define CSE_ERANGE    (-3)  /* caller buffer too small, or a size limit exceeded */
#define CSE_EHIP      (-4)  /* HIP runtime error; see cse_last_error */
#define CSE_EBUSY     (-5)  /* job not finished (cse_poll) */
#define CSE_ENOENT    (-6)  /* unknown scheme or job id */
#define CSE_ECANCELED (-7)  /* job was cancelled */

/* Strategy ids, the index into cse_run_cfg.weights (Sec. 3.4.1-3.4.3,
 * 3.5.1; Greedy-Potential of Sec. 2 and 3.4). */
#define CSE_STRAT_G   0   /* greedy: highest frequency */
#define CSE_STRAT_GA  1   /* greedy-alternative: uniform among maximal */
#define CSE_STRAT_WR  2   /* weighted-random: probability ~ c - 1 */
#define CSE_STRAT_GR  3   /* greedy-random: ga with prob gr_p, else wr */
#define CSE_STRAT_GI  4   /* greedy-intersections (Sec. 3.4.2) */
#define CSE_STRAT_MIX 5   /* per step one of gi/ga/gr/wr by mix_weights */
#define CSE_STRAT_GP  6   /* greedy-potential: c - 1 plus alpha x new pairs after a trial */

/* Counting paths for the pair counts of the Analysis step (Algorithm 1).
 * All paths give identical results. */
#define CSE_COUNT_AUTO     0
#define CSE_COUNT_POPCOUNT 1   /* wavefront popcount over column bitsets */
#define CSE_COUNT_MFMA     2   /* int8 MFMA Gram product for the first count */

/* Layout of a component's unit state (results never depend on it). */
#define CSE_LAYOUT_HBM     1   /* bulk state in per-unit HBM slots instead of LDS */
#define CSE_LAYOUT_RANGE   2   /* gi over per-variable ranges instead of masks */
#define CSE_LAYOUT_LDS_TABLES 4 /* with HBM | RANGE only: gi's per-step range tables in LDS
                                 * (chosen explicitly; loading and cse_autotune never pick it) */
/* Waves per unit (threads per process), bits 3-4 of a layout: one wave
 * (neither bit), two or four; more than one only with CSE_LAYOUT_RANGE.
 * Loading gives HBM | RANGE components four waves and the others one;
 * cse_autotune times one, two and four for the range form. */
#define CSE_LAYOUT_WAVES_SHIFT 3
#define CSE_LAYOUT_WAVES2  8
#define CSE_LAYOUT_WAVES4  16

/* States of a job submitted to a server. */
#define CSE_JOB_QUEUED  0   /* waiting for admission */
#define CSE_JOB_RUNNING 1   /* admitted; advances one round per tick */
#define CSE_JOB_DONE    2   /* every unit finished; results readable */
#define CSE_JOB_FAILED  3   /* its device state could not be allocated at
                               admission; no results; release it */

typedef struct cse_ctx cse_ctx;
typedef struct cse_server cse_server;

/* Run configuration (Sec. 3.5).  Zero-initialise and set what is needed. */
typedef struct {
    uint64_t seed;             /* key of every random draw */
    uint32_t n_proc;           /* processes; unit results depend on the index */
    uint32_t weights[7];       /* integer strategy weights, by CSE_STRAT_* */
    uint32_t mix_weights[4];   /* mix: gi, ga, gr, wr (paper: 8, 4, 2, 1) */
    uint32_t proc0_greedy;     /* process 0 runs g (Sec. 3.5.1) */
    uint32_t gr_p_q16;         /* greedy-random: P(ga) in 2^-16 units (<= 65536) */
    uint32_t step_cap;         /* maximal program length; 0 = none */
    uint32_t share_every;      /* steps per sharing round; 0 = no sharing */
    uint32_t share_src_pm;     /* sources: first ceil(N pm/1000) by (cost, process) */
    uint32_t share_dst_pm;     /* P(an active non-source unit is a target), per mille */
    uint32_t share_max_rounds; /* at most this many sharing events (<= 1023) */
    uint32_t iteration;        /* outer iteration (keys per-process draws) */
    uint32_t count_path;       /* CSE_COUNT_* */
    uint32_t reserved[3];      /* must be 0 */
} cse_run_cfg;

/* Library ABI version (this header: 1). */
int32_t cse_version(void);

/* Create a context on HIP device `device`.  *out receives the handle. */
int32_t cse_ctx_create(int32_t device, cse_ctx** out);
void cse_ctx_destroy(cse_ctx* ctx);
/* Text of the last error on this context (static storage of the context). */
const char* cse_last_error(const cse_ctx* ctx);

/* Load one system (Sec. 3.2.1) as a one-component scheme.  A is rows x cols
 * int8 row-major, entries in {-1, 0, 1}, no zero row; rows <= 512 and
 * cols + floor((nnz - rows) / 2) < 32768.  Returns CSE_EINVAL otherwise. */
int32_t cse_system_load(cse_ctx* ctx, const int8_t* A, int32_t rows, int32_t cols,
                        int32_t* scheme_id);

/* Load a scheme's three systems U (u_rows x u_cols), V and W^T (Sec. 3.2),
 * with the same rules as cse_system_load for each. */
int32_t cse_scheme_load(cse_ctx* ctx,
                        const int8_t* U, int32_t u_rows, int32_t u_cols,
                        const int8_t* V, int32_t v_rows, int32_t v_cols,
                        const int8_t* Wt, int32_t w_rows, int32_t w_cols,
                        int32_t* scheme_id);

/* cse_scheme_load from device memory: U, V and W^T are device pointers
 * (HIP), read on `stream` after the work already queued there, copied (the
 * caller keeps them) and validated and sized on the device; V and W^T both
 * NULL loads U alone as a one-component scheme.  Same rules and errors as
 * cse_scheme_load (CSE_ENOMEM also when a system's variable lists cannot
 * fit a workgroup's LDS); blocking. */
int32_t cse_scheme_load_device(cse_ctx* ctx,
                               const int8_t* U, int32_t u_rows, int32_t u_cols,
                               const int8_t* V, int32_t v_rows, int32_t v_cols,
                               const int8_t* Wt, int32_t w_rows, int32_t w_cols,
                               void* stream, int32_t* scheme_id);

/* Shape of a loaded scheme: *n_comp components; info (4 per component):
 * n_e, n_x, n_fmax (the fresh-variable bound floor((nnz - n_e) / 2)), and
 * the naive count (Sec. 3.2.1). */
int32_t cse_scheme_info(cse_ctx* ctx, int32_t scheme_id, int32_t* n_comp, int32_t info[12]);
/* Free a scheme; CSE_EBUSY while a job of it has not been released. */
int32_t cse_scheme_free(cse_ctx* ctx, int32_t scheme_id);

/* Query (layout < 0) or set the layout (CSE_LAYOUT_* bits) of component
 * `comp`; *current (may be NULL) receives the layout in effect before the
 * call.  Loading picks a layout from the system's size: the range form of gi
 * for large candidate sets, and state in HBM with the range form when the
 * state would leave room in a CU's 160 KB of LDS for fewer than four units
 * (those run on four waves).  Valid layouts: 0..3 and HBM | RANGE |
 * LDS_TABLES, each range layout with or without CSE_LAYOUT_WAVES2 or
 * CSE_LAYOUT_WAVES4 (several waves only for systems of at most 2047
 * variables, n_x + floor((nnz - rows) / 2)); CSE_EINVAL otherwise.  CSE_EBUSY while a job of the
 * scheme exists; CSE_ENOMEM if the unit's LDS share does not fit a
 * workgroup.  Unit results are the same in every layout. */
int32_t cse_scheme_layout(cse_ctx* ctx, int32_t scheme_id, int32_t comp, int32_t layout, int32_t* current);

/* Pick each component's fastest layout by timing bounded probe runs of
 * `cfg` (at most 1024 processes, 32 steps each, no sharing) on `stream`, for
 * every layout 0..3 that fits (the mask form of gi only where the input's masks
 * fit their capacity), the range layouts on one, two and four waves per
 * unit; layouts[c] (may be NULL) receives the choice.
 * Blocking.  CSE_EBUSY while a job of the scheme exists. */
int32_t cse_autotune(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, void* stream, int32_t layouts[3]);

/* Launch n_proc processes on every component of a scheme (Algorithm 1 per
 * unit, strategies of Sec. 3.4, sharing rounds of Sec. 3.5.2 when
 * share_every > 0).  Asynchronous on `stream`; *job_id receives the job. */
int32_t cse_launch(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, void* stream,
                   int32_t* job_id);

/* Launch n jobs (scheme_ids[i] with cfgs[i]) as one batch: the units of
 * all their components share device launches (one launch per row-word
 * count), and sharing rounds, if any, advance all jobs together.  Every unit
 * result equals that of the separate cse_launch of its job.  Unit finish
 * times count from the batch start. */
int32_t cse_launch_batch(cse_ctx* ctx, const int32_t* scheme_ids, const cse_run_cfg* cfgs,
                         int32_t n, void* stream, int32_t* job_ids);

/* Run a job again on its own device buffers, optionally with a new
 * configuration (NULL = the same one; n_proc and whether it shares must not
 * change).  A job launched in a batch reruns the whole batch, and then cfg
 * must be NULL.  Results of the earlier run are overwritten.  No device
 * memory is allocated, so the launches can be timed on `stream` without
 * allocation in between; on the same stream the call does not block. */
int32_t cse_relaunch(cse_ctx* ctx, int32_t job_id, const cse_run_cfg* cfg, void* stream);

/* Continue a cancelled job from where its units stopped: every unit keeps
 * its program prefix, epoch and counters, and the draws of a unit depend
 * only on its process, epoch and step (Sec. 3.5.1), so the final results
 * equal those of a run that was never cancelled.  A job launched in a batch
 * resumes its whole batch (units that finished are unchanged; on a finished
 * job the call changes nothing).  CSE_EINVAL for server and driver jobs and
 * for jobs with sharing rounds (their round schedule is not kept across a
 * cancellation).  Waits for the earlier launch; allocates no device memory;
 * on `stream` the call does not block. */
int32_t cse_resume(cse_ctx* ctx, int32_t job_id, void* stream);

/* The tool's outer iterations (Sec. 3.5.1, 3.5.2) and its convergence rule
 * (Sec. 4).  Zero-initialise and set the three fields. */
typedef struct {
    uint32_t reinit_pm;       /* processes restarted from the best prefix, per mille (paper: 400) */
    uint32_t patience;        /* stop once the best total is unchanged this many iterations (paper: 10) */
    uint32_t max_iterations;  /* at most this many iterations, 1..1024 */
    uint32_t reserved;        /* must be 0 */
} cse_driver_cfg;

/* Run a job of `cfg` (cfg->iteration must be 0) for iterations i = 0, 1, ...
 * Iteration i runs every unit to completion, with cfg's sharing rounds if
 * any, its strategy, alpha and beta drawn for iteration i (process 0 runs g
 * in iteration 0 only, when proc0_greedy is set).  After each iteration each
 * component keeps its best program so far: the lowest (cost, process) of
 * the iteration replaces it when its cost is strictly lower.  Before
 * iteration i >= 1 every unit restarts, with its epoch advanced: with
 * probability reinit_pm / 1000 (Philox word 0 of (process,
 * REINIT|comp|i|0, 0, 0)) from the first k = 1 + floor(u1 max(1,
 * floor(3 L / 4)) / 2^32) substitutions of that best program (L its length;
 * none when L = 0), otherwise from the input.  The run stops when the sum of
 * the component bests has not changed for `patience` iterations (0: after
 * the first), or after max_iterations.  Blocking.  *job_id receives the
 * job (release it with cse_job_release); its unit results are those of the
 * last iteration, with executed and ops summed over all iterations, and
 * finish times counted from the start of iteration 0.  *iterations (may be
 * NULL) receives the number of iterations run.  *job_id is written as soon
 * as the job exists, before iteration 0 starts, so another thread may read
 * it and call cse_cancel, which stops the run after the current iteration
 * (its units stop early): CSE_ECANCELED, with the job and its bests kept.
 * Errors after iteration 0 started leave *job_id set; if iteration 0 cannot
 * be started the job is dropped and *job_id is reset to -1. */
int32_t cse_run_driver(cse_ctx* ctx, int32_t scheme_id, const cse_run_cfg* cfg, const cse_driver_cfg* dcfg,
                       void* stream, int32_t* job_id, int32_t* iterations);

/* The best program so far of component `comp` of a driver job: triples
 * (cap x 3 int32, as in cse_get_program), its length, cost, and the
 * iteration and process that found it; CSE_ERANGE with *needed set when
 * cap is too small. */
int32_t cse_driver_best(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t* triples, int32_t cap,
                        int32_t* n_fresh, int32_t* cost, int32_t* iteration, int32_t* proc, int32_t* needed);

/* Per iteration of a driver job: the best total (sum of the component
 * bests) after it, and the host time in ns from the start of
 * cse_run_driver to its end.  *n receives the iteration count; totals and
 * elapsed_ns (either may be NULL; both NULL only counts) receive *n
 * entries; CSE_ERANGE when cap < *n. */
int32_t cse_driver_totals(cse_ctx* ctx, int32_t job_id, int32_t* totals, uint64_t* elapsed_ns, int32_t cap,
                          int32_t* n);

/* The component-wise hybrid over several finished jobs of one scheme
 * (Sec. 4: the best U, V and W^T may come from different runs or strategy
 * mixes; jobs of different scheme ids give CSE_EINVAL): for each component,
 * the lowest cost
 * over the jobs, the job and the process holding it (ties: the earlier job
 * in the list, then the lower process).  A driver job counts with its best
 * program so far (read it with cse_driver_best), any other job with its
 * best unit (cse_get_program with that process).  Absent components: -1.
 * best_job and best_proc may be NULL.  Blocking. */
int32_t cse_hybrid_best(cse_ctx* ctx, const int32_t* job_ids, int32_t n, int32_t best_cost[3], int32_t best_job[3],
                        int32_t best_proc[3]);

/* Non-blocking: *done = 1 when the job's device work has completed, else 0.
 * best_cost (3 entries, may be NULL) receives, once done, the lowest cost
 * over the units of each component (the best of each pool, Sec. 3.5, and
 * Sec. 4's per-component bests); -1 for absent components and while the
 * job runs.  Computing it waits briefly on the job's stream. */
int32_t cse_poll(cse_ctx* ctx, int32_t job_id, int32_t* done, int32_t best_cost[3]);
/* Block until the job is done.  CSE_ECANCELED if it was cancelled (its
 * results are still readable). */
int32_t cse_wait(cse_ctx* ctx, int32_t job_id);
/* Stop a job early.  A running launch checks the request every 256
 * selection steps of each unit (shorter units run to their end); a unit
 * that stops keeps a consistent state whose program is a prefix of the one
 * it would have built.  A queued server
 * job leaves the queue; a running server job stops after the current round.
 * A job whose device work already completed is left as it is.  Returns
 * CSE_OK once the request is recorded; cse_wait then returns CSE_ECANCELED.
 * A relaunch or cse_resume clears the request.  This is the one call that may run on
 * another thread while cse_wait or cse_run_driver blocks on the same job
 * (a driver run stops after its current iteration); otherwise a context is
 * used by one thread at a time. */
int32_t cse_cancel(cse_ctx* ctx, int32_t job_id);

/* Per-unit results of component `comp` for processes 0..n-1 (n = n_proc);
 * any pointer may be NULL.  cost: Sec. 3.2.1 cost; steps: program length;
 * executed: selection steps run (replays of shared prefixes excluded);
 * epoch: times the unit restarted from a shared prefix; k0: program length
 * right after the last restart (0 if none); ops: algorithmic work tally;
 * strat: the process strategy (CSE_STRAT_*); finish: device wall-clock ticks
 * from job start until the unit finished. */
int32_t cse_get_unit_results(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t n,
                             int32_t* cost, int32_t* steps, int32_t* executed,
                             int32_t* epoch, int32_t* k0, int64_t* ops, int32_t* strat,
                             uint64_t* finish);

/* Programs of all n units of component `comp`: triples is n x cap x 3
 * int32; entries past a unit's length are zero.  cap must be >= n_fmax. */
int32_t cse_get_programs(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t n,
                         int32_t* triples, int32_t cap);

/* Program of one unit (proc = -1: the lowest-cost unit, ties to the lower
 * process index).  triples holds cap x 3 int32; *n_fresh and *cost receive
 * its length and cost; if cap < length, returns CSE_ERANGE and sets *needed. */
int32_t cse_get_program(cse_ctx* ctx, int32_t job_id, int32_t comp, int32_t proc,
                        int32_t* triples, int32_t cap, int32_t* n_fresh, int32_t* cost,
                        int32_t* needed);

/* Device time of step-kernel launches, per kernel class. */
typedef struct {
    int32_t row_words;   /* W: rows <= 64 W */
    int32_t layout;      /* CSE_LAYOUT_* of the components it ran */
    int32_t launches;    /* launches timed */
    int32_t reserved;
    uint64_t device_ns;  /* summed time between the HIP events around them */
} cse_kernel_time;

/* Kernel timing on a context (off by default).  While on, every step-kernel
 * launch is bracketed by two HIP events on the stream it runs on, and the
 * rounds of sharing jobs and servers are launched directly rather than
 * replayed as a captured graph (so their launches can be timed). */
int32_t cse_ctx_set_timing(cse_ctx* ctx, int32_t on);

/* The timed launches of the batch (or server) that runs job_id, summed per
 * kernel class (row words, layout) over its runs since the last reset;
 * waits for a non-server batch to finish.  *n receives the number of
 * classes; out (may be NULL) receives them when cap >= *n, else
 * CSE_ERANGE.  reset != 0 clears the sums after reading. */
int32_t cse_kernel_times(cse_ctx* ctx, int32_t job_id, cse_kernel_time* out, int32_t cap, int32_t* n,
                         int32_t reset);

/* Timing of a finished job: device ticks from job start to the last unit's
 * finish, and the tick rate in Hz. */
int32_t cse_job_timing(cse_ctx* ctx, int32_t job_id, uint64_t* ticks, uint64_t* tick_hz);

/* Free a job's device memory (the other jobs of its batch keep theirs).
 * Server jobs are released with cse_server_release. */
int32_t cse_job_release(cse_ctx* ctx, int32_t job_id);

/* ---- Serving: continuous batching of reduction jobs -------------------
 * A server admits submitted jobs first come, first served while the device
 * state of the admitted, unreleased jobs fits max_state_bytes, and advances
 * every admitted job by one round per tick: one launch per row-word class
 * covers the units of all admitted jobs, so a job admitted between ticks
 * joins the next launch.  A round is at most share_every selection steps
 * per unit for a job that shares (then its sharing event), else at most
 * round_steps.  Every job's results equal those of its own cse_launch. */

/* Create a server on ctx issuing its work on `stream`; round_steps >= 1. */
int32_t cse_server_create(cse_ctx* ctx, uint64_t max_state_bytes, uint32_t round_steps, void* stream,
                          cse_server** out);
/* Queue a job (not yet admitted).  CSE_ENOMEM if it alone exceeds the
 * server's budget or its unit state cannot fit a workgroup's LDS. */
int32_t cse_server_submit(cse_server* s, int32_t scheme_id, const cse_run_cfg* cfg, int32_t* job_id);
/* Admit what fits, run one round of every admitted job, retire finished
 * jobs; blocks until the round's device work is done.  Reports how many
 * jobs are running and queued afterwards.  A job whose device state cannot
 * be allocated at admission leaves the queue as CSE_JOB_FAILED (reading its
 * results gives CSE_ENOMEM) and the other jobs go on. */
int32_t cse_server_tick(cse_server* s, int32_t* n_running, int32_t* n_queued);
/* State (CSE_JOB_*) and host steady-clock times in ns of submission,
 * admission and completion (0 until reached). */
int32_t cse_server_job_info(cse_server* s, int32_t job_id, int32_t* state, uint64_t times_ns[3]);
/* Free a done job's device memory and return it to the admission budget.
 * Results are read with cse_get_* while the job is done and unreleased. */
int32_t cse_server_release(cse_server* s, int32_t job_id);
/* Destroy the server and every job it owns. */
void cse_server_destroy(cse_server* s);

/* ---------------------------------------------------------------------------
 * Random flips of a scheme (Sec. 3.5.3).  A scheme of format (n, m, p : r) is
 * r products t = U_t (x) V_t (x) W_t: U (r x nm) over the entries of A
 * (n x m), V (r x mp) over B (m x p), W (r x np) over C (n x p), all
 * row-major and ternary; its systems E_U, E_V, E_W of Sec. 3.2 are U, V and
 * W transposed.  A flip rewrites two products that share a factor up to
 * sign, X_j = s X_i (X one of U, V, W), into two others computing the same
 * tensor: X_i (x) (Y_i + s Y_j) (x) Z_i + X_j (x) Y_j (x) (Z_j - Z_i), or
 * the same with Y and Z exchanged ((Y, Z) = (V, W), (U, W), (U, V) for
 * X = U, V, W); it is valid when both changed vectors stay ternary and
 * nonzero, so every variant computes C = A B with the same rank.  Valid
 * flips are numbered in the order (X, i, j, Y-or-Z first).  Variant 0 is
 * the scheme itself; variant v > 0 at iteration `it` applies
 * 1 + floor(u max_flips / 2^32) flips (u: word 0 of Philox (v,
 * FLIP|0|it|0, 0, 0), FLIP = 6 in the tag nibble), flip f taking valid flip
 * floor(u' n_valid / 2^32), u' word 0 of (v, FLIP|0|it|f+1, 0, 0), and
 * stops early when none is valid.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n, m, p;      /* format: A n x m, B m x p, C n x p (each <= 4096 entries) */
    int32_t n_variants;   /* M (paper: 32), variant 0 the scheme itself */
    int32_t max_flips;    /* flips per variant uniform in [1, max_flips], <= 65534 */
    int32_t reserved;     /* must be 0 */
} cse_flip_cfg;

/* The M variants of one iteration, generated on the device from host
 * arrays (copied): outU (M x r x nm), outV (M x r x mp), outW (M x r x np)
 * host arrays; n_flips (M, may be NULL) receives the flips applied.
 * CSE_EINVAL for a bad format or non-ternary coefficients, CSE_ENOMEM when
 * r (nm + mp + np) bytes exceed a workgroup's LDS.  Blocking. */
int32_t cse_flip_variants(cse_ctx* ctx, const int8_t* U, const int8_t* V, const int8_t* W, int32_t rank,
                          const cse_flip_cfg* fcfg, uint64_t seed, uint32_t iteration,
                          int8_t* outU, int8_t* outV, int8_t* outW, int32_t* n_flips);

/* The random-flip mode (Sec. 3.5.3).  Iteration it (from 0) generates the M
 * variants of iteration it (seed cfg->seed) and reduces each of them with
 * cfg->n_proc processes, variant v with seed cfg->seed + v and cfg's
 * iteration field set to it, all in one batch (sharing rounds as cfg says).
 * A variant's total is the sum of its three component bests (components
 * only combine within one variant); the lowest total over the variants of
 * an iteration (ties: lower v) replaces the best so far when strictly lower.
 * Stops when the best total has not changed for `patience` iterations or
 * after max_iterations (<= 1024).  *run_id receives the run (read it with
 * cse_flip_best / cse_flip_program, free it with cse_flip_release);
 * *iterations (may be NULL) the iterations run.  Blocking. */
int32_t cse_run_flips(cse_ctx* ctx, const int8_t* U, const int8_t* V, const int8_t* W, int32_t rank,
                      const cse_flip_cfg* fcfg, const cse_run_cfg* cfg, int32_t patience, int32_t max_iterations,
                      void* stream, int32_t* run_id, int32_t* iterations);

/* The best variant of a flip run: its U, V, W (host arrays of the input's
 * sizes; each may be NULL), component costs, variant and iteration, and the
 * best total after each iteration (totals, cap entries; may be NULL;
 * CSE_ERANGE when cap is too small), *n_iter the iteration count. */
int32_t cse_flip_best(cse_ctx* ctx, int32_t run_id, int8_t* U, int8_t* V, int8_t* W, int32_t best_cost[3],
                      int32_t* variant, int32_t* iteration, int32_t* totals, int32_t cap, int32_t* n_iter);

/* Program of component comp (0 U, 1 V, 2 W^T) of the best variant, as in
 * cse_get_program. */
int32_t cse_flip_program(cse_ctx* ctx, int32_t run_id, int32_t comp, int32_t* triples, int32_t cap,
                         int32_t* n_fresh, int32_t* needed);

/* Free a flip run's results. */
int32_t cse_flip_release(cse_ctx* ctx, int32_t run_id);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * system reduced by cfg->n_proc processes exactly as cse_system_load +
 * cse_launch would (component index `comp` keys the random draws: 0 for a
 * lone system, 0 / 1 / 2 for U / V / W^T of a scheme, whose units then equal
 * that component's units of cse_scheme_load + cse_launch), with every
 * working buffer (the input's bitsets and candidate lists, per-unit state,
 * the launch table) in a static device array of CSE_STATIC_SCRATCH_BYTES
 * per GPU instead of allocated memory.  Calls no hipMalloc or hipFree.
 *   A          device pointer, rows x cols int8 row-major; read on `stream`
 *              after the work queued there, not kept.  Rules of
 *              cse_system_load.
 *   cfg        as for cse_launch, without sharing (share_every, share_src_pm
 *              or share_max_rounds 0) and not CSE_COUNT_MFMA.
 *   cost, length
 *              device int32[n_proc]: each unit's additions and program
 *              length.
 *   prog       device uint32[n_proc x prog_cap]: unit p's program at
 *              prog[p prog_cap ...], entry t = a << 16 | b << 1 | (s < 0)
 *              (a < b 1-based ids, s the sign; the t-th fresh variable is
 *              n_x + t + 1 = x_a + s x_b).  Entries past length are unset.
 *   needed     (may be NULL) receives max(1, floor((nnz - rows) / 2)), the
 *              smallest prog_cap; a smaller prog_cap gives CSE_ERANGE
 *              before any unit runs.
 * CSE_ENOMEM when the working set (about 36 B per process, 6 B per pair
 * occurrence of the input for its candidate lists, and per-process HBM
 * state for systems that need it) exceeds CSE_STATIC_SCRATCH_BYTES.  Blocking: returns
 * once the units are done.  Every call on one GPU uses that GPU's array and
 * overwrites what the previous call left there; calls that overlap on one
 * GPU (from several threads or contexts) race and must be serialised by the
 * caller. */
#define CSE_STATIC_SCRATCH_BYTES (64u << 20)
int32_t cse_reduce_static(cse_ctx* ctx, const int8_t* A, int32_t rows, int32_t cols, int32_t comp,
                          const cse_run_cfg* cfg, void* stream, int32_t* cost, int32_t* length, uint32_t* prog,
                          int32_t prog_cap, int32_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* CSE_H_ */
