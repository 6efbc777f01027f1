"""ctypes wrapper of the plain CPU oracle (``cse_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to produce expected values.  The product library and
its Python binding never import this module.

Strategy ids: 0 g, 1 ga, 2 wr, 3 gr, 4 gi, 5 mix, 6 gp (Sec. 3.4, 3.5.1).
Programs are int32 triples (a, b, s): 1-based variable ids a < b and s = +-1;
the t-th substitution (t = 0, 1, ...) defines variable n_x + t + 1 as
x_a + s x_b (Sec. 3.2.1, 3.6).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcse_oracle.so")

STRATEGIES = ("g", "ga", "wr", "gr", "gi", "mix", "gp")
COMPONENTS = ("U", "V", "Wt")
TAG_REINIT = 5  # random-stream tag of the driver's restart draws


class OracleCfg(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("n_proc", ctypes.c_uint32),
        ("weights", ctypes.c_uint32 * 7),
        ("mix_weights", ctypes.c_uint32 * 4),
        ("proc0_greedy", ctypes.c_uint32),
        ("gr_p_q16", ctypes.c_uint32),
        ("step_cap", ctypes.c_uint32),
        ("share_every", ctypes.c_uint32),
        ("share_src_pm", ctypes.c_uint32),
        ("share_dst_pm", ctypes.c_uint32),
        ("share_max_rounds", ctypes.c_uint32),
        ("iteration", ctypes.c_uint32),
    ]


class OracleCand(ctypes.Structure):
    _fields_ = [("key", ctypes.c_uint32), ("c", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run the build entry point)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.oc_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.oc_philox4x32_10.restype = None
        L.oc_domain_word.argtypes = [ctypes.c_uint32] * 4
        L.oc_domain_word.restype = ctypes.c_uint32
        L.oc_naive.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oc_naive.restype = ctypes.c_int64
        L.oc_pair_occurrences.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oc_pair_occurrences.restype = ctypes.c_int64
        L.oc_analyse.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 P(ctypes.c_uint32), P(OracleCand)]
        L.oc_analyse.restype = ctypes.c_int
        L.oc_select_g.argtypes = [P(OracleCand), ctypes.c_int]
        L.oc_select_g.restype = ctypes.c_int
        L.oc_select_ga.argtypes = [P(OracleCand), ctypes.c_int, ctypes.c_uint32]
        L.oc_select_ga.restype = ctypes.c_int
        L.oc_select_wr.argtypes = [P(OracleCand), ctypes.c_int, ctypes.c_uint32]
        L.oc_select_wr.restype = ctypes.c_int
        L.oc_select_gi.argtypes = [P(OracleCand), ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, P(ctypes.c_int64), P(ctypes.c_int64)]
        L.oc_select_gi.restype = ctypes.c_int
        L.oc_select_gp.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int, ctypes.c_int, P(OracleCand),
                                   ctypes.c_int, ctypes.c_uint32, P(ctypes.c_int64)]
        L.oc_select_gp.restype = ctypes.c_int
        L.oc_substitute.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oc_substitute.restype = ctypes.c_int
        L.oc_proc_init.argtypes = [P(OracleCfg), ctypes.c_uint32, P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.oc_proc_init.restype = ctypes.c_int
        L.oc_run_pool.argtypes = [
            P(ctypes.c_int8), ctypes.c_int, ctypes.c_int, ctypes.c_int, P(OracleCfg),
            ctypes.c_int, P(ctypes.c_int32),
            P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32),
            P(ctypes.c_int64), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32),
            P(ctypes.c_int64), P(ctypes.c_int32), P(ctypes.c_int32), ctypes.c_int, ctypes.c_int]
        L.oc_run_pool.restype = ctypes.c_int
        L.oc_bounds.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int,
                                P(ctypes.c_int32), P(ctypes.c_int64)]
        L.oc_bounds.restype = ctypes.c_int
        L.oc_flip_variant.argtypes = [P(ctypes.c_int8), P(ctypes.c_int8), P(ctypes.c_int8), ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, P(ctypes.c_int8), P(ctypes.c_int8),
                                      P(ctypes.c_int8), P(ctypes.c_int32)]
        L.oc_flip_variant.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_cfg(seed=0, n_proc=1, weights=None, mix_weights=(8, 4, 2, 1), proc0_greedy=False,
             gr_p_q16=49152, step_cap=0, share_every=0, share_src_pm=0, share_dst_pm=0,
             share_max_rounds=0, iteration=0):
    """weights: dict strategy-name -> integer weight, or a 7-sequence."""
    cfg = OracleCfg()
    cfg.seed = seed
    cfg.n_proc = n_proc
    w = [0] * 7
    if weights is None:
        weights = {"gi": 1}
    if isinstance(weights, dict):
        for k, v in weights.items():
            w[STRATEGIES.index(k)] = int(v)
    else:
        w = [int(x) for x in weights]
    cfg.weights = (ctypes.c_uint32 * 7)(*w)
    cfg.mix_weights = (ctypes.c_uint32 * 4)(*[int(x) for x in mix_weights])
    cfg.proc0_greedy = int(bool(proc0_greedy))
    cfg.gr_p_q16 = gr_p_q16
    cfg.step_cap = step_cap
    cfg.share_every = share_every
    cfg.share_src_pm = share_src_pm
    cfg.share_dst_pm = share_dst_pm
    cfg.share_max_rounds = share_max_rounds
    cfg.iteration = iteration
    return cfg


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oc_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def domain_word(tag, comp, epoch, step):
    return int(lib().oc_domain_word(tag, comp, epoch, step))


def naive(A):
    A = np.ascontiguousarray(A, dtype=np.int8)
    return int(lib().oc_naive(_ptr(A, ctypes.c_int8), A.shape[0], A.shape[1], A.shape[1]))


def analyse(A):
    """Candidate list of system A: list of (a, b, s, c) in canonical order."""
    A = np.ascontiguousarray(A, dtype=np.int8)
    n_e, n_v = A.shape
    cap = int(lib().oc_pair_occurrences(_ptr(A, ctypes.c_int8), n_e, n_v, n_v)) + 1
    occ = np.zeros(cap, dtype=np.uint32)
    cand = (OracleCand * cap)()
    m = lib().oc_analyse(_ptr(A, ctypes.c_int8), n_e, n_v, n_v, _ptr(occ, ctypes.c_uint32), cand)
    out = []
    for i in range(m):
        k = cand[i].key
        out.append((k >> 16, (k >> 1) & 0x7FFF, -1 if k & 1 else 1, cand[i].c))
    return out


def _cands(cands):
    arr = (OracleCand * max(1, len(cands)))()
    for i, (a, b, s, c) in enumerate(cands):
        arr[i].key = (a << 16) | (b << 1) | (1 if s < 0 else 0)
        arr[i].c = c
    return arr


def select_g(cands):
    return int(lib().oc_select_g(_cands(cands), len(cands)))


def select_ga(cands, u):
    return int(lib().oc_select_ga(_cands(cands), len(cands), u))


def select_wr(cands, u):
    return int(lib().oc_select_wr(_cands(cands), len(cands), u))


def select_gi(cands, alpha_q, beta_q, seed=0, proc=0, comp=0, epoch=0, step=0):
    n_int = ctypes.c_int64()
    n_blk = ctypes.c_int64()
    i = lib().oc_select_gi(_cands(cands), len(cands), alpha_q, beta_q, seed, proc, comp, epoch, step,
                           ctypes.byref(n_int), ctypes.byref(n_blk))
    return int(i), int(n_int.value), int(n_blk.value)


def select_gp(A, alpha_q):
    """Greedy-Potential pick on system A (n_e x n_v, all columns current
    variables): (index into analyse(A), n_cols)."""
    A = np.ascontiguousarray(A, dtype=np.int8)
    n_e, n_v = A.shape
    W = np.zeros((n_e, n_v + 1), np.int8)
    W[:, :n_v] = A
    cands = analyse(A)
    n_cols = ctypes.c_int64()
    i = lib().oc_select_gp(_ptr(W, ctypes.c_int8), n_e, n_v, n_v + 1, _cands(cands), len(cands), alpha_q,
                           ctypes.byref(n_cols))
    return int(i), int(n_cols.value)


def substitute(A, a, b, s, k):
    """Apply x_k = x_a + s x_b in place on a copy; returns (new A, c)."""
    A = np.ascontiguousarray(A, dtype=np.int8).copy()
    n_e, n_v = A.shape
    if k > n_v:
        A = np.concatenate([A, np.zeros((n_e, k - n_v), np.int8)], axis=1)
        A = np.ascontiguousarray(A)
    c = lib().oc_substitute(_ptr(A, ctypes.c_int8), n_e, A.shape[1], a, b, s, k)
    return A, int(c)


def proc_init(cfg, proc):
    a = ctypes.c_uint32()
    b = ctypes.c_uint32()
    s = lib().oc_proc_init(ctypes.byref(cfg), proc, ctypes.byref(a), ctypes.byref(b))
    return int(s), int(a.value), int(b.value)


def bounds(A):
    A = np.ascontiguousarray(A, dtype=np.int8)
    nf = ctypes.c_int32()
    occ = ctypes.c_int64()
    lib().oc_bounds(_ptr(A, ctypes.c_int8), A.shape[0], A.shape[1], ctypes.byref(nf), ctypes.byref(occ))
    return int(nf.value), int(occ.value)


def run_pool(A, cfg, comp=0, procs=None, init_prog=None, init_len=None, init_epoch=None,
             n_threads=1):
    """Run units of one component.  Returns a dict of per-unit numpy arrays:
    cost, steps, executed, epoch, k0, ops, strat, prog (units x n_fmax x 3)."""
    A = np.ascontiguousarray(A, dtype=np.int8)
    n_e, n_x = A.shape
    n_fmax, _ = bounds(A)
    cap = max(1, n_fmax)
    if procs is None:
        n_units = cfg.n_proc
        procs_p = None
    else:
        procs = np.ascontiguousarray(procs, dtype=np.int32)
        n_units = len(procs)
        procs_p = _ptr(procs, ctypes.c_int32)
    out = {
        "cost": np.zeros(n_units, np.int64),
        "steps": np.zeros(n_units, np.int32),
        "executed": np.zeros(n_units, np.int32),
        "epoch": np.zeros(n_units, np.int32),
        "k0": np.zeros(n_units, np.int32),
        "ops": np.zeros(n_units, np.int64),
        "strat": np.zeros(n_units, np.int32),
        "prog": np.zeros((n_units, cap, 3), np.int32),
    }
    ip = il = ie = None
    if init_len is not None:
        init_prog = np.ascontiguousarray(init_prog, dtype=np.int32)
        assert init_prog.shape == (n_units, cap, 3)
        init_len = np.ascontiguousarray(init_len, dtype=np.int32)
        init_epoch = np.ascontiguousarray(init_epoch, dtype=np.int32)
        ip = _ptr(init_prog, ctypes.c_int32)
        il = _ptr(init_len, ctypes.c_int32)
        ie = _ptr(init_epoch, ctypes.c_int32)
    rc = lib().oc_run_pool(
        _ptr(A, ctypes.c_int8), n_e, n_x, comp, ctypes.byref(cfg), n_units, procs_p, ip, il, ie,
        _ptr(out["cost"], ctypes.c_int64), _ptr(out["steps"], ctypes.c_int32),
        _ptr(out["executed"], ctypes.c_int32), _ptr(out["epoch"], ctypes.c_int32),
        _ptr(out["k0"], ctypes.c_int32), _ptr(out["ops"], ctypes.c_int64),
        _ptr(out["strat"], ctypes.c_int32), _ptr(out["prog"], ctypes.c_int32), cap, n_threads)
    if rc != 0:
        raise ValueError(f"oracle run_pool failed with status {rc}")
    out["n_fmax"] = n_fmax
    return out


def _scale(u, n):
    """floor(u n / 2^32): an index in [0, n) from a 32-bit word."""
    return (int(u) * int(n)) >> 32


def run_driver(systems, cfg, reinit_pm=400, patience=10, max_iterations=100, n_threads=1):
    """The tool's outer iterations (Sec. 3.5.1, 3.5.2), run until the best
    total addition count has not changed for `patience` consecutive
    iterations (the convergence rule of Sec. 4) or `max_iterations` ran.

    Iteration i runs every process on every component: run_pool with
    cfg.iteration = i, so strategy, alpha and beta are drawn afresh and
    process 0 is greedy only in iteration 0.  Each component keeps its best
    program so far: a strictly lower cost replaces it; within an iteration
    the lowest (cost, process) wins.  Before iteration i >= 1 every unit draws
    Philox(process, REINIT|comp|i|0, 0, 0): with probability reinit_pm / 1000
    (word 0) it restarts from the first k = 1 + floor(u1 max(1, floor(3 L / 4))
    / 2^32) substitutions of that best program (word 1; L its length, no copy
    when L = 0), otherwise from the input system; either way its epoch goes
    up by one, so its step and coin draws are new.

    Returns a dict: iterations; totals, the best total after each iteration;
    best[c] = dict(cost, prog (L x 3 int32), iteration, proc); last[c] = the
    final iteration's run_pool output, with executed and ops summed over all
    iterations."""
    if not 1 <= max_iterations <= 1024:
        raise ValueError("max_iterations must be in 1..1024 (10-bit iteration field)")
    n = cfg.n_proc
    key = (cfg.seed & 0xFFFFFFFF, cfg.seed >> 32)
    best = [None] * len(systems)
    starts = [None] * len(systems)
    executed = [np.zeros(n, np.int64) for _ in systems]
    ops = [np.zeros(n, np.int64) for _ in systems]
    last = [None] * len(systems)
    totals = []
    unchanged = 0
    it = 0
    while True:
        cfg.iteration = it
        for c, A in enumerate(systems):
            if starts[c] is None:
                r = run_pool(A, cfg, comp=c, n_threads=n_threads)
            else:
                ip, il, ie = starts[c]
                r = run_pool(A, cfg, comp=c, init_prog=ip, init_len=il, init_epoch=ie, n_threads=n_threads)
            executed[c] += r["executed"]
            ops[c] += r["ops"]
            u = int(np.lexsort((np.arange(n), r["cost"]))[0])
            if best[c] is None or int(r["cost"][u]) < best[c]["cost"]:
                L = int(r["steps"][u])
                best[c] = dict(cost=int(r["cost"][u]), prog=r["prog"][u, :L].copy(), iteration=it, proc=u)
            last[c] = r
        total = sum(b["cost"] for b in best)
        unchanged = unchanged + 1 if totals and total == totals[-1] else 0
        totals.append(total)
        it += 1
        if unchanged >= patience or it >= max_iterations:
            break
        for c in range(len(systems)):
            r = last[c]
            cap = r["prog"].shape[1]
            ip = np.zeros((n, cap, 3), np.int32)
            il = np.zeros(n, np.int32)
            ie = (r["epoch"] + 1).astype(np.int32)
            bp = best[c]["prog"]
            L = len(bp)
            for p in range(n):
                w = philox4x32_10((p, domain_word(TAG_REINIT, c, it, 0), 0, 0), key)
                if L > 0 and _scale(w[0], 1000) < reinit_pm:
                    k = 1 + _scale(w[1], max(1, (3 * L) // 4))
                    ip[p, :k] = bp[:k]
                    il[p] = k
            starts[c] = (ip, il, ie)
    for c in range(len(systems)):
        last[c] = dict(last[c], executed=executed[c], ops=ops[c])
    return dict(iterations=it, totals=totals, best=best, last=last)



def flip_variant(U, V, W, n, m, p, seed, variant, iteration, max_flips):
    """Variant `variant` of the scheme (U r x nm, V r x mp, W r x np; W holds
    the products' C coefficients, W^T is the E_W system) at `iteration`:
    (U', V', W', flips applied)."""
    U, V, W = (np.ascontiguousarray(x, dtype=np.int8) for x in (U, V, W))
    r = U.shape[0]
    assert U.shape == (r, n * m) and V.shape == (r, m * p) and W.shape == (r, n * p)
    oU, oV, oW = np.zeros_like(U), np.zeros_like(V), np.zeros_like(W)
    done = ctypes.c_int32()
    rc = lib().oc_flip_variant(_ptr(U, ctypes.c_int8), _ptr(V, ctypes.c_int8), _ptr(W, ctypes.c_int8), n, m, p, r,
                               seed, variant, iteration, max_flips, _ptr(oU, ctypes.c_int8),
                               _ptr(oV, ctypes.c_int8), _ptr(oW, ctypes.c_int8), ctypes.byref(done))
    if rc != 0:
        raise ValueError(f"oracle flip_variant failed with status {rc}")
    return oU, oV, oW, int(done.value)
