"""ctypes binding of libcse (include/cse.h): the same entry points, argument
marshalling only.  Every step of the reduction runs in the library's HIP
kernels; this module never computes a result itself and raises if the
built library is missing.

Typical use::

    ctx = cse_ctx_create(0)
    sid = cse_scheme_load(ctx, U, V, Wt)
    job = cse_launch(ctx, sid, cse_run_cfg(n_proc=4096, weights={"gi": 1}), stream)
    res = cse_get_unit_results(ctx, job, comp=0)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcse.so")

STRATEGIES = ("g", "ga", "wr", "gr", "gi", "mix", "gp")
CSE_COUNT_AUTO, CSE_COUNT_POPCOUNT, CSE_COUNT_MFMA = 0, 1, 2
CSE_LAYOUT_HBM, CSE_LAYOUT_RANGE, CSE_LAYOUT_LDS_TABLES = 1, 2, 4
CSE_LAYOUT_WAVES_SHIFT, CSE_LAYOUT_WAVES2, CSE_LAYOUT_WAVES4 = 3, 8, 16

STATUS = {0: "CSE_OK", -1: "CSE_EINVAL", -2: "CSE_ENOMEM", -3: "CSE_ERANGE", -4: "CSE_EHIP",
          -5: "CSE_EBUSY", -6: "CSE_ENOENT", -7: "CSE_ECANCELED"}

# Every symbol declared in include/cse.h.
EXPORTS = ("cse_version", "cse_ctx_create", "cse_ctx_destroy", "cse_last_error", "cse_system_load",
           "cse_scheme_load", "cse_scheme_load_device", "cse_scheme_info", "cse_scheme_free", "cse_scheme_layout",
           "cse_autotune",
           "cse_launch", "cse_launch_batch",
           "cse_relaunch", "cse_resume", "cse_poll", "cse_wait", "cse_cancel", "cse_get_unit_results",
           "cse_get_programs",
           "cse_get_program", "cse_job_timing", "cse_job_release", "cse_server_create", "cse_server_submit",
           "cse_server_tick", "cse_server_job_info", "cse_server_release", "cse_server_destroy",
           "cse_run_driver", "cse_driver_best", "cse_driver_totals", "cse_hybrid_best", "cse_ctx_set_timing",
           "cse_kernel_times", "cse_flip_variants", "cse_run_flips", "cse_flip_best", "cse_flip_program",
           "cse_flip_release", "cse_reduce_static")
CSE_JOB_QUEUED, CSE_JOB_RUNNING, CSE_JOB_DONE, CSE_JOB_FAILED = 0, 1, 2, 3


class CseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CseKernelTime(ctypes.Structure):
    _fields_ = [("row_words", ctypes.c_int32), ("layout", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("device_ns", ctypes.c_uint64)]


class CseFlipCfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("p", ctypes.c_int32),
                ("n_variants", ctypes.c_int32), ("max_flips", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CseRunCfg(ctypes.Structure):
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
        ("count_path", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 3),
    ]


class CseDriverCfg(ctypes.Structure):
    _fields_ = [
        ("reinit_pm", ctypes.c_uint32),
        ("patience", ctypes.c_uint32),
        ("max_iterations", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcse.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcse.so not built at {path}: run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    i32, u32, vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p
    L.cse_version.restype = i32
    L.cse_ctx_create.argtypes = [i32, P(vp)]
    L.cse_ctx_create.restype = i32
    L.cse_ctx_destroy.argtypes = [vp]
    L.cse_ctx_destroy.restype = None
    L.cse_last_error.argtypes = [vp]
    L.cse_last_error.restype = ctypes.c_char_p
    L.cse_system_load.argtypes = [vp, P(ctypes.c_int8), i32, i32, P(i32)]
    L.cse_system_load.restype = i32
    L.cse_scheme_load.argtypes = [vp, P(ctypes.c_int8), i32, i32, P(ctypes.c_int8), i32, i32,
                                  P(ctypes.c_int8), i32, i32, P(i32)]
    L.cse_scheme_load.restype = i32
    L.cse_scheme_load_device.argtypes = [vp, vp, i32, i32, vp, i32, i32, vp, i32, i32, vp, P(i32)]
    L.cse_scheme_load_device.restype = i32
    L.cse_scheme_info.argtypes = [vp, i32, P(i32), P(i32)]
    L.cse_flip_variants.argtypes = [vp, P(ctypes.c_int8), P(ctypes.c_int8), P(ctypes.c_int8), i32, P(CseFlipCfg),
                                    ctypes.c_uint64, ctypes.c_uint32, P(ctypes.c_int8), P(ctypes.c_int8),
                                    P(ctypes.c_int8), P(i32)]
    L.cse_flip_variants.restype = i32
    L.cse_run_flips.argtypes = [vp, P(ctypes.c_int8), P(ctypes.c_int8), P(ctypes.c_int8), i32, P(CseFlipCfg),
                                P(CseRunCfg), i32, i32, vp, P(i32), P(i32)]
    L.cse_run_flips.restype = i32
    L.cse_flip_best.argtypes = [vp, i32, P(ctypes.c_int8), P(ctypes.c_int8), P(ctypes.c_int8), P(i32), P(i32),
                                P(i32), P(i32), i32, P(i32)]
    L.cse_flip_best.restype = i32
    L.cse_flip_program.argtypes = [vp, i32, i32, P(i32), i32, P(i32), P(i32)]
    L.cse_flip_program.restype = i32
    L.cse_flip_release.argtypes = [vp, i32]
    L.cse_flip_release.restype = i32
    L.cse_ctx_set_timing.argtypes = [vp, i32]
    L.cse_ctx_set_timing.restype = i32
    L.cse_kernel_times.argtypes = [vp, i32, P(CseKernelTime), i32, P(i32), i32]
    L.cse_kernel_times.restype = i32
    L.cse_scheme_info.restype = i32
    L.cse_scheme_free.argtypes = [vp, i32]
    L.cse_scheme_free.restype = i32
    L.cse_launch.argtypes = [vp, i32, P(CseRunCfg), vp, P(i32)]
    L.cse_launch.restype = i32
    L.cse_launch_batch.argtypes = [vp, P(i32), P(CseRunCfg), i32, vp, P(i32)]
    L.cse_launch_batch.restype = i32
    L.cse_relaunch.argtypes = [vp, i32, P(CseRunCfg), vp]
    L.cse_relaunch.restype = i32
    L.cse_resume.argtypes = [vp, i32, vp]
    L.cse_resume.restype = i32
    L.cse_poll.argtypes = [vp, i32, P(i32), P(i32)]
    L.cse_poll.restype = i32
    L.cse_cancel.argtypes = [vp, i32]
    L.cse_cancel.restype = i32
    L.cse_scheme_layout.argtypes = [vp, i32, i32, i32, P(i32)]
    L.cse_scheme_layout.restype = i32
    L.cse_autotune.argtypes = [vp, i32, ctypes.c_void_p, vp, P(i32)]
    L.cse_autotune.restype = i32
    L.cse_wait.argtypes = [vp, i32]
    L.cse_wait.restype = i32
    L.cse_get_unit_results.argtypes = [vp, i32, i32, i32, P(i32), P(i32), P(i32), P(i32), P(i32),
                                       P(ctypes.c_int64), P(i32), P(ctypes.c_uint64)]
    L.cse_get_unit_results.restype = i32
    L.cse_get_programs.argtypes = [vp, i32, i32, i32, P(i32), i32]
    L.cse_get_programs.restype = i32
    L.cse_get_program.argtypes = [vp, i32, i32, i32, P(i32), i32, P(i32), P(i32), P(i32)]
    L.cse_get_program.restype = i32
    L.cse_job_timing.argtypes = [vp, i32, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    L.cse_job_timing.restype = i32
    L.cse_job_release.argtypes = [vp, i32]
    L.cse_job_release.restype = i32
    L.cse_server_create.argtypes = [vp, ctypes.c_uint64, u32, vp, P(vp)]
    L.cse_server_create.restype = i32
    L.cse_server_submit.argtypes = [vp, i32, P(CseRunCfg), P(i32)]
    L.cse_server_submit.restype = i32
    L.cse_server_tick.argtypes = [vp, P(i32), P(i32)]
    L.cse_server_tick.restype = i32
    L.cse_server_job_info.argtypes = [vp, i32, P(i32), P(ctypes.c_uint64)]
    L.cse_server_job_info.restype = i32
    L.cse_server_release.argtypes = [vp, i32]
    L.cse_server_release.restype = i32
    L.cse_server_destroy.argtypes = [vp]
    L.cse_server_destroy.restype = None
    L.cse_run_driver.argtypes = [vp, i32, P(CseRunCfg), P(CseDriverCfg), vp, P(i32), P(i32)]
    L.cse_run_driver.restype = i32
    L.cse_driver_best.argtypes = [vp, i32, i32, P(i32), i32, P(i32), P(i32), P(i32), P(i32), P(i32)]
    L.cse_driver_best.restype = i32
    L.cse_driver_totals.argtypes = [vp, i32, P(i32), P(ctypes.c_uint64), i32, P(i32)]
    L.cse_driver_totals.restype = i32
    L.cse_hybrid_best.argtypes = [vp, P(i32), i32, P(i32), P(i32), P(i32)]
    L.cse_hybrid_best.restype = i32
    L.cse_reduce_static.argtypes = [vp, vp, i32, i32, i32, P(CseRunCfg), vp, vp, vp, vp, i32, P(i32)]
    L.cse_reduce_static.restype = i32
    _lib = L
    return L


def _check(ctx, rc):
    if rc != 0:
        msg = load_library().cse_last_error(ctx).decode() if ctx else ""
        raise CseError(rc, msg)


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _i8(A):
    A = np.ascontiguousarray(A, dtype=np.int8)
    if A.ndim != 2:
        raise ValueError("system must be a 2-D matrix")
    return A


def cse_run_cfg(seed=0, n_proc=1, weights=None, mix_weights=(8, 4, 2, 1), proc0_greedy=False,
                gr_p_q16=49152, step_cap=0, share_every=0, share_src_pm=0, share_dst_pm=0,
                share_max_rounds=0, iteration=0, count_path=CSE_COUNT_AUTO) -> CseRunCfg:
    """Build a cse_run_cfg; weights is {strategy name: integer weight}."""
    cfg = CseRunCfg()
    cfg.seed = seed
    cfg.n_proc = n_proc
    w = [0] * 7
    for k, v in (weights or {"gi": 1}).items():
        w[STRATEGIES.index(k)] = int(v)
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
    cfg.count_path = count_path
    return cfg


def cse_version() -> int:
    return int(load_library().cse_version())


def cse_ctx_create(device: int = 0):
    L = load_library()
    h = ctypes.c_void_p()
    _check(None, L.cse_ctx_create(device, ctypes.byref(h)))
    return h


def cse_ctx_destroy(ctx):
    load_library().cse_ctx_destroy(ctx)


def cse_last_error(ctx) -> str:
    return load_library().cse_last_error(ctx).decode()


def cse_system_load(ctx, A) -> int:
    A = _i8(A)
    sid = ctypes.c_int32()
    _check(ctx, load_library().cse_system_load(ctx, _p(A, ctypes.c_int8), A.shape[0], A.shape[1],
                                               ctypes.byref(sid)))
    return sid.value


def cse_scheme_load(ctx, U, V, Wt) -> int:
    U, V, Wt = _i8(U), _i8(V), _i8(Wt)
    sid = ctypes.c_int32()
    _check(ctx, load_library().cse_scheme_load(
        ctx, _p(U, ctypes.c_int8), U.shape[0], U.shape[1], _p(V, ctypes.c_int8), V.shape[0], V.shape[1],
        _p(Wt, ctypes.c_int8), Wt.shape[0], Wt.shape[1], ctypes.byref(sid)))
    return sid.value


def cse_scheme_load_device(ctx, U, V=None, Wt=None, stream=None) -> int:
    """U, V, W^T as int8 device tensors (rows x cols, contiguous); V and W^T
    None load U alone."""
    mats = [U, V, Wt]
    args = []
    for M in mats:
        if M is None:
            args += [None, 0, 0]
            continue
        if M.dtype != __import__("torch").int8 or not M.is_cuda or not M.is_contiguous() or M.dim() != 2:
            raise ValueError("device systems must be contiguous 2-D int8 GPU tensors")
        args += [ctypes.c_void_p(M.data_ptr()), M.shape[0], M.shape[1]]
    sid = ctypes.c_int32()
    _check(ctx, load_library().cse_scheme_load_device(ctx, *args, _stream_ptr(stream), ctypes.byref(sid)))
    return sid.value


def _flip_args(U, V, W, n, m, p, n_variants, max_flips):
    U, V, W = _i8(U), _i8(V), _i8(W)
    r = U.shape[0]
    if U.shape != (r, n * m) or V.shape != (r, m * p) or W.shape != (r, n * p):
        raise ValueError("U, V, W must be r x nm, r x mp, r x np")
    f = CseFlipCfg()
    f.n, f.m, f.p, f.n_variants, f.max_flips, f.reserved = n, m, p, n_variants, max_flips, 0
    return U, V, W, r, f


def cse_flip_variants(ctx, U, V, W, n, m, p, n_variants, max_flips, seed=0, iteration=0):
    """[(U_v, V_v, W_v, flips)] for the M variants of one iteration."""
    U, V, W, r, f = _flip_args(U, V, W, n, m, p, n_variants, max_flips)
    oU = np.zeros((n_variants, r, n * m), np.int8)
    oV = np.zeros((n_variants, r, m * p), np.int8)
    oW = np.zeros((n_variants, r, n * p), np.int8)
    nf = np.zeros(n_variants, np.int32)
    i8 = ctypes.c_int8
    _check(ctx, load_library().cse_flip_variants(ctx, _p(U, i8), _p(V, i8), _p(W, i8), r, ctypes.byref(f), seed,
                                                 iteration, _p(oU, i8), _p(oV, i8), _p(oW, i8),
                                                 _p(nf, ctypes.c_int32)))
    return [(oU[v], oV[v], oW[v], int(nf[v])) for v in range(n_variants)]


def cse_run_flips(ctx, U, V, W, n, m, p, cfg: CseRunCfg, n_variants=32, max_flips=32, patience=10,
                  max_iterations=100, stream=None):
    """Random-flip mode (blocking).  Returns (run id, iterations)."""
    U, V, W, r, f = _flip_args(U, V, W, n, m, p, n_variants, max_flips)
    run, its = ctypes.c_int32(-1), ctypes.c_int32(0)
    i8 = ctypes.c_int8
    _check(ctx, load_library().cse_run_flips(ctx, _p(U, i8), _p(V, i8), _p(W, i8), r, ctypes.byref(f),
                                             ctypes.byref(cfg), patience, max_iterations, _stream_ptr(stream),
                                             ctypes.byref(run), ctypes.byref(its)))
    return run.value, its.value


def cse_flip_best(ctx, run_id, shape):
    """shape = (n, m, p, r): dict(U, V, W, cost[3], variant, iteration, totals)."""
    n, m, p, r = shape
    U = np.zeros((r, n * m), np.int8)
    V = np.zeros((r, m * p), np.int8)
    W = np.zeros((r, n * p), np.int8)
    cost = (ctypes.c_int32 * 3)()
    var, it, ni = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    L = load_library()
    i8 = ctypes.c_int8
    _check(ctx, L.cse_flip_best(ctx, run_id, None, None, None, None, None, None, None, 0, ctypes.byref(ni)))
    totals = np.zeros(max(1, ni.value), np.int32)
    _check(ctx, L.cse_flip_best(ctx, run_id, _p(U, i8), _p(V, i8), _p(W, i8), cost, ctypes.byref(var),
                                ctypes.byref(it), _p(totals, ctypes.c_int32), ni.value, ctypes.byref(ni)))
    return dict(U=U, V=V, W=W, cost=list(cost), variant=var.value, iteration=it.value,
                totals=[int(x) for x in totals[:ni.value]])


def cse_flip_program(ctx, run_id, comp):
    L = load_library()
    n, need = ctypes.c_int32(), ctypes.c_int32()
    rc = L.cse_flip_program(ctx, run_id, comp, None, 0, ctypes.byref(n), ctypes.byref(need))
    if rc not in (0, -3):
        _check(ctx, rc)
    tr = np.zeros((max(1, need.value), 3), np.int32)
    _check(ctx, L.cse_flip_program(ctx, run_id, comp, _p(tr, ctypes.c_int32), need.value, ctypes.byref(n),
                                   ctypes.byref(need)))
    return tr[:n.value]


def cse_flip_release(ctx, run_id):
    _check(ctx, load_library().cse_flip_release(ctx, run_id))


def cse_ctx_set_timing(ctx, on: bool):
    _check(ctx, load_library().cse_ctx_set_timing(ctx, 1 if on else 0))


def cse_kernel_times(ctx, job_id, reset=False):
    """[{row_words, layout, launches, device_ns}] per step-kernel class."""
    L = load_library()
    n = ctypes.c_int32()
    _check(ctx, L.cse_kernel_times(ctx, job_id, None, 0, ctypes.byref(n), 0))
    out = (CseKernelTime * max(1, n.value))()
    _check(ctx, L.cse_kernel_times(ctx, job_id, out, n.value, ctypes.byref(n), 1 if reset else 0))
    return [dict(row_words=t.row_words, layout=t.layout, launches=t.launches, device_ns=int(t.device_ns))
            for t in out[:n.value]]


def cse_scheme_info(ctx, scheme_id):
    """[(n_e, n_x, n_fmax, naive) per component]"""
    n = ctypes.c_int32()
    info = (ctypes.c_int32 * 12)()
    _check(ctx, load_library().cse_scheme_info(ctx, scheme_id, ctypes.byref(n), info))
    return [tuple(info[4 * c:4 * c + 4]) for c in range(n.value)]


def cse_scheme_free(ctx, scheme_id):
    _check(ctx, load_library().cse_scheme_free(ctx, scheme_id))


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def cse_launch(ctx, scheme_id, cfg: CseRunCfg, stream=None) -> int:
    job = ctypes.c_int32()
    _check(ctx, load_library().cse_launch(ctx, scheme_id, ctypes.byref(cfg), _stream_ptr(stream),
                                          ctypes.byref(job)))
    return job.value


def cse_launch_batch(ctx, scheme_ids, cfgs, stream=None):
    n = len(scheme_ids)
    ids = np.ascontiguousarray(scheme_ids, dtype=np.int32)
    arr = (CseRunCfg * n)(*cfgs)
    jobs = np.zeros(n, np.int32)
    _check(ctx, load_library().cse_launch_batch(ctx, _p(ids, ctypes.c_int32), arr, n, _stream_ptr(stream),
                                                _p(jobs, ctypes.c_int32)))
    return [int(j) for j in jobs]


def cse_relaunch(ctx, job_id, cfg: CseRunCfg | None = None, stream=None):
    _check(ctx, load_library().cse_relaunch(ctx, job_id, ctypes.byref(cfg) if cfg is not None else None,
                                            _stream_ptr(stream)))


def cse_resume(ctx, job_id, stream=None):
    _check(ctx, load_library().cse_resume(ctx, job_id, _stream_ptr(stream)))


def cse_poll(ctx, job_id, best=False):
    """done (bool); with best=True, (done, [best cost per component] or None)."""
    done = ctypes.c_int32()
    bc = (ctypes.c_int32 * 3)()
    _check(ctx, load_library().cse_poll(ctx, job_id, ctypes.byref(done), bc if best else None))
    if not best:
        return bool(done.value)
    return bool(done.value), (list(bc) if done.value else None)


def cse_wait(ctx, job_id):
    _check(ctx, load_library().cse_wait(ctx, job_id))


def cse_cancel(ctx, job_id):
    _check(ctx, load_library().cse_cancel(ctx, job_id))


def cse_scheme_layout(ctx, scheme_id, comp, layout=-1) -> int:
    """Set (layout >= 0) or query the layout of a component; returns the
    layout in effect before the call."""
    cur = ctypes.c_int32()
    _check(ctx, load_library().cse_scheme_layout(ctx, scheme_id, comp, layout, ctypes.byref(cur)))
    return cur.value


def cse_autotune(ctx, scheme_id, cfg, stream):
    """Pick each component's fastest layout; returns the chosen layouts."""
    out = (ctypes.c_int32 * 3)(-1, -1, -1)
    _check(ctx, load_library().cse_autotune(ctx, scheme_id, ctypes.byref(cfg), _stream_ptr(stream), out))
    return list(out)


def cse_get_unit_results(ctx, job_id, comp, n_proc):
    out = {k: np.zeros(n_proc, np.int32) for k in ("cost", "steps", "executed", "epoch", "k0", "strat")}
    out["ops"] = np.zeros(n_proc, np.int64)
    out["finish"] = np.zeros(n_proc, np.uint64)
    i32 = ctypes.c_int32
    _check(ctx, load_library().cse_get_unit_results(
        ctx, job_id, comp, n_proc, _p(out["cost"], i32), _p(out["steps"], i32), _p(out["executed"], i32),
        _p(out["epoch"], i32), _p(out["k0"], i32), _p(out["ops"], ctypes.c_int64), _p(out["strat"], i32),
        _p(out["finish"], ctypes.c_uint64)))
    return out


def cse_get_programs(ctx, job_id, comp, n_proc, cap):
    tri = np.zeros((n_proc, max(1, cap), 3), np.int32)
    _check(ctx, load_library().cse_get_programs(ctx, job_id, comp, n_proc, _p(tri, ctypes.c_int32),
                                                max(1, cap)))
    return tri


def cse_get_program(ctx, job_id, comp, proc=-1, cap=None):
    L = load_library()
    nf, cost, need = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    if cap is None:
        rc = L.cse_get_program(ctx, job_id, comp, proc, None, 0, ctypes.byref(nf), ctypes.byref(cost),
                               ctypes.byref(need))
        if rc not in (0, -3):
            _check(ctx, rc)
        cap = need.value
    tri = np.zeros((max(1, cap), 3), np.int32)
    _check(ctx, L.cse_get_program(ctx, job_id, comp, proc, _p(tri, ctypes.c_int32), cap, ctypes.byref(nf),
                                  ctypes.byref(cost), ctypes.byref(need)))
    return tri[:nf.value], cost.value


def cse_job_timing(ctx, job_id):
    """(ticks from job start to the last unit's finish, tick rate in Hz)"""
    t, hz = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, load_library().cse_job_timing(ctx, job_id, ctypes.byref(t), ctypes.byref(hz)))
    return t.value, hz.value


def cse_job_release(ctx, job_id):
    _check(ctx, load_library().cse_job_release(ctx, job_id))


def cse_run_driver(ctx, scheme_id, cfg: CseRunCfg, stream=None, reinit_pm=400, patience=10, max_iterations=100):
    """Outer iterations until convergence (blocking).  Returns (job, iterations).
    On an error after the job was created the raised CseError carries
    job_id (release it) and iterations."""
    d = CseDriverCfg()
    d.reinit_pm, d.patience, d.max_iterations = reinit_pm, patience, max_iterations
    job, its = ctypes.c_int32(-1), ctypes.c_int32(0)
    rc = load_library().cse_run_driver(ctx, scheme_id, ctypes.byref(cfg), ctypes.byref(d), _stream_ptr(stream),
                                       ctypes.byref(job), ctypes.byref(its))
    if rc != 0:
        err = CseError(rc, load_library().cse_last_error(ctx).decode())
        err.job_id = job.value if job.value > 0 else None
        err.iterations = its.value
        raise err
    return job.value, its.value


def cse_driver_best(ctx, job_id, comp):
    """Best program so far of a component of a driver job:
    dict(prog (L x 3 int32), cost, iteration, proc)."""
    L = load_library()
    nf, cost, it, proc, need = (ctypes.c_int32() for _ in range(5))
    rc = L.cse_driver_best(ctx, job_id, comp, None, 0, ctypes.byref(nf), ctypes.byref(cost), ctypes.byref(it),
                           ctypes.byref(proc), ctypes.byref(need))
    if rc not in (0, -3):
        _check(ctx, rc)
    tri = np.zeros((max(1, need.value), 3), np.int32)
    _check(ctx, L.cse_driver_best(ctx, job_id, comp, _p(tri, ctypes.c_int32), need.value, ctypes.byref(nf),
                                  ctypes.byref(cost), ctypes.byref(it), ctypes.byref(proc), ctypes.byref(need)))
    return dict(prog=tri[:nf.value], cost=cost.value, iteration=it.value, proc=proc.value)


def cse_driver_totals(ctx, job_id, elapsed=False):
    """Best total after each iteration of a driver job (list of int); with
    elapsed=True also the host ns from the driver start to each iteration's end."""
    L = load_library()
    n = ctypes.c_int32()
    _check(ctx, L.cse_driver_totals(ctx, job_id, None, None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), np.int32)
    ns = np.zeros(max(1, n.value), np.uint64)
    _check(ctx, L.cse_driver_totals(ctx, job_id, _p(out, ctypes.c_int32), _p(ns, ctypes.c_uint64), n.value,
                                    ctypes.byref(n)))
    totals = [int(x) for x in out[:n.value]]
    return (totals, [int(x) for x in ns[:n.value]]) if elapsed else totals


def cse_hybrid_best(ctx, job_ids):
    """Per component over several jobs: [(cost, job, proc)] of the best (Sec. 4 hybrid)."""
    ids = np.ascontiguousarray(job_ids, dtype=np.int32)
    cost, job, proc = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)()
    _check(ctx, load_library().cse_hybrid_best(ctx, _p(ids, ctypes.c_int32), len(ids), cost, job, proc))
    return [(cost[c], job[c], proc[c]) for c in range(3) if cost[c] >= 0]


# Servers report errors through the context they were created on.
class CseServer:
    """Handle of a server; keeps the context for error messages."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle


def cse_server_create(ctx, max_state_bytes, round_steps=32, stream=None) -> CseServer:
    h = ctypes.c_void_p()
    _check(ctx, load_library().cse_server_create(ctx, max_state_bytes, round_steps, _stream_ptr(stream),
                                                 ctypes.byref(h)))
    return CseServer(ctx, h)


def cse_server_submit(server: CseServer, scheme_id, cfg: CseRunCfg) -> int:
    job = ctypes.c_int32()
    _check(server.ctx, load_library().cse_server_submit(server.handle, scheme_id, ctypes.byref(cfg),
                                                        ctypes.byref(job)))
    return job.value


def cse_server_tick(server: CseServer):
    """Returns (running, queued)."""
    r, q = ctypes.c_int32(), ctypes.c_int32()
    _check(server.ctx, load_library().cse_server_tick(server.handle, ctypes.byref(r), ctypes.byref(q)))
    return r.value, q.value


def cse_server_job_info(server: CseServer, job_id):
    """Returns (state, (t_submit_ns, t_admit_ns, t_done_ns))."""
    st = ctypes.c_int32()
    t = (ctypes.c_uint64 * 3)()
    _check(server.ctx, load_library().cse_server_job_info(server.handle, job_id, ctypes.byref(st), t))
    return st.value, tuple(int(x) for x in t)


def cse_server_release(server: CseServer, job_id):
    _check(server.ctx, load_library().cse_server_release(server.handle, job_id))


def cse_server_destroy(server: CseServer):
    load_library().cse_server_destroy(server.handle)


def _dev_i32(t, shape, name):
    torch = __import__("torch")
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous int32 GPU tensor of shape {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def cse_reduce_static_needed(ctx, A, cfg: CseRunCfg, comp=0, stream=None) -> int:
    """Program entries per process that cse_reduce_static needs for A."""
    if A.dtype != __import__("torch").int8 or not A.is_cuda or not A.is_contiguous() or A.dim() != 2:
        raise ValueError("A must be a contiguous 2-D int8 GPU tensor")
    need = ctypes.c_int32(0)
    rc = load_library().cse_reduce_static(ctx, ctypes.c_void_p(A.data_ptr()), A.shape[0], A.shape[1], comp,
                                          ctypes.byref(cfg), _stream_ptr(stream), None, None, None, 0,
                                          ctypes.byref(need))
    if rc not in (0, -3):
        _check(ctx, rc)
    return need.value


def cse_reduce_static(ctx, A, cfg: CseRunCfg, cost, length, prog, comp=0, stream=None):
    """Reduce A (int8 GPU tensor) with no device allocation; cost and length
    are int32 GPU tensors of n_proc entries, prog an int32 GPU tensor of
    n_proc x cap program keys (a << 16 | b << 1 | (s < 0))."""
    if A.dtype != __import__("torch").int8 or not A.is_cuda or not A.is_contiguous() or A.dim() != 2:
        raise ValueError("A must be a contiguous 2-D int8 GPU tensor")
    n = cfg.n_proc
    if prog.dim() != 2:
        raise ValueError("prog must be n_proc x cap")
    cap = prog.shape[1]
    need = ctypes.c_int32(0)
    _check(ctx, load_library().cse_reduce_static(
        ctx, ctypes.c_void_p(A.data_ptr()), A.shape[0], A.shape[1], comp, ctypes.byref(cfg), _stream_ptr(stream),
        _dev_i32(cost, (n,), "cost"), _dev_i32(length, (n,), "length"), _dev_i32(prog, (n, cap), "prog"), cap,
        ctypes.byref(need)))
