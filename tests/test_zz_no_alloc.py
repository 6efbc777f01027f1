"""cse_reduce_static, the entry point that allocates no device memory (its
working buffers live in a static device array), against the allocating
path cse_scheme_load / cse_system_load + cse_launch on the same inputs: every
unit's cost, program length and program, bit for bit.  Two calls in a row
reuse the array, the second on a smaller input."""
import sys

import numpy as np
import pytest

from paper_2512_13365_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_13365_amd import cse
    cse.load_library()
    ctx = cse.cse_ctx_create(0)
    yield cse, ctx, torch
    cse.cse_ctx_destroy(ctx)


def allocating_run(gpu, systems, kw):
    """Per component: cost, length and program keys of the allocating path."""
    cse, ctx, torch = gpu
    sid = cse.cse_scheme_load(ctx, *systems) if len(systems) == 3 else cse.cse_system_load(ctx, systems[0])
    info = cse.cse_scheme_info(ctx, sid)
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    cse.cse_wait(ctx, job)
    out = []
    for c in range(len(systems)):
        r = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
        tri = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
        out.append((r["cost"], r["steps"], tri))
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    return out


def static_run(gpu, A, kw, comp):
    cse, ctx, torch = gpu
    cfg = cse.cse_run_cfg(**kw)
    dA = torch.from_numpy(np.ascontiguousarray(A, dtype=np.int8)).cuda()
    stream = torch.cuda.current_stream()
    cap = cse.cse_reduce_static_needed(ctx, dA, cfg, comp, stream)
    n = kw["n_proc"]
    # Outputs prefilled with a marker, so entries the call must write are seen to be written.
    cost = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    length = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    prog = torch.full((n, cap), -1, dtype=torch.int32, device="cuda")
    cse.cse_reduce_static(ctx, dA, cfg, cost, length, prog, comp=comp, stream=stream)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), length.cpu().numpy(), prog.cpu().numpy().view(np.uint32), cap


def assert_same(ref, got, label):
    rc, rl, rtri = ref
    gc, gl, keys, cap = got
    assert np.array_equal(gc, rc), f"{label}: costs differ at {np.flatnonzero(gc != rc)[:8]}"
    assert np.array_equal(gl, rl), f"{label}: lengths differ at {np.flatnonzero(gl != rl)[:8]}"
    assert rtri.shape[1] == cap
    for p in range(len(gc)):
        L = int(gl[p])
        k = keys[p, :L].astype(np.int64)
        tri = np.stack([k >> 16, (k >> 1) & 0x7FFF, np.where(k & 1, -1, 1)], axis=1)
        assert np.array_equal(tri, rtri[p, :L]), f"{label}: program of unit {p} differs"


def test_static_matches_allocating_path_twice(gpu):
    """4x4x4 (4096 processes, all three components, LDS state), then the
    smaller 2x2x2 (64 processes): the second call reuses the array."""
    wl = workloads.plain_4x4x4()
    sc, rs = wl.schemes[0], wl.runs[0]
    kw = rs.as_kwargs()
    say(f"[gpu] static vs allocating: 4x4x4 {[A.shape for A in sc.systems]} n_proc {kw['n_proc']}")
    ref = allocating_run(gpu, sc.systems, kw)
    for c, A in enumerate(sc.systems):
        assert_same(ref[c], static_run(gpu, A, kw, c), f"4x4x4 comp {c}")
    wl2 = workloads.tiny_2x2x2()
    sc2, kw2 = wl2.schemes[0], wl2.runs[0].as_kwargs()
    say(f"[gpu] static vs allocating: 2x2x2 {[A.shape for A in sc2.systems]} n_proc {kw2['n_proc']}")
    ref2 = allocating_run(gpu, sc2.systems, kw2)
    for c, A in enumerate(sc2.systems):
        assert_same(ref2[c], static_run(gpu, A, kw2, c), f"2x2x2 comp {c}")


def test_static_hbm_state_and_lone_system(gpu):
    """A system whose units keep their state in per-unit HBM slots (inside
    the array here), with gp, then a smaller lone system with every strategy."""
    rng = np.random.default_rng(11)
    A = workloads.ternary_rows(rng, 160, 36, 0.15, 1, 12)
    kw = dict(seed=5, n_proc=96, weights={"gi": 3, "ga": 1, "wr": 1, "gr": 1, "mix": 1, "gp": 1},
              proc0_greedy=True)
    say(f"[gpu] static vs allocating: HBM-state system {A.shape} n_proc 96")
    ref = allocating_run(gpu, [A], kw)
    assert_same(ref[0], static_run(gpu, A, kw, 0), "160x36")
    B = workloads.ternary_rows(rng, 30, 12, 0.3, 1, 8)
    kw2 = dict(seed=9, n_proc=200, weights={"g": 1, "ga": 1, "wr": 1, "gr": 1, "gi": 2, "mix": 1}, step_cap=6)
    say(f"[gpu] static vs allocating: lone system {B.shape} n_proc 200")
    ref2 = allocating_run(gpu, [B], kw2)
    assert_same(ref2[0], static_run(gpu, B, kw2, 0), "30x12")


def test_static_refusals(gpu):
    cse, ctx, torch = gpu
    wl = workloads.plain_4x4x4()
    A = torch.from_numpy(wl.schemes[0].systems[0]).cuda()
    stream = torch.cuda.current_stream()
    kw = wl.runs[0].as_kwargs()
    cfg = cse.cse_run_cfg(**kw)
    cap = cse.cse_reduce_static_needed(ctx, A, cfg, 0, stream)
    n = kw["n_proc"]
    cost = torch.zeros(n, dtype=torch.int32, device="cuda")
    length = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(cse.CseError) as e:  # program buffer too small
        cse.cse_reduce_static(ctx, A, cfg, cost, length, torch.zeros((n, cap - 1), dtype=torch.int32, device="cuda"),
                              stream=stream)
    assert e.value.status == -3
    prog = torch.zeros((n, cap), dtype=torch.int32, device="cuda")
    with pytest.raises(cse.CseError) as e:  # sharing rounds are not run here
        cse.cse_reduce_static(ctx, A, cse.cse_run_cfg(**dict(kw, share_every=32, share_src_pm=10, share_dst_pm=100,
                                                               share_max_rounds=4)), cost, length, prog,
                              stream=stream)
    assert e.value.status == -1
    big = cse.cse_run_cfg(**dict(kw, n_proc=1 << 21))  # ~75 MB of unit state: beyond the array
    with pytest.raises(cse.CseError) as e:
        cse.cse_reduce_static(ctx, A, big, torch.zeros(1 << 21, dtype=torch.int32, device="cuda"),
                              torch.zeros(1 << 21, dtype=torch.int32, device="cuda"),
                              torch.zeros((1 << 21, cap), dtype=torch.int32, device="cuda"), stream=stream)
    assert e.value.status == -2
    bad = A.clone()
    bad[0, 0] = 2
    with pytest.raises(cse.CseError) as e:
        cse.cse_reduce_static(ctx, bad, cfg, cost, length, prog, stream=stream)
    assert e.value.status == -1
    # The array still serves a valid call after the refusals.
    ref = allocating_run(gpu, [wl.schemes[0].systems[0]], dict(kw, n_proc=512))
    assert_same(ref[0], static_run(gpu, wl.schemes[0].systems[0], dict(kw, n_proc=512), 0), "after refusals")
