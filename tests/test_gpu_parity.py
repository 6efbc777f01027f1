"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every unit is compared element by element: cost, program length, selection
steps, restarts, the algorithmic work tally, the strategy, and the full
program.  Integer work, so the bar is bit-exact.
"""
import os
import sys

import numpy as np
import pytest

from cse_helpers import check_program, read_golden
from paper_2512_13365_amd import workloads

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
ALL_W = {"g": 1, "ga": 2, "wr": 2, "gr": 2, "gi": 4, "mix": 2}


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


def run_gpu(gpu, systems, kw):
    cse, ctx, torch = gpu
    if len(systems) == 3:
        sid = cse.cse_scheme_load(ctx, *systems)
    else:
        sid = cse.cse_system_load(ctx, systems[0])
    info = cse.cse_scheme_info(ctx, sid)
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    cse.cse_wait(ctx, job)
    out = []
    for c in range(len(systems)):
        r = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
        r["prog"] = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
        out.append(r)
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    return out


def compare(oracle, systems, kw, label, procs=None):
    ocfg = oracle.make_cfg(**{k: v for k, v in kw.items() if k != "count_path"})
    res = []
    for c, A in enumerate(systems):
        ref = oracle.run_pool(A, ocfg, comp=c, procs=procs, n_threads=THREADS)
        res.append(ref)
    return res


def assert_same(got, ref, label):
    for k in ("cost", "steps", "executed", "epoch", "k0", "ops", "strat"):
        g, r = np.asarray(got[k]), np.asarray(ref[k])
        bad = np.flatnonzero(g != r)
        assert bad.size == 0, f"{label}: {k} differs at units {bad[:8]} gpu={g[bad[:8]]} oracle={r[bad[:8]]}"
    assert got["prog"].shape == ref["prog"].shape
    bad = np.flatnonzero((got["prog"] != ref["prog"]).any(axis=(1, 2)))
    assert bad.size == 0, f"{label}: programs differ at units {bad[:8]}"


def check_workload(gpu, oracle, systems, kw, label):
    say(f"[gpu] {label}: shapes {[A.shape for A in systems]} n_proc {kw['n_proc']}")
    got = run_gpu(gpu, systems, kw)
    ref = compare(oracle, systems, kw, label)
    for c in range(len(systems)):
        assert_same(got[c], ref[c], f"{label} comp {c}")
    return got, ref


def test_tiny_2x2x2_every_unit(gpu, oracle):
    wl = workloads.tiny_2x2x2()
    check_workload(gpu, oracle, wl.schemes[0].systems, wl.runs[0].as_kwargs(), "tiny-2x2x2")


def test_plain_4x4x4_every_unit(gpu, oracle):
    """The benchmarked workload at full size: 4096 processes x 3 components."""
    wl = workloads.plain_4x4x4()
    got, ref = check_workload(gpu, oracle, wl.schemes[0].systems, wl.runs[0].as_kwargs(), "plain-4x4x4")
    sc = wl.schemes[0]
    for c, A in enumerate(sc.systems):
        best = int(np.argmin(got[c]["cost"]))
        check_program(A, got[c]["prog"][best, :got[c]["steps"][best]], int(got[c]["cost"][best]))


@pytest.mark.parametrize("rows,cols,p,hi", [
    (2, 6, 0.6, None), (9, 5, 0.5, None), (63, 20, 0.25, 8), (64, 20, 0.25, 8), (65, 24, 0.25, 8),
    (127, 16, 0.3, 8), (130, 30, 0.2, 10), (200, 40, 0.12, 12), (512, 10, 0.4, 6), (20, 120, 0.1, 30)])
def test_ragged_shapes_all_strategies(gpu, oracle, rows, cols, p, hi):
    """Row counts across 1..8 bitset words with ragged tails, every strategy."""
    A = workloads.random_system(rows * 1000 + cols, rows, cols, p, 1, hi)
    kw = dict(seed=rows + cols, n_proc=96, weights=dict(ALL_W), proc0_greedy=True)
    check_workload(gpu, oracle, [A], kw, f"system {rows}x{cols}")


def test_mix_single_weight_is_that_strategy(gpu, oracle):
    """mix (Sec. 3.4.3) with all weight on gi, ga, gr or wr in turn runs that
    strategy on every step: each such pool equals the GPU pool of the plain
    strategy and the oracle's."""
    A = workloads.random_system(4412, 24, 12, 0.4)
    base = dict(seed=5, n_proc=256)
    for name, mixw in (("gi", (1, 0, 0, 0)), ("ga", (0, 1, 0, 0)), ("gr", (0, 0, 1, 0)), ("wr", (0, 0, 0, 1))):
        plain = run_gpu(gpu, [A], dict(base, weights={name: 1}))[0]
        got, _ = check_workload(gpu, oracle, [A], dict(base, weights={"mix": 1}, mix_weights=mixw),
                                f"mix on {name}")
        assert np.array_equal(got[0]["prog"], plain["prog"]), name
        assert np.array_equal(got[0]["cost"], plain["cost"]), name


def test_device_resident_input_load(gpu, oracle):
    """cse_scheme_load_device: systems already in HBM are validated and
    analysed on the device; the job equals the oracle's (and so the
    host-loaded job); bad entries and zero rows are refused."""
    cse, ctx, torch = gpu
    wl = workloads.plain_4x4x4(n_proc=128)
    S = wl.schemes[0].systems
    kw = dict(wl.runs[0].as_kwargs(), n_proc=128)
    st = torch.cuda.current_stream()
    dev = [torch.from_numpy(A).to("cuda") for A in S]
    sid = cse.cse_scheme_load_device(ctx, *dev, stream=st)
    assert cse.cse_scheme_info(ctx, sid) == [(A.shape[0], A.shape[1], oracle.bounds(A)[0], oracle.naive(A)) for A in S]
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), st)
    cse.cse_wait(ctx, job)
    ref = compare(oracle, S, kw, "device load")
    for c in range(3):
        got = cse.cse_get_unit_results(ctx, job, c, 128)
        got["prog"] = cse.cse_get_programs(ctx, job, c, 128, max(1, ref[c]["n_fmax"]))
        assert_same(got, ref[c], f"device load comp {c}")
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    one = cse.cse_scheme_load_device(ctx, dev[2], stream=st)
    assert cse.cse_scheme_info(ctx, one) == [(16, 49, oracle.bounds(S[2])[0], oracle.naive(S[2]))]
    cse.cse_scheme_free(ctx, one)
    for bad in (np.array([[1, 2], [1, 1]], np.int8), np.array([[1, 1], [0, 0]], np.int8)):
        with pytest.raises(cse.CseError) as e:
            cse.cse_scheme_load_device(ctx, torch.from_numpy(bad).to("cuda"), stream=st)
        assert e.value.status == -1


def test_step_cap_and_seeds(gpu, oracle):
    A = workloads.random_system(77, 49, 16, 0.3, 1, 8)
    for seed, cap in ((0, 1), (1, 5), (2 ** 40 + 3, 17)):
        kw = dict(seed=seed, n_proc=128, weights=dict(ALL_W), step_cap=cap)
        check_workload(gpu, oracle, [A], kw, f"cap {cap} seed {seed}")


def test_degenerate_systems(gpu, oracle):
    """No repeated pair (Strassen, Sec. 2.2), one row, identical rows."""
    g = read_golden("strassen_2x2x2.txt")
    S = [np.array([[int(x) for x in r] for r in g[k]], np.int8) for k in ("U", "V", "Wt")]
    got, _ = check_workload(gpu, oracle, S, dict(seed=1, n_proc=64, weights=dict(ALL_W)), "strassen")
    assert sum(int(r["cost"][0]) for r in got) == 18 and all((r["steps"] == 0).all() for r in got)
    one = np.array([[1, -1, 1, 1, -1, 0, 1]], np.int8)
    check_workload(gpu, oracle, [one], dict(seed=2, n_proc=8, weights=dict(ALL_W)), "one row")
    row = np.array([1, -1, 1, 1, -1, 1, 1, -1, 1, 1], np.int8)
    same = np.stack([row, -row, row, row, -row, row])
    got, _ = check_workload(gpu, oracle, [same], dict(seed=3, n_proc=64, weights=dict(ALL_W)), "equal rows")
    assert (got[0]["cost"] == 9).all()


def test_sharing_rounds_small_pool(gpu, oracle):
    """Sharing (Sec. 3.5.2) on the 6x6x6 shape with a 256-process pool."""
    wl = workloads.plain_6x6x6(n_proc=256)
    got, _ = check_workload(gpu, oracle, wl.schemes[0].systems, wl.runs[0].as_kwargs(), "share-6x6x6-256")
    assert max(int(r["epoch"].max()) for r in got) > 0


def test_sharing_dense_targets(gpu, oracle):
    A = workloads.random_system(91, 60, 18, 0.3, 1, 8)
    kw = dict(seed=5, n_proc=200, weights=dict(ALL_W), proc0_greedy=True, share_every=3,
              share_src_pm=50, share_dst_pm=400, share_max_rounds=6)
    got, _ = check_workload(gpu, oracle, [A], kw, "share-dense")
    assert got[0]["epoch"].max() > 1


def test_invalid_inputs_rejected(gpu):
    cse, ctx, torch = gpu
    many = np.zeros((2, 40000), np.int8)
    many[:, :30000] = 1  # 40000 columns + 29999 fresh variables exceed the 15-bit variable ids
    bad = [np.array([[1, 0], [0, 0]], np.int8), np.array([[1, 2]], np.int8), np.zeros((0, 3), np.int8),
           np.zeros((3, 0), np.int8), np.ones((513, 2), np.int8), many]
    for A in bad:
        with pytest.raises(cse.CseError) as e:
            cse.cse_system_load(ctx, A)
        assert e.value.status == -1
    sid = cse.cse_system_load(ctx, np.array([[1, 1], [1, 1]], np.int8))
    with pytest.raises(cse.CseError):
        cse.cse_launch(ctx, sid, cse.cse_run_cfg(n_proc=4, weights={"mix": 1}, mix_weights=(0, 0, 0, 0)))
    with pytest.raises(cse.CseError):
        cse.cse_launch(ctx, sid, cse.cse_run_cfg(n_proc=0))
    with pytest.raises(cse.CseError) as e:
        cse.cse_launch(ctx, 9999, cse.cse_run_cfg(n_proc=4))
    assert e.value.status == -6
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(n_proc=4))
    with pytest.raises(cse.CseError):
        cse.cse_get_unit_results(ctx, job, 1, 4)
    tri, cost = cse.cse_get_program(ctx, job, 0, -1)
    assert cost == 1 and tri.tolist() == [[1, 2, 1]]
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)


def test_dense_gi_fallback_large_candidate_set(gpu, oracle):
    """Many candidates (m ~ 2000): the gi masks exceed their LDS budget and
    the O(m^2) form runs; both forms use the same coin order."""
    A = workloads.random_system(2024, 100, 60, 0.25, 1, 20)
    kw = dict(seed=11, n_proc=16, weights={"gi": 3, "mix": 1, "wr": 1}, step_cap=30)
    check_workload(gpu, oracle, [A], kw, "dense-gi 100x60")


def test_relaunch_new_seed(gpu, oracle):
    cse, ctx, torch = gpu
    wl = workloads.plain_4x4x4(n_proc=512)
    sc, rs = wl.schemes[0], wl.runs[0]
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    kw = rs.as_kwargs()
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    for seed in (7, 8):
        kw["seed"] = seed
        say(f"[gpu] relaunch seed {seed}")
        cse.cse_relaunch(ctx, job, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
        cse.cse_wait(ctx, job)
        ocfg = oracle.make_cfg(**kw)
        for c, A in enumerate(sc.systems):
            got = cse.cse_get_unit_results(ctx, job, c, rs.n_proc)
            got["prog"] = cse.cse_get_programs(ctx, job, c, rs.n_proc, cse.cse_scheme_info(ctx, sid)[c][2])
            ref = oracle.run_pool(A, ocfg, comp=c, n_threads=THREADS)
            assert_same(got, ref, f"relaunch seed {seed} comp {c}")
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)


def test_batch_equals_separate_jobs(gpu, oracle):
    """One batched launch over uneven schemes (row words 1 and 2, with and
    without sharing) gives every unit the result of its own job."""
    cse, ctx, torch = gpu
    rng = np.random.default_rng(44)
    shapes = [(2, 3, 4), (4, 4, 3), (3, 2, 2), (5, 5, 4), (2, 2, 2), (3, 4, 4), (4, 4, 4)]
    ranks = [workloads.scheme_rank(*s) for s in shapes]
    pools = workloads.pools_by_rank(ranks, 420)
    runs = []
    for i, ((n, m, p), r) in enumerate(zip(shapes, ranks)):
        U, V, Wt = workloads.scheme_systems(rng, n, m, p, r, 0.2)
        sc = workloads.Scheme(f"{n}x{m}x{p}:{r}", U, V, Wt)
        kw = dict(seed=i, n_proc=pools[i], weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True)
        if i % 2 == 0:
            kw.update(share_every=8, share_src_pm=50, share_dst_pm=200, share_max_rounds=20)
        runs.append((sc, kw))
    sids = [cse.cse_scheme_load(ctx, *sc.systems) for sc, _ in runs]
    say(f"[gpu] batch of {len(runs)}: {[sc.name for sc, _ in runs]}")
    jobs = cse.cse_launch_batch(ctx, sids, [cse.cse_run_cfg(**kw) for _, kw in runs],
                                torch.cuda.current_stream())
    for (sc, kw), sid, job in zip(runs, sids, jobs):
        ocfg = oracle.make_cfg(**kw)
        info = cse.cse_scheme_info(ctx, sid)
        for c, A in enumerate(sc.systems):
            got = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
            got["prog"] = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
            ref = oracle.run_pool(A, ocfg, comp=c, n_threads=THREADS)
            assert_same(got, ref, f"batch {sc.name} comp {c}")
    for job in jobs:
        cse.cse_job_release(ctx, job)
    for sid in sids:
        cse.cse_scheme_free(ctx, sid)


@pytest.mark.parametrize("rows,cols,p,cap", [(42, 197, 0.2, 40), (331, 64, 0.12, 25), (64, 331, 0.12, 12),
                                             (400, 64, 0.12, 20)])
def test_hbm_state_large_systems(gpu, oracle, rows, cols, p, cap):
    """Systems whose state exceeds the LDS budget keep it in HBM slots
    (shapes of the 6x7x7-r197 W^T and the 8x8x8-r331 U and W^T components,
    the largest of the serving stream, and the 400 x 64 stress shape of an
    8x8x8 scheme of rank 400)."""
    A = workloads.random_system(rows + 7 * cols, rows, cols, p)
    kw = dict(seed=3, n_proc=12, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True, step_cap=cap)
    check_workload(gpu, oracle, [A], kw, f"hbm-state {rows}x{cols}")


def test_many_variables_single_wave(gpu, oracle):
    """A system with more than 2047 variables (n_x + its fresh-variable
    bound) keeps one wave per unit: its candidates need 64-bit entries, so
    loading gives it HBM | RANGE without waves and layouts with waves are
    refused; its units equal the oracle's."""
    cse, ctx, torch = gpu
    A = workloads.random_system(4400, 40, 2200, 0.05)
    sid = cse.cse_system_load(ctx, A)
    info = cse.cse_scheme_info(ctx, sid)
    assert info[0][1] + info[0][2] > 2047
    assert cse.cse_scheme_layout(ctx, sid, 0) == cse.CSE_LAYOUT_HBM | cse.CSE_LAYOUT_RANGE
    with pytest.raises(cse.CseError, match="CSE_EINVAL"):
        cse.cse_scheme_layout(ctx, sid, 0, cse.CSE_LAYOUT_HBM | cse.CSE_LAYOUT_RANGE | cse.CSE_LAYOUT_WAVES4)
    cse.cse_scheme_free(ctx, sid)
    kw = dict(seed=4, n_proc=6, weights={"gi": 3, "ga": 1, "wr": 1, "mix": 1}, step_cap=4)
    check_workload(gpu, oracle, [A], kw, "many variables 40x2200")


def test_sharing_6x6x6_full_size_sampled(gpu, oracle):
    """The 6x6x6 workload at full size (16384 processes, sharing every 32
    steps): every sampled unit equals the oracle continued from its last
    restart prefix and epoch (sources and copies are GPU outputs, the rest of
    the trajectory depends only on the unit's own draws); every sampled
    program re-expands to its input and ends with no repeated pair."""
    from cse_helpers import is_terminal
    cse, ctx, torch = gpu
    wl = workloads.plain_6x6x6()
    sc, rs = wl.schemes[0], wl.runs[0]
    kw = rs.as_kwargs()
    say(f"[gpu] 6x6x6 full size: n_proc {rs.n_proc}, sharing every {rs.share_every}")
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    info = cse.cse_scheme_info(ctx, sid)
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    cse.cse_wait(ctx, job)
    rng = np.random.default_rng(0)
    for c, A in enumerate(sc.systems):
        got = cse.cse_get_unit_results(ctx, job, c, rs.n_proc)
        prog = cse.cse_get_programs(ctx, job, c, rs.n_proc, info[c][2])
        assert got["epoch"].max() > 0 and (got["steps"] > 0).all()
        best = int(np.argmin(got["cost"]))
        gp_units = np.flatnonzero(got["strat"] == 6)
        assert gp_units.size > 0
        sample = np.unique(np.concatenate([[0, best], rng.choice(rs.n_proc, 14, replace=False),
                                           np.flatnonzero(got["epoch"] > 0)[:8], gp_units[:4]]))
        for u in sample:
            F = check_program(A, prog[u, :got["steps"][u]], int(got["cost"][u]))
            assert is_terminal(F)
        init = np.zeros((len(sample), prog.shape[1], 3), np.int32)
        lens = got["k0"][sample]
        for j, u in enumerate(sample):
            init[j, :lens[j]] = prog[u, :lens[j]]
        ocfg = oracle.make_cfg(**dict(kw, share_every=0))
        ref = oracle.run_pool(A, ocfg, comp=c, procs=sample, init_prog=init, init_len=lens,
                              init_epoch=got["epoch"][sample], n_threads=THREADS)
        bad = [int(u) for j, u in enumerate(sample) if not np.array_equal(ref["prog"][j], prog[u])]
        assert not bad, f"comp {c}: units {bad} differ from the oracle continuation"
        assert np.array_equal(ref["cost"], got["cost"][sample])
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)


@pytest.mark.parametrize("rows,cols,p,hi,n_proc,every", [
    (30, 12, 0.35, None, 4096, 2), (24, 12, 0.4, None, 16384, 3), (40, 16, 0.3, 8, 16384, 4),
    (70, 14, 0.25, 8, 5000, 2)])
def test_sharing_large_pools_every_unit(gpu, oracle, rows, cols, p, hi, n_proc, every):
    """Sharing rounds (Sec. 3.5.2, top 1% -> 10%) on pools of thousands of
    units, whose source ranking spans many 256-unit blocks and key tiles:
    every unit, restarts included, equals the oracle's full pool run."""
    A = workloads.random_system(rows * 100 + cols, rows, cols, p, 1, hi)
    kw = dict(seed=7, n_proc=n_proc, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True,
              share_every=every, share_src_pm=10, share_dst_pm=100, share_max_rounds=64)
    got, _ = check_workload(gpu, oracle, [A], kw, f"share {rows}x{cols} pool {n_proc} every {every}")
    assert (got[0]["epoch"] > 0).sum() > n_proc // 10


def test_batch_large_pools_with_sharing(gpu, oracle):
    """A batch whose pools hold 600-3000 units each, all sharing every 3
    steps: every unit of every pool equals the oracle's run of its job."""
    cse, ctx, torch = gpu
    rng = np.random.default_rng(46)
    shapes = [(2, 3, 2), (3, 3, 2), (2, 2, 3), (3, 2, 3), (2, 2, 2)]
    ranks = [workloads.scheme_rank(*s) for s in shapes]
    pools = workloads.pools_by_rank(ranks, 8192)
    assert min(pools) > 256
    runs = []
    for i, ((n, m, p), r) in enumerate(zip(shapes, ranks)):
        U, V, Wt = workloads.scheme_systems(rng, n, m, p, r, 0.3)
        sc = workloads.Scheme(f"{n}x{m}x{p}:{r}", U, V, Wt)
        kw = dict(seed=20 + i, n_proc=pools[i], weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True,
                  share_every=3, share_src_pm=10, share_dst_pm=100, share_max_rounds=64)
        runs.append((sc, kw))
    sids = [cse.cse_scheme_load(ctx, *sc.systems) for sc, _ in runs]
    say(f"[gpu] batch with sharing, pools {pools}")
    jobs = cse.cse_launch_batch(ctx, sids, [cse.cse_run_cfg(**kw) for _, kw in runs],
                                torch.cuda.current_stream())
    restarted = 0
    for (sc, kw), sid, job in zip(runs, sids, jobs):
        ocfg = oracle.make_cfg(**kw)
        info = cse.cse_scheme_info(ctx, sid)
        for c, A in enumerate(sc.systems):
            got = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
            got["prog"] = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
            ref = oracle.run_pool(A, ocfg, comp=c, n_threads=THREADS)
            assert_same(got, ref, f"batch {sc.name} comp {c}")
            restarted += int((got["epoch"] > 0).sum())
    assert restarted > 0
    for job in jobs:
        cse.cse_job_release(ctx, job)
    for sid in sids:
        cse.cse_scheme_free(ctx, sid)


def test_server_continuous_batching(gpu, oracle):
    """Jobs submitted while others run join later rounds (continuous
    batching); admission respects the memory budget; every job's units equal
    those of the oracle, i.e. the same alone and in the mix."""
    cse, ctx, torch = gpu
    rng = np.random.default_rng(55)
    shapes = [(3, 3, 3), (4, 3, 2), (2, 4, 4), (4, 4, 4), (3, 2, 3), (4, 4, 2)]
    jobs = []
    for i, (n, m, p) in enumerate(shapes):
        r = workloads.scheme_rank(n, m, p)
        U, V, Wt = workloads.scheme_systems(rng, n, m, p, r, 0.2)
        kw = dict(seed=100 + i, n_proc=48 + 16 * i, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True)
        if i % 3 != 1:
            kw.update(share_every=6, share_src_pm=50, share_dst_pm=150, share_max_rounds=30)
        jobs.append(((U, V, Wt), kw, cse.cse_scheme_load(ctx, U, V, Wt)))
    srv = cse.cse_server_create(ctx, max_state_bytes=24 << 20, round_steps=5, stream=torch.cuda.current_stream())
    ids = {}
    say(f"[gpu] server: {len(jobs)} jobs, budget 24 MiB")
    pending = list(range(len(jobs)))
    ticks = 0
    max_running = 0
    while pending or any(cse.cse_server_job_info(srv, j)[0] != cse.CSE_JOB_DONE for j in ids.values()):
        if pending and ticks % 2 == 0:
            i = pending.pop(0)
            ids[i] = cse.cse_server_submit(srv, jobs[i][2], cse.cse_run_cfg(**jobs[i][1]))
        running, queued = cse.cse_server_tick(srv)
        max_running = max(max_running, running)
        ticks += 1
        assert ticks < 2000
    assert max_running >= 2, "jobs should overlap on the device"
    for i, ((U, V, Wt), kw, sid) in enumerate(jobs):
        job = ids[i]
        st, (t_sub, t_adm, t_done) = cse.cse_server_job_info(srv, job)
        assert st == cse.CSE_JOB_DONE and t_sub <= t_adm <= t_done
        ocfg = oracle.make_cfg(**kw)
        info = cse.cse_scheme_info(ctx, sid)
        for c, A in enumerate((U, V, Wt)):
            got = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
            got["prog"] = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
            ref = oracle.run_pool(A, ocfg, comp=c, n_threads=THREADS)
            assert_same(got, ref, f"server job {i} comp {c}")
        cse.cse_server_release(srv, job)
    cse.cse_server_destroy(srv)
    tiny = cse.cse_server_create(ctx, max_state_bytes=1000, round_steps=5)
    with pytest.raises(cse.CseError) as e:
        cse.cse_server_submit(tiny, jobs[0][2], cse.cse_run_cfg(**jobs[0][1]))
    assert e.value.status == -2
    cse.cse_server_destroy(tiny)
    for _, _, sid in jobs:
        cse.cse_scheme_free(ctx, sid)


@pytest.mark.parametrize("rows,cols,p", [(42, 197, 0.2), (100, 60, 0.25)])
def test_large_candidate_sets_with_sharing(gpu, oracle, rows, cols, p):
    """Large candidate sets (gi over per-variable ranges) through sharing
    rounds: restarted units rebuild both candidate orderings after replay."""
    A = workloads.random_system(rows * 3 + cols, rows, cols, p)
    kw = dict(seed=8, n_proc=24, weights={"gi": 4, "mix": 2, "wr": 1}, proc0_greedy=True, step_cap=36,
              share_every=6, share_src_pm=100, share_dst_pm=400, share_max_rounds=5)
    got, _ = check_workload(gpu, oracle, [A], kw, f"adj+share {rows}x{cols}")
    assert got[0]["epoch"].max() > 0


@pytest.mark.parametrize("rows,cols,p,hi", [
    (7, 5, 0.5, None), (49, 16, 0.3, 8), (63, 33, 0.2, 10), (160, 36, 0.15, 12),
    (42, 197, 0.2, None), (512, 12, 0.4, 6)])
def test_count_paths_match(gpu, oracle, rows, cols, p, hi):
    """The input's pair counts from popcounts and from the int8 Gram product
    on the matrix cores (Sec. 3.3) give the same runs, equal to the oracle's."""
    A = workloads.random_system(rows * 7919 + cols, rows, cols, p, 1, hi)
    kw = dict(seed=rows * cols, n_proc=64, weights=dict(ALL_W), proc0_greedy=True)
    ref = compare(oracle, [A], kw, "count paths")
    cse = gpu[0]
    for path in (cse.CSE_COUNT_POPCOUNT, cse.CSE_COUNT_MFMA, cse.CSE_COUNT_AUTO):
        say(f"[gpu] count path {path}: system {rows}x{cols}")
        got = run_gpu(gpu, [A], dict(kw, count_path=path))
        assert_same(got[0], ref[0], f"count path {path} {rows}x{cols}")


def test_cancel_keeps_prefixes_and_poll_reports_best(gpu, oracle):
    """cse_cancel stops a running launch: every unit keeps a prefix of the
    run it would have made (Algorithm 1 is deterministic per unit), its cost
    matches that prefix, cse_wait reports the cancellation; a relaunch clears
    it; cse_poll gives each pool's lowest cost."""
    from cse_helpers import naive_count, replay
    cse, ctx, torch = gpu
    A = workloads.random_system(4242, 42, 197, 0.2)
    n = 4096
    kw = dict(seed=11, n_proc=n, weights={"gi": 1})
    sid = cse.cse_system_load(ctx, A)
    info = cse.cse_scheme_info(ctx, sid)
    st = torch.cuda.current_stream()
    say(f"[gpu] cancel: 42x197, {n} gi units")
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), st)
    cse.cse_cancel(ctx, job)
    with pytest.raises(cse.CseError) as err:
        cse.cse_wait(ctx, job)
    assert "CSE_ECANCELED" in str(err.value)
    done, best = cse.cse_poll(ctx, job, best=True)
    r = cse.cse_get_unit_results(ctx, job, 0, n)
    prog = cse.cse_get_programs(ctx, job, 0, n, max(1, info[0][2]))
    assert done and best[0] == int(r["cost"].min()) and best[1:] == [-1, -1]
    procs = list(range(0, n, 512))
    ref = oracle.run_pool(A, oracle.make_cfg(**dict(kw, step_cap=64)), procs=procs, n_threads=THREADS)
    stopped = 0
    for i, u in enumerate(procs):
        t = int(r["steps"][u])
        k = min(t, 64)
        assert (prog[u][:k] == ref["prog"][i][:k]).all(), f"unit {u}: cancelled program is not a prefix"
        _, cs = replay(A, prog[u][:t])
        assert int(r["cost"][u]) == naive_count(A) - sum(c - 1 for c in cs)
        stopped += t < info[0][2]
    assert stopped == len(procs), "cancellation did not stop the sampled units"
    # A relaunch clears the request and runs to its cap like the oracle.
    cse.cse_relaunch(ctx, job, cse.cse_run_cfg(**dict(kw, step_cap=40)), st)
    cse.cse_wait(ctx, job)
    r = cse.cse_get_unit_results(ctx, job, 0, n)
    prog = cse.cse_get_programs(ctx, job, 0, n, max(1, info[0][2]))
    for i, u in enumerate(procs):
        assert int(r["steps"][u]) == min(40, int(ref["steps"][i]))
        assert (prog[u][:40] == ref["prog"][i][:40]).all()
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)


def run_loaded(gpu, sid, kw):
    """Run a job on an already loaded one-component scheme."""
    cse, ctx, torch = gpu
    info = cse.cse_scheme_info(ctx, sid)
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    cse.cse_wait(ctx, job)
    r = cse.cse_get_unit_results(ctx, job, 0, kw["n_proc"])
    r["prog"] = cse.cse_get_programs(ctx, job, 0, kw["n_proc"], max(1, info[0][2]))
    return job, r


@pytest.mark.parametrize("rows,cols,p,cap", [(60, 18, 0.3, 0), (160, 36, 0.15, 40), (42, 197, 0.2, 30)])
def test_layouts_and_autotune_same_results(gpu, oracle, rows, cols, p, cap):
    """Every layout (unit state in LDS or in HBM slots, gi over masks or over
    ranges, one, two or four waves per unit) and the autotuner's choice
    reproduce the oracle's runs."""
    cse, ctx, torch = gpu
    A = workloads.random_system(rows * 31 + cols, rows, cols, p)
    kw = dict(seed=rows + 5, n_proc=64, weights=dict(ALL_W), proc0_greedy=True, step_cap=cap)
    ref = compare(oracle, [A], kw, "layouts")[0]
    sid = cse.cse_system_load(ctx, A)
    tried = 0
    W2, W4 = cse.CSE_LAYOUT_WAVES2, cse.CSE_LAYOUT_WAVES4
    for lay in (0, 1, 2, 3, 7, 2 | W2, 2 | W4, 3 | W2, 3 | W4, 7 | W2, 7 | W4):
        try:
            cse.cse_scheme_layout(ctx, sid, 0, lay)
        except cse.CseError as e:
            assert "CSE_ENOMEM" in str(e) and (not lay & cse.CSE_LAYOUT_HBM or lay & cse.CSE_LAYOUT_LDS_TABLES)
            continue
        assert cse.cse_scheme_layout(ctx, sid, 0) == lay
        say(f"[gpu] layout {lay}: system {rows}x{cols}")
        job, got = run_loaded(gpu, sid, kw)
        with pytest.raises(cse.CseError, match="CSE_EBUSY"):
            cse.cse_scheme_layout(ctx, sid, 0, (lay + 1) % 4)
        cse.cse_job_release(ctx, job)
        assert_same(got, ref, f"layout {lay} {rows}x{cols}")
        tried += 1
    assert tried >= 3
    for bad in (4, 5, 6, 8, 1 | W4, 24, 2 | 24, 32, -2 & 0xFF):
        with pytest.raises(cse.CseError, match="CSE_EINVAL"):
            cse.cse_scheme_layout(ctx, sid, 0, bad)
    say(f"[gpu] autotune: system {rows}x{cols}")
    chosen = cse.cse_autotune(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    assert chosen[0] == cse.cse_scheme_layout(ctx, sid, 0) and chosen[1:] == [-1, -1]
    job, got = run_loaded(gpu, sid, kw)
    cse.cse_job_release(ctx, job)
    assert_same(got, ref, f"autotuned layout {chosen[0]} {rows}x{cols}")
    cse.cse_scheme_free(ctx, sid)


def test_range_form_wide_weights(gpu, oracle):
    """A pair held by 300 of 320 rows gives weights c - 1 of nine bits, so the
    range form's weight planes take three 16-byte groups per word; every
    range layout (one and four waves, tables in the slot, in LDS or in the
    LDS budget) reproduces the oracle's runs."""
    cse, ctx, torch = gpu
    A = workloads.random_system(9321, 320, 14, 0.25)
    A[:300, 0] = 1
    A[:300, 1] = 1
    kw = dict(seed=77, n_proc=64, weights=dict(ALL_W), proc0_greedy=True, step_cap=24)
    ref = compare(oracle, [A], kw, "wide weights")[0]
    sid = cse.cse_system_load(ctx, A)
    W4 = cse.CSE_LAYOUT_WAVES4
    for lay in (2, 3, 2 | W4, 3 | W4, 7 | W4):
        cse.cse_scheme_layout(ctx, sid, 0, lay)
        say(f"[gpu] wide weights: layout {lay}")
        job, got = run_loaded(gpu, sid, kw)
        cse.cse_job_release(ctx, job)
        assert_same(got, ref, f"wide weights, layout {lay}")
    cse.cse_scheme_free(ctx, sid)


def test_range_form_gaps_at_word_edges(gpu, oracle):
    """Greedy-Intersections (Sec. 3.4.2) in the range form reads p's canonical
    range less p, and b's range of the second ordering less the pair's one or
    two entries, as windows with a gap over 32-candidate plane words.  On a
    45 x 150 system of the batch's W^T shape (4490 candidates at the first
    step) twin pairs (a, b, +-) straddle a word boundary in both orderings, so
    gaps of two entries split across two words and gaps at a word's first or
    last bit all occur; every range layout reproduces the oracle's gi-only
    runs."""
    from cse_helpers import pair_counts
    cse, ctx, torch = gpu
    A = workloads.random_system(7000, 45, 150, 0.2)
    pc = pair_counts(A)
    canon = sorted(k for k, c in pc.items() if c >= 2)
    second = sorted(canon, key=lambda t: (t[1], t[0], t[2]))
    def straddling(lst):
        return [i for i in range(31, len(lst) - 1, 32) if lst[i][:2] == lst[i + 1][:2]]
    assert len(canon) == 4490
    assert straddling(canon) and straddling(second), "the input no longer holds both word-edge cases"
    kw = dict(seed=5, n_proc=32, weights={"gi": 1}, proc0_greedy=False, step_cap=8)
    ref = compare(oracle, [A], kw, "gaps at word edges")[0]
    sid = cse.cse_system_load(ctx, A)
    W2, W4 = cse.CSE_LAYOUT_WAVES2, cse.CSE_LAYOUT_WAVES4
    tried = []
    for lay in (2, 3, 7, 2 | W4, 3 | W2, 3 | W4, 7 | W4):
        try:
            cse.cse_scheme_layout(ctx, sid, 0, lay)
        except cse.CseError as e:  # unit state or full tables that do not fit LDS
            assert "CSE_ENOMEM" in str(e) and (not lay & cse.CSE_LAYOUT_HBM or lay & cse.CSE_LAYOUT_LDS_TABLES)
            continue
        say(f"[gpu] gaps at word edges: layout {lay}")
        job, got = run_loaded(gpu, sid, kw)
        cse.cse_job_release(ctx, job)
        assert_same(got, ref, f"gaps at word edges, layout {lay}")
        tried.append(lay)
    assert {3, 3 | W2, 3 | W4} <= set(tried)
    cse.cse_scheme_free(ctx, sid)


def test_server_cancel_queued_and_running(gpu, oracle):
    """A queued server job cancelled before admission never runs; a running
    one stops at the end of its round and keeps prefixes of the oracle's runs;
    cse_wait reports both as cancelled."""
    from cse_helpers import naive_count, replay
    cse, ctx, torch = gpu
    A = workloads.random_system(6060, 49, 16, 0.3, 1, 8)
    kw = dict(seed=21, n_proc=128, weights=dict(ALL_W), proc0_greedy=True)
    sid = cse.cse_system_load(ctx, A)
    info = cse.cse_scheme_info(ctx, sid)
    srv = cse.cse_server_create(ctx, max_state_bytes=64 << 20, round_steps=2, stream=torch.cuda.current_stream())
    ja = cse.cse_server_submit(srv, sid, cse.cse_run_cfg(**kw))
    jb = cse.cse_server_submit(srv, sid, cse.cse_run_cfg(**dict(kw, seed=22)))
    say("[gpu] server cancel: one queued, one running")
    cse.cse_cancel(ctx, jb)
    assert cse.cse_server_job_info(srv, jb)[0] == cse.CSE_JOB_DONE
    with pytest.raises(cse.CseError, match="CSE_ECANCELED"):
        cse.cse_wait(ctx, jb)
    running, queued = cse.cse_server_tick(srv)
    assert (running, queued) == (1, 0)
    cse.cse_cancel(ctx, ja)
    running, queued = cse.cse_server_tick(srv)
    assert (running, queued) == (0, 0)
    assert cse.cse_server_job_info(srv, ja)[0] == cse.CSE_JOB_DONE
    with pytest.raises(cse.CseError, match="CSE_ECANCELED"):
        cse.cse_wait(ctx, ja)
    got = cse.cse_get_unit_results(ctx, ja, 0, kw["n_proc"])
    prog = cse.cse_get_programs(ctx, ja, 0, kw["n_proc"], max(1, info[0][2]))
    ref = oracle.run_pool(A, oracle.make_cfg(**kw), n_threads=THREADS)
    assert (got["steps"] <= 4).all() and (got["steps"] < ref["steps"]).any()
    for u in range(kw["n_proc"]):
        t = int(got["steps"][u])
        assert (prog[u][:t] == ref["prog"][u][:t]).all(), f"unit {u}: not a prefix"
        _, cs = replay(A, prog[u][:t])
        assert int(got["cost"][u]) == naive_count(A) - sum(c - 1 for c in cs)
    cse.cse_server_release(srv, ja)
    cse.cse_server_release(srv, jb)
    cse.cse_server_destroy(srv)
    cse.cse_scheme_free(ctx, sid)


def test_randomized_configurations(gpu, oracle):
    """A seeded sweep over shapes (1..8 row words), densities, strategy
    mixes, step caps, gr probabilities, sharing schedules, count paths and
    layouts: every unit equals the oracle's."""
    cse, ctx, torch = gpu
    rng = np.random.default_rng(2512)
    names = ["g", "ga", "wr", "gr", "gi", "mix"]
    for case in range(16):
        rows = int(rng.choice([3, 17, 40, 64, 65, 100, 130, 250, 380, 511]))
        cols = int(rng.integers(4, 48 if rows <= 100 else 20))
        p = float(rng.uniform(0.08, 0.45 if rows <= 100 else 0.3))
        A = workloads.random_system(int(rng.integers(1 << 30)), rows, cols, p)
        weights = {n: int(w) for n, w in zip(names, rng.integers(0, 4, len(names))) if w}
        weights = weights or {"gi": 1}
        kw = dict(seed=int(rng.integers(1 << 62)), n_proc=int(rng.integers(1, 97)), weights=weights,
                  mix_weights=tuple(int(x) for x in rng.integers(1, 9, 4)), proc0_greedy=bool(rng.integers(2)),
                  gr_p_q16=int(rng.integers(0, 65537)),
                  step_cap=int(rng.choice([0, 0, 3, 11])) if rows <= 100 else int(rng.choice([3, 11, 30])))
        if rng.integers(2):
            kw.update(share_every=int(rng.integers(1, 9)), share_src_pm=int(rng.integers(1, 300)),
                      share_dst_pm=int(rng.integers(0, 1001)), share_max_rounds=int(rng.integers(1, 20)))
        path = int(rng.choice([cse.CSE_COUNT_POPCOUNT, cse.CSE_COUNT_MFMA]))
        ref = compare(oracle, [A], kw, "random")[0]
        sid = cse.cse_system_load(ctx, A)
        lay = int(rng.integers(0, 4))
        if lay == 3 and case % 2:
            lay = 7
        if lay & cse.CSE_LAYOUT_RANGE:
            lay |= int(rng.choice([0, cse.CSE_LAYOUT_WAVES2, cse.CSE_LAYOUT_WAVES4]))
        try:
            cse.cse_scheme_layout(ctx, sid, 0, lay)
        except cse.CseError as e:
            assert "CSE_ENOMEM" in str(e)
            lay = cse.cse_scheme_layout(ctx, sid, 0)
        say(f"[gpu] random case {case}: {rows}x{cols} p={p:.2f} n_proc={kw['n_proc']} layout {lay} path {path}")
        job, got = run_loaded(gpu, sid, dict(kw, count_path=path))
        cse.cse_job_release(ctx, job)
        cse.cse_scheme_free(ctx, sid)
        assert_same(got, ref, f"random case {case} ({rows}x{cols}, layout {lay})")


def run_driver_gpu(gpu, systems, kw, layouts=None, **dkw):
    cse, ctx, torch = gpu
    sid = cse.cse_scheme_load(ctx, *systems) if len(systems) == 3 else cse.cse_system_load(ctx, systems[0])
    info = cse.cse_scheme_info(ctx, sid)
    for c, lay in enumerate(layouts or []):
        cse.cse_scheme_layout(ctx, sid, c, lay)
    job, its = cse.cse_run_driver(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream(), **dkw)
    out = dict(iterations=its, totals=cse.cse_driver_totals(ctx, job),
               best=[cse.cse_driver_best(ctx, job, c) for c in range(len(systems))], last=[])
    for c in range(len(systems)):
        r = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
        r["prog"] = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
        out["last"].append(r)
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    return out


def check_driver(gpu, oracle, systems, kw, label, layouts=None, **dkw):
    say(f"[gpu] driver {label}: shapes {[A.shape for A in systems]} n_proc {kw['n_proc']} {dkw}")
    got = run_driver_gpu(gpu, systems, kw, layouts, **dkw)
    ref = oracle.run_driver(systems, oracle.make_cfg(**kw), n_threads=THREADS, **dkw)
    assert got["iterations"] == ref["iterations"], label
    assert got["totals"] == ref["totals"], label
    for c in range(len(systems)):
        g, r = got["best"][c], ref["best"][c]
        assert (g["cost"], g["iteration"], g["proc"]) == (r["cost"], r["iteration"], r["proc"]), f"{label} comp {c}"
        assert np.array_equal(g["prog"], r["prog"]), f"{label} comp {c}: best programs differ"
        check_program(systems[c], g["prog"], g["cost"])
        assert_same(got["last"][c], ref["last"][c], f"{label} comp {c} last iteration")
    return got


def test_driver_converges_like_oracle(gpu, oracle):
    """Outer iterations (Sec. 3.5.1-3.5.2, Sec. 4 rule): improvements after
    the first iteration, restarts from best prefixes, the same stop."""
    S = [workloads.random_system(61 + i, 49, 16, 0.3, 1, 8) for i in range(3)]
    kw = dict(seed=9, n_proc=16, weights={"gi": 8, "ga": 4, "gr": 2, "wr": 1, "mix": 1}, proc0_greedy=True)
    got = check_driver(gpu, oracle, S, kw, "49x16 x3", patience=3, max_iterations=40)
    assert got["iterations"] > 4 and got["totals"][-1] < got["totals"][0]


def test_driver_with_sharing_rounds_and_layouts(gpu, oracle):
    """Sharing rounds inside every iteration (their draws keyed by the
    iteration), in LDS and in HBM slots with the range form of gi."""
    wl = workloads.plain_4x4x4()
    S = wl.schemes[0].systems
    kw = dict(seed=7, n_proc=64, weights={"gi": 8, "ga": 4, "gr": 2, "wr": 1, "mix": 1}, proc0_greedy=True,
              share_every=4, share_src_pm=50, share_dst_pm=300, share_max_rounds=64)
    check_driver(gpu, oracle, S, kw, "4x4x4 sharing", patience=2, max_iterations=5)
    check_driver(gpu, oracle, S, kw, "4x4x4 sharing hbm+range", layouts=[3 | 16, 1, 2 | 8], patience=2,
                 max_iterations=5)


def test_driver_epochs_past_ten_bits(gpu, oracle):
    """Sharing after every step with every active non-source unit a target,
    over many outer iterations: unit epochs pass 1023, where the step and
    coin draws carry the epoch's high bits.  The GPU equals the oracle."""
    A = workloads.random_system(4321, 30, 12, 0.35)
    kw = dict(seed=9, n_proc=48, weights={"gi": 8, "ga": 4, "gr": 2, "wr": 1, "mix": 1}, proc0_greedy=True,
              share_every=1, share_src_pm=25, share_dst_pm=1000, share_max_rounds=20)
    got = check_driver(gpu, oracle, [A], kw, "epochs past 1023", patience=1000, max_iterations=60)
    assert int(got["last"][0]["epoch"].min()) > 1100


def test_driver_tiny_and_edge_settings(gpu, oracle):
    """gi only on the tiny system; every process restarts from a prefix;
    no restarts; a single iteration."""
    wl = workloads.tiny_2x2x2()
    S = wl.schemes[0].systems
    kw = wl.runs[0].as_kwargs()
    check_driver(gpu, oracle, S, kw, "tiny", patience=2, max_iterations=10)
    check_driver(gpu, oracle, S, dict(kw, n_proc=32), "tiny all restart", reinit_pm=1000, patience=1,
                 max_iterations=4)
    A = workloads.random_system(77, 40, 14, 0.3, 1, 8)
    kw2 = dict(seed=5, n_proc=48, weights=dict(ALL_W), proc0_greedy=True)
    check_driver(gpu, oracle, [A], kw2, "no restarts", reinit_pm=0, patience=100, max_iterations=3)
    got = check_driver(gpu, oracle, [A], kw2, "one iteration", patience=0, max_iterations=10)
    assert got["iterations"] == 1
    kw3 = dict(kw2, step_cap=7)
    ref3 = oracle.run_driver([A], oracle.make_cfg(**kw3), n_threads=THREADS, patience=2, max_iterations=5)
    got3 = run_driver_gpu(gpu, [A], dict(kw3, count_path=2), patience=2, max_iterations=5)
    assert got3["iterations"] == ref3["iterations"] and got3["totals"] == ref3["totals"]
    assert_same(got3["last"][0], ref3["last"][0], "driver step cap, MFMA count path")
    assert int(got3["last"][0]["steps"].max()) <= 7


def test_driver_rejects_bad_use(gpu):
    cse, ctx, torch = gpu
    A = workloads.random_system(78, 20, 8, 0.3, 1, 6)
    sid = cse.cse_system_load(ctx, A)
    st = torch.cuda.current_stream()
    cfg = cse.cse_run_cfg(n_proc=8, weights={"gi": 1})
    for bad in (dict(max_iterations=0), dict(max_iterations=1025), dict(reinit_pm=1001)):
        with pytest.raises(cse.CseError) as e:
            cse.cse_run_driver(ctx, sid, cfg, st, **bad)
        assert e.value.status == -1 and e.value.job_id is None
    with pytest.raises(cse.CseError) as e:
        cse.cse_run_driver(ctx, sid, cse.cse_run_cfg(n_proc=8, weights={"gi": 1}, iteration=1), st)
    assert e.value.status == -1
    job = cse.cse_launch(ctx, sid, cfg, st)
    cse.cse_wait(ctx, job)
    with pytest.raises(cse.CseError) as e:
        cse.cse_driver_best(ctx, job, 0)
    assert e.value.status == -1
    cse.cse_job_release(ctx, job)
    job, its = cse.cse_run_driver(ctx, sid, cfg, st, patience=1, max_iterations=3)
    with pytest.raises(cse.CseError) as e:
        cse.cse_relaunch(ctx, job)
    assert e.value.status == -1
    with pytest.raises(cse.CseError) as e:
        cse.cse_driver_best(ctx, job, 1)
    assert e.value.status == -1
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)


def test_driver_cancel_from_another_thread(gpu):
    """cse_cancel on another thread stops a long driver run after the
    current iteration; the bests of the completed iterations stay readable."""
    import ctypes
    import threading
    import time
    cse, ctx, torch = gpu
    wl = workloads.plain_4x4x4()
    sid = cse.cse_scheme_load(ctx, *wl.schemes[0].systems)
    cfg = cse.cse_run_cfg(seed=1, n_proc=4096, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True)
    d = cse.CseDriverCfg()
    d.reinit_pm, d.patience, d.max_iterations = 400, 1024, 1024
    job, its, rc = ctypes.c_int32(-1), ctypes.c_int32(0), []
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = cse.load_library()

    def run():
        rc.append(L.cse_run_driver(ctx, sid, ctypes.byref(cfg), ctypes.byref(d), stream, ctypes.byref(job),
                                   ctypes.byref(its)))

    th = threading.Thread(target=run)
    th.start()
    t0 = time.time()
    while job.value <= 0 and time.time() - t0 < 30:
        time.sleep(0.001)
    assert job.value > 0
    time.sleep(0.1)
    cse.cse_cancel(ctx, job.value)
    th.join(60)
    assert not th.is_alive()
    assert rc == [-7], rc
    assert 1 <= its.value < 1024
    totals = cse.cse_driver_totals(ctx, job.value)
    assert len(totals) == its.value
    best = [cse.cse_driver_best(ctx, job.value, c) for c in range(3)]
    assert sum(b["cost"] for b in best) == totals[-1]
    for c, A in enumerate(wl.schemes[0].systems):
        check_program(A, best[c]["prog"], best[c]["cost"])
    cse.cse_job_release(ctx, job.value)
    cse.cse_scheme_free(ctx, sid)


@pytest.mark.parametrize("rows,cols,p,every", [(60, 18, 0.3, 1), (160, 36, 0.15, 3), (24, 80, 0.2, 4)])
def test_hbm_units_resume_across_rounds(gpu, oracle, rows, cols, p, every):
    """Units with state in HBM slots resume from the slot between sharing
    rounds unless they were restarted; with rounds every few steps and many
    targets, resumed and replayed units alternate, in both HBM layouts."""
    cse, ctx, torch = gpu
    A = workloads.random_system(rows * 7 + cols, rows, cols, p)
    kw = dict(seed=rows + every, n_proc=48, weights=dict(ALL_W), proc0_greedy=True, share_every=every,
              share_src_pm=60, share_dst_pm=400, share_max_rounds=1000)
    ref = compare(oracle, [A], kw, "resume")[0]
    assert ref["epoch"].max() > 1
    for lay in (cse.CSE_LAYOUT_HBM, cse.CSE_LAYOUT_HBM | cse.CSE_LAYOUT_RANGE,
                cse.CSE_LAYOUT_HBM | cse.CSE_LAYOUT_RANGE | cse.CSE_LAYOUT_WAVES4,
                cse.CSE_LAYOUT_HBM | cse.CSE_LAYOUT_RANGE | cse.CSE_LAYOUT_LDS_TABLES,
                cse.CSE_LAYOUT_HBM | cse.CSE_LAYOUT_RANGE | cse.CSE_LAYOUT_LDS_TABLES | cse.CSE_LAYOUT_WAVES2):
        sid = cse.cse_system_load(ctx, A)
        cse.cse_scheme_layout(ctx, sid, 0, lay)
        say(f"[gpu] resume: system {rows}x{cols} every {every} layout {lay}")
        job, got = run_loaded(gpu, sid, kw)
        cse.cse_job_release(ctx, job)
        cse.cse_scheme_free(ctx, sid)
        assert_same(got, ref, f"resume {rows}x{cols} layout {lay}")


def test_hybrid_best_over_jobs(gpu, oracle):
    """Component-wise hybrid (Sec. 4): per component, the lowest cost over a
    gi-only job, a ga-only job and a driver job, with the job and process that
    hold it (ties: the earlier job, then the lower process).  The expected
    hybrid is computed from the oracle's runs of the same jobs; each chosen
    program re-expands exactly.  Jobs of different schemes are refused."""
    cse, ctx, torch = gpu
    wl = workloads.plain_4x4x4(n_proc=256)
    S = wl.schemes[0].systems
    sid = cse.cse_scheme_load(ctx, *S)
    st = torch.cuda.current_stream()
    jobs, ref_best = [], []
    for w in ({"gi": 1}, {"ga": 1}):
        kw = dict(seed=4, n_proc=256, weights=w)
        j = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), st)
        cse.cse_wait(ctx, j)
        jobs.append(j)
        per_comp = []
        for c, A in enumerate(S):
            r = oracle.run_pool(A, oracle.make_cfg(**kw), comp=c, n_threads=THREADS)
            u = int(np.lexsort((np.arange(256), r["cost"]))[0])
            per_comp.append((int(r["cost"][u]), u))
        ref_best.append(per_comp)
    dkw = dict(seed=5, n_proc=256, weights=dict(workloads.PAPER_WEIGHTS))
    dj, _ = cse.cse_run_driver(ctx, sid, cse.cse_run_cfg(**dkw), st, patience=2, max_iterations=6)
    jobs.append(dj)
    dref = oracle.run_driver(S, oracle.make_cfg(**dkw), patience=2, max_iterations=6, n_threads=THREADS)
    ref_best.append([(b["cost"], b["proc"]) for b in dref["best"]])
    hyb = cse.cse_hybrid_best(ctx, jobs)
    assert len(hyb) == 3
    for c in range(3):
        want = None
        for j, per_comp in zip(jobs, ref_best):
            cost, u = per_comp[c]
            if want is None or cost < want[0]:
                want = (cost, j, u)
        assert hyb[c] == want, (c, hyb[c], ref_best)
        cost, j, u = hyb[c]
        if j == dj:
            prog = cse.cse_driver_best(ctx, j, c)["prog"]
        else:
            prog, pc = cse.cse_get_program(ctx, j, c, proc=u)
            assert pc == cost
        check_program(S[c], prog, cost)
    # A job of another scheme (even with the same shapes) is refused.
    sid2 = cse.cse_scheme_load(ctx, *S)
    j2 = cse.cse_launch(ctx, sid2, cse.cse_run_cfg(seed=4, n_proc=64, weights={"gi": 1}), st)
    cse.cse_wait(ctx, j2)
    with pytest.raises(cse.CseError) as e:
        cse.cse_hybrid_best(ctx, [jobs[0], j2])
    assert e.value.status == -1
    cse.cse_job_release(ctx, j2)
    cse.cse_scheme_free(ctx, sid2)
    for j in jobs:
        cse.cse_job_release(ctx, j)
    cse.cse_scheme_free(ctx, sid)


def test_refusals_keep_other_work_going(gpu, oracle):
    """A system whose variable lists alone exceed a workgroup's LDS is refused
    at load (CSE_ENOMEM).  A served job whose device state cannot be
    allocated at admission (far beyond HBM) leaves the queue as failed, and
    the jobs before and after it run to the oracle's results."""
    cse, ctx, torch = gpu
    rng = np.random.default_rng(3)
    big = np.zeros((512, 10000), np.int8)
    for i in range(512):
        big[i, rng.choice(10000, 45, replace=False)] = rng.choice(np.array([-1, 1], np.int8), 45)
    with pytest.raises(cse.CseError) as e:
        cse.cse_system_load(ctx, big)
    assert e.value.status == -2
    huge_sys = workloads.random_system(42 + 7 * 197, 42, 197, 0.2)
    small = workloads.random_system(4321, 30, 12, 0.35)
    hid = cse.cse_system_load(ctx, huge_sys)
    sid = cse.cse_system_load(ctx, small)
    srv = cse.cse_server_create(ctx, max_state_bytes=1 << 52, round_steps=4, stream=torch.cuda.current_stream())
    kws = [dict(seed=1, n_proc=64, weights=dict(ALL_W)), dict(seed=2, n_proc=96, weights=dict(ALL_W))]
    say("[gpu] server with a job far beyond device memory")
    ja = cse.cse_server_submit(srv, sid, cse.cse_run_cfg(**kws[0]))
    jh = cse.cse_server_submit(srv, hid, cse.cse_run_cfg(seed=3, n_proc=1 << 24, weights={"gi": 1}))
    jb = cse.cse_server_submit(srv, sid, cse.cse_run_cfg(**kws[1]))
    for _ in range(500):
        running, queued = cse.cse_server_tick(srv)
        if running == 0 and queued == 0:
            break
    assert cse.cse_server_job_info(srv, jh)[0] == cse.CSE_JOB_FAILED
    with pytest.raises(cse.CseError) as e:
        cse.cse_get_unit_results(ctx, jh, 0, 1)
    assert e.value.status == -2
    for j, kw in ((ja, kws[0]), (jb, kws[1])):
        assert cse.cse_server_job_info(srv, j)[0] == cse.CSE_JOB_DONE
        got = cse.cse_get_unit_results(ctx, j, 0, kw["n_proc"])
        got["prog"] = cse.cse_get_programs(ctx, j, 0, kw["n_proc"], max(1, oracle.bounds(small)[0]))
        assert_same(got, oracle.run_pool(small, oracle.make_cfg(**kw), n_threads=THREADS), "served beside a failure")
        cse.cse_server_release(srv, j)
    cse.cse_server_release(srv, jh)
    cse.cse_server_destroy(srv)
    cse.cse_scheme_free(ctx, hid)
    cse.cse_scheme_free(ctx, sid)


GP_W = {"gp": 4, "gi": 2, "ga": 1, "wr": 1, "mix": 1}


@pytest.mark.parametrize("rows,cols,p,hi,cap", [
    (9, 5, 0.5, None, 0), (40, 16, 0.3, 8, 0), (65, 24, 0.25, 8, 40), (130, 30, 0.2, 10, 30),
    (200, 24, 0.12, 12, 24), (300, 20, 0.2, 8, 20), (330, 16, 0.25, 8, 16), (420, 14, 0.3, 8, 14),
    (511, 10, 0.4, 6, 12)])
def test_greedy_potential_shapes(gpu, oracle, rows, cols, p, hi, cap):
    """Greedy-Potential units (the trial substitution score) over 1..8 row
    words with ragged tails: gp alone, then beside the other strategies."""
    A = workloads.random_system(rows * 977 + cols, rows, cols, p, 1, hi)
    kw = dict(seed=rows * 3 + cols, n_proc=96, weights={"gp": 1}, step_cap=cap)
    got, _ = check_workload(gpu, oracle, [A], kw, f"gp {rows}x{cols}")
    assert (got[0]["strat"] == 6).all()
    kw = dict(kw, seed=kw["seed"] + 1, weights=GP_W, proc0_greedy=True)
    check_workload(gpu, oracle, [A], kw, f"gp mixed {rows}x{cols}")


def test_greedy_potential_6x6x6_and_large_candidate_set(gpu, oracle):
    """gp on the three 6x6x6 components at full size (no step cap) and on a
    42 x 197 system whose candidate set exceeds 2000 pairs."""
    wl = workloads.plain_6x6x6(n_proc=16)
    check_workload(gpu, oracle, wl.schemes[0].systems, dict(seed=5, n_proc=16, weights={"gp": 3, "gi": 1}, step_cap=0),
                   "gp 6x6x6")
    A = workloads.random_system(42 * 31 + 197, 42, 197, 0.2)
    check_workload(gpu, oracle, [A], dict(seed=6, n_proc=12, weights={"gp": 1}, step_cap=12), "gp 42x197")


def test_greedy_potential_layouts_sharing_driver(gpu, oracle):
    """gp units in every layout of the unit state, with sharing rounds, and
    under the outer-iteration driver."""
    cse, ctx, torch = gpu
    for rows, cols, p, cap in ((60, 18, 0.3, 0), (160, 36, 0.15, 25)):
        A = workloads.random_system(rows * 131 + cols, rows, cols, p)
        kw = dict(seed=rows + 9, n_proc=64, weights=GP_W, proc0_greedy=True, step_cap=cap,
                  share_every=3, share_src_pm=150, share_dst_pm=500, share_max_rounds=6)
        ref = compare(oracle, [A], kw, "gp layouts")[0]
        sid = cse.cse_system_load(ctx, A)
        for lay in (0, 1, 2, 3, 7, 3 | cse.CSE_LAYOUT_WAVES4, 2 | cse.CSE_LAYOUT_WAVES2):
            try:
                cse.cse_scheme_layout(ctx, sid, 0, lay)
            except cse.CseError as e:
                assert "CSE_ENOMEM" in str(e)
                continue
            say(f"[gpu] gp layout {lay}: system {rows}x{cols}")
            job, got = run_loaded(gpu, sid, kw)
            cse.cse_job_release(ctx, job)
            assert_same(got, ref, f"gp layout {lay} {rows}x{cols}")
        cse.cse_scheme_free(ctx, sid)
    S = [workloads.random_system(71 + i, 30, 12, 0.3, 1, 8) for i in range(3)]
    check_driver(gpu, oracle, S, dict(seed=8, n_proc=48, weights=GP_W, proc0_greedy=True), "gp driver",
                 patience=2, max_iterations=6)


def test_greedy_potential_mixed_batch_and_relaunch(gpu, oracle):
    """One batched launch where some jobs weight gp and others do not (the
    launch enters the gp body for every segment of its class), with sharing
    on some, run twice (the relaunch reruns the whole batch); then a gp job
    relaunched alone with a new seed: every unit equals its own job's oracle
    run."""
    cse, ctx, torch = gpu
    rng = np.random.default_rng(45)
    shapes = [(3, 3, 3), (2, 3, 4), (4, 3, 3), (3, 2, 4)]
    weights = [{"gp": 1}, dict(ALL_W), dict(GP_W), {"gi": 1, "ga": 1}]
    runs = []
    for i, (n, m, p) in enumerate(shapes):
        r = workloads.scheme_rank(n, m, p)
        U, V, Wt = workloads.scheme_systems(rng, n, m, p, r, 0.25)
        kw = dict(seed=20 + i, n_proc=40 + 8 * i, weights=weights[i], proc0_greedy=bool(i % 2))
        if i >= 2:
            kw.update(share_every=4, share_src_pm=100, share_dst_pm=300, share_max_rounds=8)
        runs.append(((U, V, Wt), kw))
    sids = [cse.cse_scheme_load(ctx, *S) for S, _ in runs]

    def check(job, S, kw, sid, label):
        info = cse.cse_scheme_info(ctx, sid)
        for c, A in enumerate(S):
            got = cse.cse_get_unit_results(ctx, job, c, kw["n_proc"])
            got["prog"] = cse.cse_get_programs(ctx, job, c, kw["n_proc"], max(1, info[c][2]))
            assert_same(got, oracle.run_pool(A, oracle.make_cfg(**kw), comp=c, n_threads=THREADS),
                        f"{label} {A.shape} comp {c}")
            if kw["weights"] == {"gp": 1}:
                assert (got["strat"] == 6).all()

    say(f"[gpu] gp mixed batch: {[S[0].shape for S, _ in runs]}")
    jobs = cse.cse_launch_batch(ctx, sids, [cse.cse_run_cfg(**kw) for _, kw in runs], torch.cuda.current_stream())
    for attempt in range(2):
        if attempt:
            cse.cse_relaunch(ctx, jobs[0], None, torch.cuda.current_stream())
        for j in jobs:
            cse.cse_wait(ctx, j)
        for (S, kw), sid, job in zip(runs, sids, jobs):
            check(job, S, kw, sid, f"gp batch run {attempt}")
    for job in jobs:
        cse.cse_job_release(ctx, job)
    S, kw = runs[0]
    job = cse.cse_launch(ctx, sids[0], cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    kw = dict(kw, seed=99)
    cse.cse_relaunch(ctx, job, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
    cse.cse_wait(ctx, job)
    check(job, S, kw, sids[0], "gp relaunch seed 99")
    cse.cse_job_release(ctx, job)
    for sid in sids:
        cse.cse_scheme_free(ctx, sid)


def test_cancel_then_resume_equals_uncancelled(gpu, oracle):
    """Failure injection from the host: a job cancelled mid-run through its
    host flag and resumed from its units' saved prefixes and epochs ends
    exactly as a run that was never cancelled (every unit against an
    uncancelled launch, sampled units against the oracle); server, driver
    and sharing jobs are refused."""
    cse, ctx, torch = gpu
    A = workloads.random_system(4243, 42, 197, 0.2)
    n = 2048
    kw = dict(seed=12, n_proc=n, weights={"gi": 2, "ga": 1, "wr": 1})
    sid = cse.cse_system_load(ctx, A)
    info = cse.cse_scheme_info(ctx, sid)
    st = torch.cuda.current_stream()

    def results(job):
        r = cse.cse_get_unit_results(ctx, job, 0, n)
        r["prog"] = cse.cse_get_programs(ctx, job, 0, n, max(1, info[0][2]))
        return r

    say(f"[gpu] cancel + resume: 42x197, {n} units")
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), st)
    cse.cse_cancel(ctx, job)
    with pytest.raises(cse.CseError, match="CSE_ECANCELED"):
        cse.cse_wait(ctx, job)
    cut = results(job)
    cse.cse_resume(ctx, job, st)
    cse.cse_wait(ctx, job)
    got = results(job)
    ref_job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), st)
    cse.cse_wait(ctx, ref_job)
    ref = results(ref_job)
    assert (cut["steps"] < ref["steps"]).sum() > n // 2, "the cancellation stopped few units"
    assert_same(got, ref, "resumed vs uncancelled")
    # Oracle samples among the cheaper ga and wr units (gi units of this
    # system take the oracle seconds each); all units were compared above.
    procs = [int(u) for u in np.flatnonzero(np.isin(got["strat"], (1, 2)))[::97][:8]]
    orc = oracle.run_pool(A, oracle.make_cfg(**kw), procs=procs, n_threads=THREADS)
    for i, u in enumerate(procs):
        assert int(got["cost"][u]) == int(orc["cost"][i]) and (got["prog"][u] == orc["prog"][i]).all(), u
    cse.cse_resume(ctx, job, st)  # a finished job: nothing changes
    cse.cse_wait(ctx, job)
    assert_same(results(job), ref, "resume of a finished job")
    cse.cse_job_release(ctx, job)
    cse.cse_job_release(ctx, ref_job)
    share = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**dict(kw, n_proc=64, share_every=4, share_src_pm=100,
                                                                share_dst_pm=300, share_max_rounds=4)), st)
    cse.cse_wait(ctx, share)
    with pytest.raises(cse.CseError, match="CSE_EINVAL"):
        cse.cse_resume(ctx, share, st)
    cse.cse_job_release(ctx, share)
    cse.cse_scheme_free(ctx, sid)


def test_units_independent_of_pool_size(gpu):
    """Without sharing a unit's result depends only on its process index: a
    pool of 384 processes reproduces the first 384 units of a pool of 1536
    field by field (the premise of sharding a pool by process index)."""
    cse, ctx, torch = gpu
    wl = workloads.plain_4x4x4()
    sc = wl.schemes[0]
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    info = cse.cse_scheme_info(ctx, sid)
    out = {}
    for n in (1536, 384):
        kw = dict(seed=21, n_proc=n, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True)
        say(f"[gpu] pool of {n}")
        job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), torch.cuda.current_stream())
        cse.cse_wait(ctx, job)
        out[n] = []
        for c in range(3):
            r = cse.cse_get_unit_results(ctx, job, c, n)
            r["prog"] = cse.cse_get_programs(ctx, job, c, n, max(1, info[c][2]))
            out[n].append(r)
        cse.cse_job_release(ctx, job)
    for c in range(3):
        big = {k: v[:384] for k, v in out[1536][c].items() if k != "finish"}
        small = {k: v for k, v in out[384][c].items() if k != "finish"}
        assert_same(small, big, f"pool size comp {c}")
    cse.cse_scheme_free(ctx, sid)


def _flip_schemes():
    from cse_helpers import standard_scheme
    g = read_golden("strassen_2x2x2.txt")
    S = [np.array([[int(x) for x in r] for r in g[k]], np.int8) for k in ("U", "V", "Wt")]
    out = [((2, 2, 2), (S[0], S[1], np.ascontiguousarray(S[2].T)))]
    for shape in ((2, 3, 4), (3, 3, 3), (4, 4, 4)):
        out.append((shape, standard_scheme(*shape)))
    return out


def test_flip_variants_match_oracle(gpu, oracle):
    """Random flips (Sec. 3.5.3) generated on the device equal the oracle's
    variant for variant, over three iterations; every variant satisfies the
    Brent equations."""
    from cse_helpers import brent_ok
    cse, ctx, torch = gpu
    for (n, m, p), (U, V, W) in _flip_schemes():
        for it in range(3):
            got = cse.cse_flip_variants(ctx, U, V, W, n, m, p, n_variants=8, max_flips=40, seed=11, iteration=it)
            for v, (gU, gV, gW, nf) in enumerate(got):
                rU, rV, rW, rn = oracle.flip_variant(U, V, W, n, m, p, seed=11, variant=v, iteration=it,
                                                     max_flips=40)
                assert nf == rn, ((n, m, p), it, v)
                assert np.array_equal(gU, rU) and np.array_equal(gV, rV) and np.array_equal(gW, rW), \
                    ((n, m, p), it, v)
                assert brent_ok(gU, gV, gW, n, m, p)


def test_flip_mode_against_oracle(gpu, oracle):
    """The flip mode: every iteration regenerates the variants and reduces
    each with its own pool; the best total per iteration, the chosen variant
    and its component costs equal what the oracle computes from its own
    variants and pool runs, and the best programs re-expand exactly on the
    chosen variant (which is a valid scheme)."""
    from cse_helpers import brent_ok, standard_scheme
    cse, ctx, torch = gpu
    n, m, p = 3, 3, 3
    U, V, W = standard_scheme(n, m, p)
    kw = dict(seed=21, n_proc=24, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True)
    M, F, its = 6, 12, 3
    run, n_it = cse.cse_run_flips(ctx, U, V, W, n, m, p, cse.cse_run_cfg(**kw), n_variants=M, max_flips=F,
                                  patience=100, max_iterations=its, stream=torch.cuda.current_stream())
    assert n_it == its
    best = cse.cse_flip_best(ctx, run, (n, m, p, 27))
    want_tot, want = [], None
    for it in range(its):
        for v in range(M):
            vU, vV, vW, _ = oracle.flip_variant(U, V, W, n, m, p, seed=21, variant=v, iteration=it, max_flips=F)
            cfg = oracle.make_cfg(**dict(kw, seed=21 + v, iteration=it))
            costs = [int(oracle.run_pool(A, cfg, comp=c, n_threads=THREADS)["cost"].min())
                     for c, A in enumerate((vU, vV, np.ascontiguousarray(vW.T)))]
            if want is None or sum(costs) < want[0]:
                want = (sum(costs), v, it, costs, (vU, vV, vW))
        want_tot.append(want[0])
    assert best["totals"] == want_tot
    assert (best["variant"], best["iteration"], best["cost"]) == (want[1], want[2], want[3])
    assert np.array_equal(best["U"], want[4][0]) and np.array_equal(best["V"], want[4][1])
    assert np.array_equal(best["W"], want[4][2])
    assert brent_ok(best["U"], best["V"], best["W"], n, m, p)
    for c, A in enumerate((best["U"], best["V"], np.ascontiguousarray(best["W"].T))):
        check_program(A, cse.cse_flip_program(ctx, run, c), best["cost"][c])
    cse.cse_flip_release(ctx, run)
