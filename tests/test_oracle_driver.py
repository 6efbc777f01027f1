"""Pins of the oracle's outer-iteration driver (Sec. 3.5.1, 3.5.2 and the
convergence rule of Sec. 4) against what the paper fixes: the stopping
rule, exact best programs, the share of restarted processes and the bounds
of their copied prefixes, and the composition of iterations from pool runs
that the other pins check."""
import numpy as np

from cse_helpers import check_program
from paper_2512_13365_amd.workloads import random_system

KW = dict(seed=3, n_proc=96, weights={"gi": 8, "ga": 4, "gr": 2, "wr": 1, "mix": 1}, proc0_greedy=True)


def _systems():
    return [random_system(51, 30, 12, 0.3, 1, 8), random_system(52, 30, 12, 0.3, 1, 8),
            random_system(53, 12, 30, 0.3, 1, 8)]


def test_driver_convergence_rule(oracle):
    """Sec. 4: a run ends once the best total has stayed the same for
    `patience` consecutive iterations; the best total never rises.  Few
    processes on 49 x 16 systems keep improving after the first iteration."""
    S = [random_system(61 + i, 49, 16, 0.3, 1, 8) for i in range(3)]
    patience, cap = 3, 40
    # seed 9: a run whose best total still falls at iteration 6
    d = oracle.run_driver(S, oracle.make_cfg(**dict(KW, n_proc=16, seed=9)), patience=patience, max_iterations=cap)
    t = d["totals"]
    assert len(t) == d["iterations"] < cap
    assert all(b <= a for a, b in zip(t, t[1:]))
    last_drop = max(i for i in range(1, len(t)) if t[i] < t[i - 1])
    assert last_drop >= 2
    assert d["iterations"] == last_drop + patience + 1
    assert sum(b["cost"] for b in d["best"]) == t[-1]
    assert max(b["iteration"] for b in d["best"]) == last_drop


def test_driver_best_programs_exact(oracle):
    """Each component's best program is a complete valid reduction of its
    input with the reported cost (Sec. 3.2.1), found at the reported
    iteration, and no unit of the last iteration is better."""
    S = _systems()
    d = oracle.run_driver(S, oracle.make_cfg(**KW), patience=2, max_iterations=6)
    for A, b, r in zip(S, d["best"], d["last"]):
        check_program(A, b["prog"], b["cost"])
        assert 0 <= b["iteration"] < d["iterations"]
        assert b["cost"] <= int(r["cost"].min())


def test_driver_restart_share_and_prefix(oracle):
    """Sec. 3.5.2: before the second iteration about 40% of the processes
    copy the first k substitutions of the best program so far, k between 1
    and 3/4 of its length; the others start from the input."""
    S = _systems()
    cfg = dict(KW, n_proc=400)
    first = oracle.run_driver(S, oracle.make_cfg(**cfg), max_iterations=1)
    two = oracle.run_driver(S, oracle.make_cfg(**cfg), patience=5, max_iterations=2)
    assert first["iterations"] == 1 and two["iterations"] == 2
    for c in range(3):
        bp = first["best"][c]["prog"]
        L = len(bp)
        assert L > 0
        r = two["last"][c]
        k0 = r["k0"]
        # Binomial(400, 0.4): standard deviation 0.0245.
        assert abs(float(np.mean(k0 > 0)) - 0.4) < 0.1
        assert k0.max() <= max(1, (3 * L) // 4)
        for u in np.flatnonzero(k0 > 0):
            assert np.array_equal(r["prog"][u, :k0[u]], bp[:k0[u]])
        assert np.array_equal(r["epoch"], first["last"][c]["epoch"] + 1)
        assert np.array_equal(r["executed"] - first["last"][c]["executed"] + k0,
                              r["steps"])


def test_driver_all_restart_from_prefix(oracle):
    """reinit_pm = 1000: every process of every later iteration starts from
    a prefix of the best program."""
    S = _systems()
    d = oracle.run_driver(S, oracle.make_cfg(**KW), reinit_pm=1000, patience=9, max_iterations=3)
    for c in range(3):
        assert np.all(d["last"][c]["k0"] >= 1)


def test_driver_iterations_compose_pool_runs(oracle):
    """With no restarts and no sharing, iteration i is the pool run with
    cfg.iteration = i from the input at epoch i: its draws are keyed by the
    iteration (strategy, alpha, beta) and the epoch (steps, coins) only."""
    A = _systems()[0]
    d = oracle.run_driver([A], oracle.make_cfg(**KW), reinit_pm=0, patience=100, max_iterations=3)
    n = KW["n_proc"]
    cap = d["last"][0]["prog"].shape[1]
    r = oracle.run_pool(A, oracle.make_cfg(iteration=2, **KW), init_prog=np.zeros((n, cap, 3), np.int32),
                        init_len=np.zeros(n, np.int32), init_epoch=np.full(n, 2, np.int32))
    assert np.array_equal(r["prog"], d["last"][0]["prog"])
    assert np.array_equal(r["cost"], d["last"][0]["cost"])
    assert not np.array_equal(r["strat"], oracle.run_pool(A, oracle.make_cfg(**KW))["strat"])
