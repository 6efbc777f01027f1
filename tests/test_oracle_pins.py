"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the
paper's worked example (Sec. 3.2.2), its closed forms (Sec. 3.2.1), the
published Philox known-answer vectors, an independent dictionary count and
symbolic replay, exhaustive search on tiny systems, and special cases whose
answer is known in closed form.
"""
import numpy as np
import pytest

from cse_helpers import (brute_force_optimum, check_program, is_terminal, naive_count,
                         pair_counts, read_golden, replay)
from paper_2512_13365_amd.workloads import random_system

ALL = ("g", "ga", "wr", "gr", "gi", "mix", "gp")


def _golden_matrix(rows):
    return np.array([[int(x) for x in r] for r in rows], np.int8)


def test_philox_known_answers(oracle):
    """Philox4x32-10 against the generator authors' published vectors."""
    with open(__import__("cse_helpers").GOLDEN + "/philox_kat.txt") as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(lines) == 3
    for ln in lines:
        v = [int(x, 16) for x in ln]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_worked_example_substitutions(oracle):
    """Sec. 3.2.2: x5 = x2 + x4 and x6 = x1 - x3 give the printed forms.
    Pair (2, +4) rewrites -x2 - x4 in e2 as -x5 and leaves -x2 + x4 in e3."""
    g = read_golden("worked_example.txt")
    A = _golden_matrix(g["input"])
    assert oracle.naive(A) == g["naive"] == 8
    k = A.shape[1]
    for a, b, s in g["subst"]:
        k += 1
        A, c = oracle.substitute(A, a, b, s, k)
        assert c >= 2
    final = _golden_matrix(g["final"])
    assert np.array_equal(A, final)
    assert oracle.naive(A) == g["final_naive"] == 4
    assert len(g["subst"]) + oracle.naive(A) == g["cost"] == 6


def test_worked_example_candidates(oracle):
    """Canonical pairs of the worked example, counted independently."""
    g = read_golden("worked_example.txt")
    A = _golden_matrix(g["input"])
    ref = sorted((a, b, s, c) for (a, b, s), c in pair_counts(A).items() if c >= 2)
    ref.sort(key=lambda t: (t[0], t[1], t[2] < 0))
    assert oracle.analyse(A) == ref


@pytest.mark.parametrize("strategy", ALL)
def test_worked_example_every_strategy_reaches_6(oracle, strategy):
    """Every maximal substitution sequence of the example ends at Cost 6 with
    two fresh variables (exhaustive search below confirms 6 is optimal)."""
    g = read_golden("worked_example.txt")
    A = _golden_matrix(g["input"])
    assert brute_force_optimum(A) == 6
    for seed in range(5):
        cfg = oracle.make_cfg(seed=seed, n_proc=32, weights={strategy: 1})
        r = oracle.run_pool(A, cfg)
        assert np.all(r["cost"] == 6)
        assert np.all(r["steps"] == 2)
        for i in range(32):
            check_program(A, r["prog"][i, :2], 6)


def test_naive_closed_form(oracle):
    for seed in range(20):
        A = random_system(seed, 9, 7, 0.5)
        assert oracle.naive(A) == naive_count(A)


def test_analysis_matches_dictionary_count(oracle):
    for seed in range(30):
        A = random_system(100 + seed, 12, 9, 0.45)
        ref = [(a, b, s, c) for (a, b, s), c in pair_counts(A).items() if c >= 2]
        ref.sort(key=lambda t: (t[0], t[1], t[2] < 0))
        assert oracle.analyse(A) == ref


def test_substitution_against_replay(oracle):
    """Oracle substitution equals the independent replay on random moves."""
    rng = np.random.default_rng(7)
    for seed in range(20):
        A = random_system(200 + seed, 10, 6, 0.5)
        cands = oracle.analyse(A)
        if not cands:
            continue
        a, b, s, c = cands[rng.integers(len(cands))]
        B, cc = oracle.substitute(A, a, b, s, A.shape[1] + 1)
        R, cs = replay(A, [(a, b, s)])
        assert cc == c == cs[0]
        assert np.array_equal(B, R)


@pytest.mark.parametrize("strategy", ALL)
def test_programs_valid_and_terminal(oracle, strategy):
    """Cost bookkeeping, re-expansion and the stopping rule on random systems."""
    for seed in range(6):
        A = random_system(300 + seed, 14, 8, 0.4)
        cfg = oracle.make_cfg(seed=seed, n_proc=8, weights={strategy: 1})
        r = oracle.run_pool(A, cfg)
        for i in range(8):
            n = int(r["steps"][i])
            F = check_program(A, r["prog"][i, :n], int(r["cost"][i]))
            assert is_terminal(F)
            assert r["executed"][i] == n


@pytest.mark.parametrize("strategy", ALL)
def test_brute_force_lower_bound(oracle, strategy):
    """Exhaustive optimum over the same move set bounds every heuristic."""
    for seed in range(8):
        A = random_system(400 + seed, 7, 4, 0.55)
        opt = brute_force_optimum(A)
        cfg = oracle.make_cfg(seed=seed, n_proc=16, weights={strategy: 1})
        r = oracle.run_pool(A, cfg)
        assert np.all(r["cost"] >= opt)
        assert r["cost"].min() >= opt


def test_brute_force_reached_on_tiny(oracle):
    """With enough random processes the optimum of 7x4 systems is found."""
    hits = 0
    for seed in range(8):
        A = random_system(500 + seed, 7, 4, 0.55)
        opt = brute_force_optimum(A)
        cfg = oracle.make_cfg(seed=seed, n_proc=64, weights={"wr": 1, "gi": 1})
        r = oracle.run_pool(A, cfg)
        hits += int(r["cost"].min() == opt)
    assert hits >= 6


def test_disjoint_rows_take_no_step(oracle):
    A = np.zeros((4, 12), np.int8)
    for i in range(4):
        A[i, 3 * i:3 * i + 3] = [1, -1, 1]
    for s in ALL:
        r = oracle.run_pool(A, oracle.make_cfg(n_proc=4, weights={s: 1}))
        assert np.all(r["steps"] == 0) and np.all(r["cost"] == naive_count(A))


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_identical_and_negated_rows(oracle, k):
    """n_e equal (or negated) rows of k terms cost exactly k - 1."""
    rng = np.random.default_rng(k)
    row = (rng.integers(0, 2, k) * 2 - 1).astype(np.int8)
    A = np.stack([row, -row, row, row, -row])
    for s in ALL:
        r = oracle.run_pool(A, oracle.make_cfg(seed=k, n_proc=8, weights={s: 1}))
        assert np.all(r["cost"] == k - 1)
        assert np.all(r["steps"] == k - 1)


def test_strassen_has_no_repeated_pair(oracle):
    """Strassen's scheme needs 18 additions (Sec. 2.2); no signed pair
    repeats in U, V or W^T, so CSE takes no step."""
    g = read_golden("strassen_2x2x2.txt")
    total = 0
    for name in ("U", "V", "Wt"):
        A = _golden_matrix(g[name])
        for s in ALL:
            r = oracle.run_pool(A, oracle.make_cfg(n_proc=4, weights={s: 1}))
            assert np.all(r["steps"] == 0)
        total += int(r["cost"][0])
    assert total == g["additions"] == 18


def _random_cands(rng, m, n_v, disjoint=False):
    out = set()
    used = set()
    while len(out) < m:
        a, b = sorted(rng.choice(np.arange(1, n_v + 1), 2, replace=False))
        if disjoint and (a in used or b in used):
            continue
        s = int(rng.choice([1, -1]))
        if (a, b, s) in out:
            continue
        out.add((int(a), int(b), s))
        used.update((a, b))
    cands = [(a, b, s, int(rng.integers(2, 9))) for a, b, s in out]
    cands.sort(key=lambda t: (t[0], t[1], t[2] < 0))
    return cands


def test_gi_alpha_zero_is_greedy(oracle):
    """With alpha = 0 the score is c_p - 1 alone, so gi picks what g picks."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        cands = _random_cands(rng, int(rng.integers(1, 40)), 12)
        i, _, _ = oracle.select_gi(cands, 0, 50000, seed=int(rng.integers(1 << 30)))
        assert i == oracle.select_g(cands)


def test_gi_disjoint_candidates_is_greedy(oracle):
    """Pairwise disjoint candidates: sum I = T - (c_p - 1) decreases slower
    than the immediate gain grows (alpha < 1), so gi equals g."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        cands = _random_cands(rng, int(rng.integers(1, 8)), 30, disjoint=True)
        i, n_int, _ = oracle.select_gi(cands, int(rng.integers(0, 32768)), 40000,
                                       seed=int(rng.integers(1 << 30)))
        assert n_int == 0
        assert i == oracle.select_g(cands)


def test_gi_score_against_float_formula(oracle):
    """The fixed-point score ranks as the real-valued H of Sec. 3.4.2 when
    evaluated with the same coins (ties aside)."""
    rng = np.random.default_rng(13)
    checked = 0
    for trial in range(100):
        cands = _random_cands(rng, int(rng.integers(2, 25)), 10)
        aq, bq = int(rng.integers(0, 32768)), int(32768 + rng.integers(0, 32768))
        seed, proc, step = int(rng.integers(1 << 30)), int(rng.integers(1000)), int(rng.integers(100))
        dw = oracle.domain_word(3, 1, 2, step)
        H = []
        for p, (pa, pb, ps, pc) in enumerate(cands):
            # coins: the candidates holding pa (twin included), then those
            # holding pb but not pa, each list in canonical order, numbered
            # i = 0, 1, ... across both; coin i is bit i mod 128 of the Philox
            # block with counter word 3 = i div 128
            n_a = sum(1 for q, (qa, qb, _, _) in enumerate(cands) if q != p and pa in (qa, qb))
            idx = {pa: 0, pb: n_a}
            tot = 0.0
            for q, (qa, qb, qs, qc) in enumerate(cands):
                if q == p:
                    continue
                shared = pa if pa in (qa, qb) else pb if pb in (qa, qb) else None
                if shared is None:
                    tot += qc - 1
                    continue
                i = idx[shared]
                idx[shared] += 1
                key = (pa << 16) | (pb << 1) | (ps < 0)
                c3 = i // 128
                blk = oracle.philox4x32_10((proc, dw, key, c3), (seed & 0xFFFFFFFF, seed >> 32))
                coin = (blk[(i % 128) // 32] >> (i % 32)) & 1
                tot += (bq / 65536.0) * (qc - 1) if coin else 0.0
            H.append((pc - 1) + (aq / 65536.0) * tot)
        i, _, _ = oracle.select_gi(cands, aq, bq, seed=seed, proc=proc, comp=1, epoch=2, step=step)
        order = sorted(H, reverse=True)
        if len(order) > 1 and order[0] - order[1] < 1e-9:
            continue
        assert i == int(np.argmax(H))
        checked += 1
    assert checked > 50


def _chi2_uniform(counts):
    counts = np.asarray(counts, float)
    e = counts.sum() / len(counts)
    return float(((counts - e) ** 2 / e).sum())


def test_ga_uniform_over_ties(oracle):
    cands = [(1, 2, 1, 5), (1, 3, -1, 5), (2, 3, 1, 2), (2, 4, 1, 5), (3, 4, -1, 5)]
    rng = np.random.default_rng(5)
    hist = np.zeros(len(cands), int)
    for _ in range(8000):
        hist[oracle.select_ga(cands, int(rng.integers(0, 1 << 32)))] += 1
    assert hist[2] == 0
    assert _chi2_uniform(hist[[0, 1, 3, 4]]) < 16.3   # 3 dof, p = 0.001


def test_wr_proportional_to_profit(oracle):
    cands = [(1, 2, 1, 2), (1, 3, -1, 3), (2, 3, 1, 5), (2, 4, 1, 9)]
    w = np.array([c - 1 for *_, c in cands], float)
    rng = np.random.default_rng(6)
    n = 20000
    hist = np.zeros(len(cands), int)
    for _ in range(n):
        hist[oracle.select_wr(cands, int(rng.integers(0, 1 << 32)))] += 1
    e = n * w / w.sum()
    assert float(((hist - e) ** 2 / e).sum()) < 16.3


def test_coin_rate_and_parameter_ranges(oracle):
    """Coins are fair; alpha in [0, 0.5), beta in [0.5, 1) (Sec. 3.4.2);
    strategies follow their weights (Sec. 3.5.1)."""
    ones = tot = 0
    for proc in range(300):
        blk = oracle.philox4x32_10((proc, oracle.domain_word(3, 0, 0, 7), 12345, 0), (9, 0))
        ones += sum(bin(x).count("1") for x in blk)
        tot += 128
    assert abs(ones / tot - 0.5) < 0.01
    cfg = oracle.make_cfg(seed=3, weights={"gi": 8, "ga": 4, "gr": 2, "wr": 1})
    hist = {}
    for proc in range(6000):
        s, a, b = oracle.proc_init(cfg, proc)
        assert 0 <= a < 32768 and 32768 <= b < 65536
        hist[s] = hist.get(s, 0) + 1
    obs = np.array([hist.get(i, 0) for i in (4, 1, 3, 2)], float)
    e = 6000 * np.array([8, 4, 2, 1]) / 15
    assert float(((obs - e) ** 2 / e).sum()) < 16.3
    cfg0 = oracle.make_cfg(seed=3, weights={"gi": 1}, proc0_greedy=True)
    assert oracle.proc_init(cfg0, 0)[0] == 0 and oracle.proc_init(cfg0, 1)[0] == 4


def test_mix_and_gr_degenerate_weights(oracle):
    """mix with all weight on gi is gi; gr with p = 1 is ga and p = 0 is wr."""
    A = random_system(42, 20, 10, 0.4)
    base = dict(seed=4, n_proc=24)
    gi = oracle.run_pool(A, oracle.make_cfg(weights={"gi": 1}, **base))
    mix = oracle.run_pool(A, oracle.make_cfg(weights={"mix": 1}, mix_weights=(1, 0, 0, 0), **base))
    assert np.array_equal(gi["prog"], mix["prog"])
    ga = oracle.run_pool(A, oracle.make_cfg(weights={"ga": 1}, **base))
    gr1 = oracle.run_pool(A, oracle.make_cfg(weights={"gr": 1}, gr_p_q16=65536, **base))
    assert np.array_equal(ga["prog"], gr1["prog"])
    wr = oracle.run_pool(A, oracle.make_cfg(weights={"wr": 1}, **base))
    gr0 = oracle.run_pool(A, oracle.make_cfg(weights={"gr": 1}, gr_p_q16=0, **base))
    assert np.array_equal(wr["prog"], gr0["prog"])


@pytest.mark.parametrize("name,mixw", [("gi", (1, 0, 0, 0)), ("ga", (0, 1, 0, 0)),
                                       ("gr", (0, 0, 1, 0)), ("wr", (0, 0, 0, 1))])
def test_mix_single_weight_is_that_strategy(oracle, name, mixw):
    """mix (Sec. 3.4.3) draws one of gi, ga, gr, wr per step by the weights
    8, 4, 2, 1; with all weight on one of them every step is that strategy,
    so the whole pool equals a pool of that strategy.  The four strategies
    give different pools here, so a permuted map fails one of the cases."""
    A = random_system(44, 24, 12, 0.4)
    base = dict(seed=5, n_proc=48)
    pools = {s: oracle.run_pool(A, oracle.make_cfg(weights={s: 1}, **base))["prog"]
             for s in ("gi", "ga", "gr", "wr")}
    names = list(pools)
    for i in range(4):
        for j in range(i + 1, 4):
            assert not np.array_equal(pools[names[i]], pools[names[j]]), (names[i], names[j])
    mix = oracle.run_pool(A, oracle.make_cfg(weights={"mix": 1}, mix_weights=mixw, **base))
    assert np.array_equal(mix["prog"], pools[name])


def test_gr_exploit_rate(oracle):
    """Greedy-Random (Sec. 3.4.1) takes the ga branch with probability p
    (0.75 here) and wr otherwise.  On a system whose candidates are one pair
    of count 3 and K disjoint pairs of count 2, ga always takes the count-3
    pair and wr takes it with probability 2 / (2 + K), so the first pick of
    a gr process is that pair with probability p + (1 - p) 2 / (2 + K).
    Estimated over 6000 processes and compared with a 4.5-sigma binomial
    band; p = 0.5 or a reversed comparison lie far outside it."""
    K = 30
    rows = []
    n_x = 2 + 2 * K
    for _ in range(3):
        r = np.zeros(n_x, np.int8); r[0] = 1; r[1] = 1; rows.append(r)
    for i in range(K):
        for _ in range(2):
            r = np.zeros(n_x, np.int8); r[2 + 2 * i] = 1; r[3 + 2 * i] = -1; rows.append(r)
    A = np.array(rows, np.int8)
    n = 6000
    r = oracle.run_pool(A, oracle.make_cfg(seed=17, n_proc=n, weights={"gr": 1}, step_cap=1), n_threads=8)
    assert np.all(r["steps"] == 1)
    hit = int(np.sum((r["prog"][:, 0, 0] == 1) & (r["prog"][:, 0, 1] == 2)))
    q = 2.0 / (2 + K)
    for p, inside in ((0.75, True), (0.5, False), (0.25, False)):
        f = p + (1 - p) * q
        z = abs(hit - n * f) / np.sqrt(n * f * (1 - f))
        assert (z < 4.5) == inside, (p, hit, z)


def test_gi_work_tally_independent_count(oracle):
    """The gi work tally (n_int = sum over p of the candidates intersecting p;
    n_blk = the coin blocks, ceil((|A_p| + |B_p|) / 128) per p with A_p the
    candidates holding p's first variable and B_p those holding only its
    second, whose coins follow A_p's) against a count written here from the intersection rule
    (shared variable index, p itself excluded), on candidate sets large
    enough that some lists exceed 128."""
    rng = np.random.default_rng(15)
    big = 0
    for trial in range(40):
        n_v = int(rng.integers(4, 40))
        m = int(rng.integers(1, min(400, n_v * (n_v - 1))))
        cands = _random_cands(rng, m, n_v)
        if trial % 4 == 0:
            # hub variables: every pair (h, x, +-) of two hubs h, so the
            # candidates holding a hub intersect well over 128 others
            n_v = int(rng.integers(70, 90))
            hub = {(h, x, s) for h in (1, 2) for x in range(h + 1, n_v + 1) for s in (1, -1)}
            rest = {(a, b, s) for a, b, s, _ in _random_cands(rng, 150, n_v)}
            cands = [(a, b, s, int(rng.integers(2, 9))) for a, b, s in hub | rest]
            cands.sort(key=lambda t: (t[0], t[1], t[2] < 0))
        n_int = n_blk = 0
        for p, (pa, pb, _, _) in enumerate(cands):
            ka = sum(1 for q, (qa, qb, _, _) in enumerate(cands) if q != p and pa in (qa, qb))
            kb = sum(1 for q, (qa, qb, _, _) in enumerate(cands) if q != p and pa not in (qa, qb) and pb in (qa, qb))
            n_int += ka + kb
            n_blk += -(-(ka + kb) // 128)
            big += max(ka, kb) > 128
        _, got_int, got_blk = oracle.select_gi(cands, int(rng.integers(0, 32768)), 40000, seed=trial)
        assert (got_int, got_blk) == (n_int, n_blk)
    assert big > 0


def test_epochs_never_reuse_draws(oracle):
    """A unit's epoch counts its restarts and may pass 1023; its step and
    coin draws must then still be new (no random key is reused, so a unit
    restarted 1024 times does not repeat the choices of its first epochs).
    Units started at epoch e, e + 1024 and e + 2048 from the input choose
    differently; epochs below 1024 keep the draws they always had."""
    A = random_system(45, 30, 12, 0.4)
    n = 64
    cfg = oracle.make_cfg(seed=11, n_proc=n, weights={"gi": 2, "ga": 1, "wr": 1, "mix": 1})
    cap = max(1, oracle.bounds(A)[0])
    zero = np.zeros((n, cap, 3), np.int32)
    runs = {}
    for e in (3, 3 + 1024, 3 + 2048):
        runs[e] = oracle.run_pool(A, cfg, init_prog=zero, init_len=np.zeros(n, np.int32),
                                  init_epoch=np.full(n, e, np.int32))
    for e1, e2 in ((3, 1027), (3, 2051), (1027, 2051)):
        differ = sum(not np.array_equal(runs[e1]["prog"][u], runs[e2]["prog"][u]) for u in range(n))
        assert differ > n // 2, (e1, e2, differ)
    # Epoch 0 from an explicit start equals the plain pool run.
    plain = oracle.run_pool(A, cfg)
    again = oracle.run_pool(A, cfg, init_prog=zero, init_len=np.zeros(n, np.int32),
                            init_epoch=np.zeros(n, np.int32))
    assert np.array_equal(plain["prog"], again["prog"])


def test_step_cap(oracle):
    A = random_system(43, 30, 10, 0.5)
    r = oracle.run_pool(A, oracle.make_cfg(n_proc=8, weights={"gi": 1, "wr": 1}, step_cap=3))
    assert np.all(r["steps"] <= 3)
    for i in range(8):
        check_program(A, r["prog"][i, :r["steps"][i]], int(r["cost"][i]))


def test_subset_of_processes_equals_pool(oracle):
    """Without sharing a unit depends only on its own process index."""
    A = random_system(44, 25, 10, 0.35)
    cfg = oracle.make_cfg(seed=9, n_proc=40, weights={"gi": 1, "ga": 1, "wr": 1, "mix": 1})
    full = oracle.run_pool(A, cfg)
    sub = [3, 17, 39, 0]
    part = oracle.run_pool(A, cfg, procs=sub)
    for j, p in enumerate(sub):
        assert np.array_equal(part["prog"][j], full["prog"][p])
        assert part["cost"][j] == full["cost"][p]
        assert part["ops"][j] == full["ops"][p]


def test_sharing_rounds(oracle):
    """Sharing (Sec. 3.5.2): programs stay valid; targets continue from a
    copied prefix; a unit continued from its last prefix without sharing
    reproduces its program; no sharing when the target share is zero."""
    A = random_system(45, 40, 14, 0.3, 1, 8)
    kw = dict(seed=2, n_proc=64, weights={"gi": 8, "ga": 4, "gr": 2, "wr": 1, "mix": 1},
              proc0_greedy=True)
    plain = oracle.run_pool(A, oracle.make_cfg(**kw))
    zero = oracle.run_pool(A, oracle.make_cfg(share_every=4, share_src_pm=100, share_dst_pm=0,
                                              share_max_rounds=64, **kw))
    assert np.array_equal(plain["prog"], zero["prog"])
    r = oracle.run_pool(A, oracle.make_cfg(share_every=4, share_src_pm=50, share_dst_pm=300,
                                           share_max_rounds=64, **kw))
    assert r["epoch"].max() > 0
    for i in range(64):
        check_program(A, r["prog"][i, :r["steps"][i]], int(r["cost"][i]))
    idx = np.flatnonzero(r["epoch"] > 0)
    init = np.zeros_like(r["prog"][idx])
    lens = r["k0"][idx]
    for j, i in enumerate(idx):
        init[j, :lens[j]] = r["prog"][i, :lens[j]]
    cont = oracle.run_pool(A, oracle.make_cfg(**kw), procs=idx, init_prog=init, init_len=lens,
                           init_epoch=r["epoch"][idx])
    assert np.array_equal(cont["prog"], r["prog"][idx])
    assert np.array_equal(cont["cost"], r["cost"][idx])


def _gp_reference(A, alpha_q):
    """Independent Greedy-Potential pick: symbolic replay of each trial
    substitution and a dictionary count of the fresh variable's pairs."""
    cands = sorted(((a, b, s, c) for (a, b, s), c in pair_counts(A).items() if c >= 2),
                   key=lambda t: (t[0], t[1], t[2] < 0))
    k = A.shape[1] + 1
    best, best_h = -1, None
    for i, (a, b, s, c) in enumerate(cands):
        F, _ = replay(A, [(a, b, s)])
        n_new = sum(1 for (x, y, _), cnt in pair_counts(F).items() if cnt >= 2 and k in (x, y))
        h = ((c - 1) << 16) + alpha_q * n_new
        if best_h is None or h > best_h:
            best, best_h = i, h
    return best


def test_substitution_only_lowers_old_pair_counts():
    """The premise of the Greedy-Potential reading: after any substitution
    every pair of old variables occurs at most as often as before, so the new
    substitution possibilities are exactly the fresh variable's pairs that
    occur at least twice (brute force over every candidate)."""
    rng = np.random.default_rng(23)
    checked = 0
    for case in range(10):
        rows, cols = int(rng.integers(5, 20)), int(rng.integers(4, 10))
        A = random_system(int(rng.integers(1 << 30)), rows, cols, float(rng.uniform(0.3, 0.6)))
        before = pair_counts(A)
        k = A.shape[1] + 1
        for (a, b, sgn), c in before.items():
            if c < 2:
                continue
            after = pair_counts(replay(A, [(a, b, sgn)])[0])
            for key, c_new in after.items():
                if k in key[:2]:
                    continue
                assert c_new <= before.get(key, 0), (case, (a, b, sgn), key)
            checked += 1
    assert checked > 50


def test_gp_matches_independent_potential(oracle):
    """Greedy-Potential (Sec. 2, 3.4; the potential read as the number of the
    fresh variable's pairs that occur at least twice after the trial
    substitution): the oracle's pick equals one computed from an independent
    replay and pair count, for several alphas, and alpha = 0 is greedy."""
    rng = np.random.default_rng(17)
    for case in range(12):
        rows, cols = int(rng.integers(6, 30)), int(rng.integers(4, 12))
        A = random_system(int(rng.integers(1 << 30)), rows, cols, float(rng.uniform(0.25, 0.6)))
        if not oracle.analyse(A):
            continue
        m = sum(1 for c in pair_counts(A).values() if c >= 2)
        live = int(np.count_nonzero(np.abs(A).sum(axis=0)))
        for alpha_q in (0, 1, 4096, 32767):
            got, n_cols = oracle.select_gp(A, alpha_q)
            assert got == _gp_reference(A, alpha_q), (case, alpha_q)
            # The work tally counts every candidate against every live
            # column other than its own two.
            assert n_cols == m * max(0, live - 2), (case, n_cols)
        assert oracle.select_gp(A, 0)[0] == oracle.select_g(oracle.analyse(A))



def _strassen():
    g = read_golden("strassen_2x2x2.txt")
    U, V, Wt = (_golden_matrix(g[k]) for k in ("U", "V", "Wt"))
    return U, V, np.ascontiguousarray(Wt.T)


@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 3, 4), (3, 3, 3), "strassen"])
def test_flip_variants_stay_valid_schemes(oracle, shape):
    """Random flips (Sec. 3.5.3) keep a scheme a valid matrix multiplication
    algorithm of the same rank: every variant satisfies the Brent equations
    (checked by the tensor identity in the test helpers), its coefficients
    stay ternary and no product loses a factor; variant 0 is the input and
    the others differ from it; the same draws give the same variant."""
    from cse_helpers import brent_ok, standard_scheme
    if shape == "strassen":
        n = m = p = 2
        U, V, W = _strassen()
    else:
        n, m, p = shape
        U, V, W = standard_scheme(n, m, p)
    assert brent_ok(U, V, W, n, m, p)
    changed = 0
    for it in range(3):
        for v in range(8):
            U2, V2, W2, done = oracle.flip_variant(U, V, W, n, m, p, seed=3, variant=v, iteration=it, max_flips=40)
            assert brent_ok(U2, V2, W2, n, m, p), (v, it)
            for M in (U2, V2, W2):
                assert M.min() >= -1 and M.max() <= 1 and (np.abs(M).sum(axis=1) > 0).all()
            if v == 0 or shape == "strassen":
                assert done == 0 and np.array_equal(U2, U) and np.array_equal(V2, V) and np.array_equal(W2, W)
            else:
                assert 1 <= done <= 40
                changed += not (np.array_equal(U2, U) and np.array_equal(V2, V) and np.array_equal(W2, W))
            again = oracle.flip_variant(U, V, W, n, m, p, seed=3, variant=v, iteration=it, max_flips=40)
            assert all(np.array_equal(a, b) for a, b in zip(again[:3], (U2, V2, W2)))
    if shape == "strassen":
        # No two of Strassen's products share a factor up to sign, so no
        # flip applies and every variant is the scheme itself.
        for M in (U, V, W):
            for i in range(7):
                for j in range(7):
                    assert i == j or not (np.array_equal(M[i], M[j]) or np.array_equal(M[i], -M[j]))
    else:
        assert changed >= 20


def test_flip_breaks_when_the_identity_is_broken(oracle):
    """The Brent check used above rejects a scheme with one coefficient
    changed, and one where a flip updates only one of the two products."""
    from cse_helpers import brent_ok, standard_scheme
    U, V, W = standard_scheme(2, 2, 2)
    U2, V2, W2, done = oracle.flip_variant(U, V, W, 2, 2, 2, seed=1, variant=1, iteration=0, max_flips=5)
    assert done >= 1 and brent_ok(U2, V2, W2, 2, 2, 2)
    bad = V2.copy()
    bad[0, 0] = 1 - bad[0, 0] if bad[0, 0] != 1 else 0
    assert not brent_ok(U2, bad, W2, 2, 2, 2)
    half = V.copy()
    half[0] = half[0] + half[4]  # products 0 and 4 share U; the matching W update is left out
    assert not brent_ok(U, half, W, 2, 2, 2)
