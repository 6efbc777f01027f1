"""Seeded synthetic workloads: ternary linear-form systems shaped like the
components of fast matrix-multiplication schemes (Sec. 3.1, 3.2).

This module only draws inputs; it holds none of the method's arithmetic, so
both the HIP path and the CPU oracle can be fed from it.  The paper evaluates
149 real schemes from an external database that is not available here; these
systems stand in for them with the shapes of (m, n, p : r) schemes and
random supports.

A system is an int8 matrix in {-1, 0, 1}, rows = linear forms, columns =
variables.  A scheme has three: U (r x nm), V (r x mp) and W^T (np x r).

Row recipe: each entry is nonzero with probability p; a row with fewer than
`lo` nonzeros gets that many more at uniformly chosen zero positions, a row
with more than `hi` keeps a uniformly chosen subset of `hi`; signs are fair
coins.  The generator is numpy's default_rng seeded with the configuration
number, drawn in a fixed order, so every input is reproducible.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field

import numpy as np

STRATEGIES = ("g", "ga", "wr", "gr", "gi", "mix", "gp")

# Default strategy weights of Sec. 3.5.1 scaled by 100 (gi 8, ga 4, gr 2,
# wr 1, mix 0.1, gp 0.01).
PAPER_WEIGHTS = {"gi": 800, "ga": 400, "gr": 200, "wr": 100, "mix": 10, "gp": 1}


def ternary_rows(rng: np.random.Generator, rows: int, cols: int, p: float,
                 lo: int = 1, hi: int | None = None) -> np.ndarray:
    hi = cols if hi is None else min(hi, cols)
    lo = min(lo, cols)
    A = np.zeros((rows, cols), np.int8)
    for i in range(rows):
        mask = rng.random(cols) < p
        nz = np.flatnonzero(mask)
        if nz.size < lo:
            zeros = np.flatnonzero(~mask)
            extra = rng.choice(zeros, size=lo - nz.size, replace=False)
            nz = np.sort(np.concatenate([nz, extra]))
        elif nz.size > hi:
            nz = np.sort(rng.choice(nz, size=hi, replace=False))
        signs = rng.integers(0, 2, size=nz.size) * 2 - 1
        A[i, nz] = signs.astype(np.int8)
    return A


def scheme_rank(n: int, m: int, p: int) -> int:
    """Rank used for uneven synthetic schemes: round((n m p)^0.93), half up."""
    return int(np.floor((n * m * p) ** 0.93 + 0.5))


def scheme_systems(rng, n, m, p, r, prob, lo=1, hi=None):
    U = ternary_rows(rng, r, n * m, prob, lo, hi)
    V = ternary_rows(rng, r, m * p, prob, lo, hi)
    Wt = ternary_rows(rng, n * p, r, prob, lo, hi)
    return U, V, Wt


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


@dataclass
class RunSpec:
    """Run parameters of a workload (interpreted identically by both sides)."""
    n_proc: int
    weights: dict
    proc0_greedy: bool = False
    seed: int = 0
    gr_p_q16: int = 49152
    step_cap: int = 0
    share_every: int = 0
    share_src_pm: int = 0
    share_dst_pm: int = 0
    share_max_rounds: int = 0
    mix_weights: tuple = (8, 4, 2, 1)

    def as_kwargs(self) -> dict:
        return dict(seed=self.seed, n_proc=self.n_proc, weights=dict(self.weights),
                    mix_weights=tuple(self.mix_weights), proc0_greedy=self.proc0_greedy,
                    gr_p_q16=self.gr_p_q16, step_cap=self.step_cap,
                    share_every=self.share_every, share_src_pm=self.share_src_pm,
                    share_dst_pm=self.share_dst_pm, share_max_rounds=self.share_max_rounds)


@dataclass
class Scheme:
    name: str
    U: np.ndarray
    V: np.ndarray
    Wt: np.ndarray
    shape: tuple = ()

    @property
    def systems(self):
        return (self.U, self.V, self.Wt)


@dataclass
class Workload:
    name: str
    schemes: list
    runs: list                      # one RunSpec per scheme
    arrivals_s: np.ndarray | None = None
    notes: str = ""
    extra: dict = field(default_factory=dict)


def tiny_2x2x2() -> Workload:
    """One system shaped like a 2x2x2 rank-7 scheme: U, V 7x4, W^T 4x7,
    p = 0.45, 64 processes of Greedy-Intersections only, seed 0."""
    rng = np.random.default_rng(1)
    U = ternary_rows(rng, 7, 4, 0.45, 1, 4)
    V = ternary_rows(rng, 7, 4, 0.45, 1, 4)
    Wt = ternary_rows(rng, 4, 7, 0.45, 1, 7)
    return Workload("tiny-2x2x2-r7", [Scheme("2x2x2:7", U, V, Wt, (2, 2, 2, 7))],
                    [RunSpec(n_proc=64, weights={"gi": 1})])


def plain_4x4x4(n_proc: int = 4096) -> Workload:
    """A system shaped like a 4x4x4 rank-49 scheme: U, V 49x16, W^T 16x49,
    p = 0.30, row nonzeros clamped to [1, 8]; 4096 processes, gi / ga / wr in
    equal shares."""
    rng = np.random.default_rng(2)
    U = ternary_rows(rng, 49, 16, 0.30, 1, 8)
    V = ternary_rows(rng, 49, 16, 0.30, 1, 8)
    Wt = ternary_rows(rng, 16, 49, 0.30, 1, 8)
    return Workload("plain-4x4x4-r49", [Scheme("4x4x4:49", U, V, Wt, (4, 4, 4, 49))],
                    [RunSpec(n_proc=n_proc, weights={"gi": 1, "ga": 1, "wr": 1})])


def plain_6x6x6(n_proc: int = 16384) -> Workload:
    """A system shaped like a 6x6x6 rank-160 scheme: U, V 160x36, W^T 36x160,
    p = 0.15, row nonzeros clamped to [1, 12]; 16384 processes with the
    default strategy weights; the best 1% shared with 10% of the active
    processes every 32 steps."""
    rng = np.random.default_rng(3)
    U = ternary_rows(rng, 160, 36, 0.15, 1, 12)
    V = ternary_rows(rng, 160, 36, 0.15, 1, 12)
    Wt = ternary_rows(rng, 36, 160, 0.15, 1, 12)
    return Workload("plain-6x6x6-r160", [Scheme("6x6x6:160", U, V, Wt, (6, 6, 6, 160))],
                    [RunSpec(n_proc=n_proc, weights=dict(PAPER_WEIGHTS), proc0_greedy=True,
                             share_every=32, share_src_pm=10, share_dst_pm=100,
                             share_max_rounds=64)])


def pools_by_rank(ranks, total: int) -> list:
    """Split `total` processes proportionally to rank: floors, then the
    largest remainders (ties to the lower index) get one more each."""
    ranks = np.asarray(ranks, dtype=np.int64)
    quota = ranks * total
    base = quota // ranks.sum()
    rem = quota - base * ranks.sum()
    left = total - int(base.sum())
    order = sorted(range(len(ranks)), key=lambda i: (-int(rem[i]), i))
    for i in order[:left]:
        base[i] += 1
    return [int(x) for x in base]


def batch_uneven(n_schemes: int = 32, total_proc: int = 65536) -> Workload:
    """32 schemes of uneven shape: (n, m, p) uniform in {2..7}^3, rank
    round((nmp)^0.93); U r x nm, V r x mp, W^T np x r, p = 0.2, at least one
    nonzero per row; pools proportional to rank summing to 65536 processes,
    default strategy weights, sharing as in the 6x6x6 workload."""
    rng = np.random.default_rng(4)
    schemes = []
    for s in range(n_schemes):
        n, m, p = (int(x) for x in rng.integers(2, 8, size=3))
        r = scheme_rank(n, m, p)
        U, V, Wt = scheme_systems(rng, n, m, p, r, 0.2)
        schemes.append(Scheme(f"{n}x{m}x{p}:{r}", U, V, Wt, (n, m, p, r)))
    pools = pools_by_rank([sc.shape[3] for sc in schemes], total_proc)
    runs = [RunSpec(n_proc=pools[i], weights=dict(PAPER_WEIGHTS), proc0_greedy=True,
                    share_every=32, share_src_pm=10, share_dst_pm=100, share_max_rounds=64)
            for i in range(n_schemes)]
    return Workload("batch-32-uneven", schemes, runs)


def serving_stream(n_jobs: int = 2000, rate_hz: float = 20.0, n_proc: int = 2048,
                   step_cap: int = 4000) -> Workload:
    """Poisson stream of reduction jobs: exponential inter-arrival times with
    mean 1 / rate; (n, m, p) uniform in {2..8}^3, rank round((nmp)^0.93),
    p = 0.12, at least one nonzero per row; each job 2048 processes with the
    default weights, program length capped at 4000, sharing as above."""
    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / rate_hz, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    schemes = []
    for j in range(n_jobs):
        n, m, p = (int(x) for x in rng.integers(2, 9, size=3))
        r = scheme_rank(n, m, p)
        U, V, Wt = scheme_systems(rng, n, m, p, r, 0.12)
        schemes.append(Scheme(f"{n}x{m}x{p}:{r}", U, V, Wt, (n, m, p, r)))
    runs = [RunSpec(n_proc=n_proc, weights=dict(PAPER_WEIGHTS), proc0_greedy=True,
                    step_cap=step_cap, share_every=32, share_src_pm=10, share_dst_pm=100,
                    share_max_rounds=64, seed=j)
            for j in range(n_jobs)]
    return Workload("serve-poisson-2000", schemes, runs, arrivals_s=arrivals)


def random_system(seed: int, rows: int, cols: int, p: float, lo: int = 1, hi: int | None = None):
    """A single seeded system for tests."""
    return ternary_rows(np.random.default_rng(seed), rows, cols, p, lo, hi)


WORKLOADS = {
    "tiny": tiny_2x2x2,
    "plain44": plain_4x4x4,
    "plain66": plain_6x6x6,
    "batch": batch_uneven,
    "serve": serving_stream,
}

DIGEST_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload_digests.txt")


def workload_digest(wl: Workload) -> str:
    """sha256 over every input matrix of a workload (and its arrival times)."""
    arrs = [A for sc in wl.schemes for A in sc.systems]
    if wl.arrivals_s is not None:
        arrs.append(wl.arrivals_s)
    return digest(*arrs)


def stored_digests() -> dict:
    """{workload name: sha256} as persisted in workload_digests.txt."""
    out = {}
    with open(DIGEST_FILE) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if len(line) == 2:
                out[line[0]] = line[1]
    return out


def write_digests() -> None:
    """Persist the digest of every workload's inputs (run when a generator
    is deliberately changed; the tests check the inputs still match)."""
    lines = ["# sha256 of each workload's inputs (workloads.workload_digest); written by",
             "# python -m paper_2512_13365_amd.workloads"]
    for fn in WORKLOADS.values():
        wl = fn()
        lines.append(f"{wl.name} {workload_digest(wl)}")
    with open(DIGEST_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    write_digests()
