"""Independent pure-Python helpers for checking CSE results.

Written from the definitions of Sec. 3.2.1 and Algorithm 1, sharing nothing
with the oracle's C code or the HIP library: symbolic replay of a program,
re-expansion of fresh variables, pair counting with a dictionary, and an
exhaustive search over all substitution orders for tiny systems.
"""
from __future__ import annotations

import os
from functools import lru_cache

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """Parse a golden text file into {section: list of rows or int}."""
    out = {}
    cur = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if len(parts) == 1 and not parts[0].lstrip("-").isdigit():
                cur = parts[0]
                out[cur] = []
            elif len(parts) == 2 and not parts[0].lstrip("-").isdigit():
                if parts[0] in out and isinstance(out[parts[0]], list):
                    out[parts[0]].append([int(parts[1])])
                else:
                    out[parts[0]] = int(parts[1])
                cur = None
            elif parts[0] == "subst":
                out.setdefault("subst", []).append([int(x) for x in parts[1:]])
            else:
                out[cur].append(parts)
    return out


def naive_count(A) -> int:
    A = np.asarray(A)
    return int(sum(int(np.count_nonzero(r)) - 1 for r in A))


def pair_counts(A) -> dict:
    """{(a, b, s): c} over canonical pairs of every row (1-based a < b)."""
    A = np.asarray(A)
    counts = {}
    for row in A:
        nz = np.flatnonzero(row)
        for i in range(len(nz)):
            for j in range(i + 1, len(nz)):
                a, b = int(nz[i]) + 1, int(nz[j]) + 1
                s = int(row[nz[i]]) * int(row[nz[j]])
                counts[(a, b, s)] = counts.get((a, b, s), 0) + 1
    return counts


def replay(A0, prog):
    """Apply program triples to A0 following Algorithm 1's substitution.
    Returns (final matrix, list of c per step)."""
    A0 = np.asarray(A0, dtype=np.int64)
    n_e, n_x = A0.shape
    A = np.zeros((n_e, n_x + len(prog)), np.int64)
    A[:, :n_x] = A0
    cs = []
    for t, (a, b, s) in enumerate(prog):
        k = n_x + t
        c = 0
        for i in range(n_e):
            va, vb = A[i, a - 1], A[i, b - 1]
            if va != 0 and vb != 0 and va * vb == s:
                A[i, k] = va
                A[i, a - 1] = 0
                A[i, b - 1] = 0
                c += 1
        cs.append(c)
    return A, cs


def expansions(n_x, prog):
    """Expansion of every variable over x_1..x_{n_x} (Sec. 3.2.1 definition
    x_k = x_a + s x_b)."""
    E = [np.eye(n_x, dtype=np.int64)[i] for i in range(n_x)]
    for a, b, s in prog:
        E.append(E[a - 1] + s * E[b - 1])
    return np.array(E)


def check_program(A0, prog, cost):
    """Validate a program against the definitions; returns the final matrix.
    - every step rewrites c >= 2 rows (Algorithm 1 selects c > 1);
    - cost = n_f + naive(final) = naive(A0) - sum(c - 1) (Sec. 3.2.1);
    - every fresh variable expands to a ternary vector with >= 2 terms;
    - every final row re-expands to its input row;
    - no pair occurs twice at the end (Algorithm 1's stopping rule)."""
    A0 = np.asarray(A0)
    n_x = A0.shape[1]
    prog = [tuple(int(v) for v in p) for p in prog]
    for t, (a, b, s) in enumerate(prog):
        assert 1 <= a < b <= n_x + t and s in (1, -1), (t, a, b, s)
    F, cs = replay(A0, prog)
    assert all(c >= 2 for c in cs), cs
    assert cost == len(prog) + naive_count(F)
    assert cost == naive_count(A0) - sum(c - 1 for c in cs)
    E = expansions(n_x, prog)
    for k in range(n_x, len(E)):
        assert np.all(np.abs(E[k]) <= 1) and np.count_nonzero(E[k]) >= 2
    assert np.array_equal(F @ E, A0.astype(np.int64))
    return F


def is_terminal(F):
    return all(c < 2 for c in pair_counts(F).values())


def brute_force_optimum(A0) -> int:
    """Minimal Cost(E) over every sequence of pair substitutions with c >= 2
    (Sec. 3.2.1 cost).  Substitutions with c = 1 cannot help: the fresh
    variable then sits in one row only, so no later pair with it repeats.
    Variables are identified by their expansion, so states reached by
    commuting substitutions coincide in the memo."""
    A0 = np.asarray(A0, dtype=np.int64)
    n_x = A0.shape[1]
    unit = [tuple(int(v) for v in np.eye(n_x, dtype=np.int64)[i]) for i in range(n_x)]
    rows = []
    for r in A0:
        rows.append(frozenset((unit[j], int(r[j])) for j in np.flatnonzero(r)))
    naive = naive_count(A0)

    def canon(state):
        return tuple(sorted(tuple(sorted(r)) for r in state))

    @lru_cache(maxsize=None)
    def best_saving(key):
        state = [dict((v, s) for v, s in r) for r in key]
        counts = {}
        for r in state:
            vs = sorted(r)
            for i in range(len(vs)):
                for j in range(i + 1, len(vs)):
                    pk = (vs[i], vs[j], r[vs[i]] * r[vs[j]])
                    counts[pk] = counts.get(pk, 0) + 1
        best = 0
        for (va, vb, s), c in counts.items():
            if c < 2:
                continue
            vk = tuple(x + s * y for x, y in zip(va, vb))
            new = []
            for r in state:
                if va in r and vb in r and r[va] * r[vb] == s:
                    r2 = dict(r)
                    sa = r2.pop(va)
                    r2.pop(vb)
                    r2[vk] = sa
                    new.append(tuple(sorted(r2.items())))
                else:
                    new.append(tuple(sorted(r.items())))
            best = max(best, (c - 1) + best_saving(tuple(sorted(new))))
        return best

    return naive - best_saving(canon(rows))


def standard_scheme(n, m, p):
    """The definition of the product C = A B as a scheme of rank n m p: one
    product A_ij B_jk per (i, j, k), added into C_ik.  U over A (n x m), V
    over B (m x p), W over C (n x p), all row-major."""
    r = n * m * p
    U = np.zeros((r, n * m), np.int8)
    V = np.zeros((r, m * p), np.int8)
    W = np.zeros((r, n * p), np.int8)
    t = 0
    for i in range(n):
        for j in range(m):
            for k in range(p):
                U[t, i * m + j] = V[t, j * p + k] = W[t, i * p + k] = 1
                t += 1
    return U, V, W


def brent_ok(U, V, W, n, m, p) -> bool:
    """The Brent equations: sum_t U_t[i,j] V_t[j',k] W_t[i',k'] equals 1 when
    j = j', i = i', k = k' and 0 otherwise, i.e. the products reconstruct
    C = A B for every A and B."""
    T = np.einsum("ta,tb,tc->abc", U.astype(np.int64), V.astype(np.int64), W.astype(np.int64))
    ref = np.zeros((n * m, m * p, n * p), np.int64)
    for i in range(n):
        for j in range(m):
            for k in range(p):
                ref[i * m + j, j * p + k, i * p + k] = 1
    return bool(np.array_equal(T, ref))
