"""Pins of the Dörfler marking oracle (oracle/dpg_marking.py): on tiny
inputs, brute force over all subsets -- the refined set is a smallest set of
cells whose values reach the refinement fraction of the total and carries the
largest sum among sets of its size; the coarsened set is a largest set whose
values stay within the coarsening fraction; the two never meet -- and closed
cases (equal values, fraction 0 and 1, zeros)."""
import itertools
import math

import numpy as np
import pytest

from oracle import dpg_marking as M


def _subsets(n):
    for k in range(n + 1):
        for s in itertools.combinations(range(n), k):
            yield s


@pytest.mark.parametrize("seed", range(12))
def test_marking_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    v = rng.exponential(1.0, n) ** 2
    fr, fc = 0.3, 0.05
    f = M.dorfler_mark(v, fr, fc)
    T = float(np.sum(v))
    ref = [i for i in range(n) if f[i] == 1]
    crs = [i for i in range(n) if f[i] == -1]
    assert not set(ref) & set(crs)
    # refinement: minimal cardinality reaching fr T, and the largest sum of that size
    kmin = min(len(s) for s in _subsets(n) if sum(v[list(s)]) >= fr * T - 1e-12 * T)
    assert len(ref) == kmin
    best = max(sum(v[list(s)]) for s in itertools.combinations(range(n), kmin))
    assert math.isclose(sum(v[ref]), best, rel_tol=1e-12)
    # coarsening: maximal cardinality within fc T (among cells not refined)
    rest = [i for i in range(n) if f[i] != 1]
    kmax = max(len(s) for s in _subsets(len(rest)) if sum(v[[rest[j] for j in s]]) <= fc * T + 1e-12 * T)
    assert len(crs) == kmax
    assert sum(v[crs]) <= fc * T * (1 + 1e-12)


def test_marking_closed_cases():
    v = np.ones(20)
    f = M.dorfler_mark(v, 0.3, 0.05)
    assert list(np.nonzero(f == 1)[0]) == list(range(6))        # ceil(0.3 * 20) cells, lowest indices first
    assert list(np.nonzero(f == -1)[0]) == [19]                 # 1 / 20 = 0.05 of the total
    assert np.all(M.dorfler_mark(v, 0.0, 0.0) == 0)
    assert np.all(M.dorfler_mark(v, 1.0, 0.0) == 1)
    w = np.array([0.0, 3.0, 0.0, 1.0])
    f = M.dorfler_mark(w, 0.5, 0.0)
    assert list(f) == [-1, 1, -1, 0]                            # zeros sum to 0 <= 0
    assert list(M.dorfler_mark(np.zeros(3), 0.3, 0.05)) == [-1, -1, -1]
    assert len(M.dorfler_mark(np.zeros(0), 0.3, 0.05)) == 0


def test_marking_planted_ranking_mistake_fails(monkeypatch):
    def bad(values, fr, fc):
        # ranks by increasing value: a plausible slip in the ranking
        v = [float(x) for x in values]
        order = sorted(range(len(v)), key=lambda i: (v[i], i))
        total = sum(v[i] for i in order)
        flags = np.zeros(len(v), np.int8)
        before = 0.0
        for i in order:
            if before < fr * total:
                flags[i] = 1
            before += v[i]
        return flags
    monkeypatch.setattr(M, "dorfler_mark", bad)
    with pytest.raises(AssertionError):
        for seed in range(12):
            test_marking_against_brute_force(seed)
