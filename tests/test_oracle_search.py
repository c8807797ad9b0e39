"""Pins of the oracle's iGNNS (Section 3): exhaustive limit, budget,
budget-prefix property, expansion test and the eager step's closed form
(Table 1)."""

import json
import os
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle as O
from oracle.ignns import expansion_rejects

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gmm_u8(seed, n, dim, clusters, sigma):
    rng = np.random.default_rng(seed)
    c = rng.uniform(40, 215, (clusters, dim))
    lab = rng.integers(0, clusters, n)
    return np.clip(np.rint(c[lab] + rng.standard_normal((n, dim)) * sigma), 0, 255).astype(np.uint8)


@pytest.fixture(scope="module")
def small_graph():
    X = _gmm_u8(1, 400, 8, 5, 12.0)
    ids, d = O.exact_graph(X[:300], 6)
    return O.OracleGraph(X[:300].copy(), ids, d, 6), X[300:]


def test_exhaustive_budget_returns_exact_neighbours(small_graph):
    """speedup = 1 gives B = n; the restart permutation covers every node, so
    the result is the exact top-k of the snapshot (brute force)."""
    g, Q = small_graph
    p = O.Params(k=6, speedup=1, e_num=5, e_den=1)
    for j in range(40):
        r = O.ignns(g, Q[j], key=1000 + j, p=p)
        assert r.evals == g.n
        assert r.pairs == O.exact_row(g.X, 0, 6, q=Q[j], exclude=None)


@pytest.mark.parametrize("speedup", [1, 2, 7, 50, 1000])
def test_evals_equal_budget(small_graph, speedup):
    g, Q = small_graph
    p = O.Params(k=6, speedup=speedup)
    B = O.budget(g.n, 6, speedup)
    for j in range(10):
        r = O.ignns(g, Q[j], key=j, p=p, record=True)
        assert r.evals == B == len(r.sequence)
        assert len(set(r.sequence)) == B          # never re-evaluated
        assert len(r.pairs) == min(6, B)


def test_budget_prefix_property(small_graph):
    """The evaluation sequence at budget B is a prefix of the sequence at any
    larger budget (deterministic draws + stop right after the B-th
    evaluation); hence the k-th distance never increases with the budget."""
    g, Q = small_graph
    for j in range(10):
        runs = []
        for sp in (30, 12, 5, 2, 1):
            p = O.Params(k=6, speedup=sp)
            runs.append(O.ignns(g, Q[j], key=77 + j, p=p, record=True))
        for a, b in zip(runs, runs[1:]):
            assert b.sequence[: len(a.sequence)] == a.sequence
            assert b.pairs[-1] <= a.pairs[-1]


def test_expansion_rule_integer_form():
    # e = 5: reject iff 1 + d_r > 5 (1 + d_best)
    assert not expansion_rejects(9, 1, 5, 1)      # 10 == 5 * 2
    assert expansion_rejects(10, 1, 5, 1)         # 11 > 10
    # e = 6/5
    assert not expansion_rejects(11, 9, 6, 5)     # 5*12 = 60 == 6*10
    assert expansion_rejects(12, 9, 6, 5)
    # a restart that is the new best is always kept (d_best includes it)
    assert not expansion_rejects(3, 3, 6, 5)


def test_first_evaluation_is_first_permutation_node(small_graph):
    g, Q = small_graph
    p = O.Params(k=6, speedup=10)
    r = O.ignns(g, Q[0], key=5, p=p, record=True)
    first = O.RestartOrder(g.n, p.seed, 5).next_unvisited(set())
    assert r.sequence[0] == first


def _eager_scan_count(k: int, improving_positions: tuple, seed: int) -> int:
    """Build a graph in which the first restart is node c, whose stored list
    holds k neighbours at strictly increasing distances from c; the ones at
    ``improving_positions`` lie between c and q (closer to q than c), the
    others lie beyond c.  Run the oracle's iGNNS and count the evaluations
    between c and the first improving neighbour (exclusive)."""
    n = k + 1
    dim = 2
    q = np.array([200, 128], dtype=np.int64)
    c_pt = np.array([100, 128], dtype=np.int64)          # distance 100 from q
    # place c at the id the permutation draws first
    p = O.Params(k=k, speedup=1, e_num=5, e_den=1, seed=seed)
    key = 3
    first = O.RestartOrder(n, p.seed, key).next_unvisited(set())
    others = [i for i in range(n) if i != first]
    X = np.zeros((n, dim), dtype=np.uint8)
    X[first] = c_pt
    for pos, node in enumerate(others):
        r = pos + 1                                        # distinct radii
        sign = 1 if pos in improving_positions else -1
        X[node] = c_pt + np.array([sign * r, 0])
    ids = np.full((n, k), -1, dtype=np.int64)
    d = np.full((n, k), O.INF_INT, dtype=np.int64)
    ids[first] = others                                    # sorted by radius
    d[first] = [(pos + 1) ** 2 for pos in range(k)]
    for node in others:                                   # any valid lists
        lst = [v for v in range(n) if v != node][:k]
        ids[node] = lst
        d[node] = [O.sqdist(X[node], X[v]) for v in lst]
    g = O.OracleGraph(X, ids, d, k)
    res = O.ignns(g, q.astype(np.uint8), key=key, p=p, record=True)
    assert res.sequence[0] == first
    scan = res.sequence[1:]
    improving = {others[pos] for pos in improving_positions}
    for cnt, v in enumerate(scan):
        if v in improving:
            return cnt
    raise AssertionError("no improving neighbour evaluated")


@pytest.mark.parametrize("k,h", [(4, 1), (10, 1), (10, 2), (10, 3), (6, 2)])
def test_eager_step_matches_negative_hypergeometric_mean(k, h):
    """Section 3: the eager step moves to the first improving neighbour, so
    with h improving entries placed at random among k the expected number of
    non-improving evaluations before it is (k - h) / (h + 1) (the paper's
    e_s = e_l / (1 + e_h)).  Averaged exactly over every placement."""
    total = Fraction(0)
    cnt = 0
    for positions in combinations(range(k), h):
        total += _eager_scan_count(k, positions, seed=11)
        cnt += 1
    assert total / cnt == Fraction(k - h, h + 1)


def test_table1_values_follow_from_the_eager_step_formula():
    """Table 1: e_h = k / 2^d, e_l = k - e_h, e_s = e_l / (1 + e_h),
    speedup = k / e_s; compared with the printed (truncated) values."""
    with open(os.path.join(GOLDEN, "table1_eager_step.json")) as f:
        table = json.load(f)
    for col in table["columns"]:
        k, dim = col["k"], col["d"]
        e_h = k / 2 ** dim
        e_l = k - e_h
        e_s = e_l / (1 + e_h)
        assert e_h == pytest.approx(col["e_h"], abs=1e-9)
        assert e_l == pytest.approx(col["e_l"], abs=1e-9)
        assert e_s == pytest.approx(col["e_s"], abs=0.01)
        assert k / e_s == pytest.approx(col["speedup"], abs=0.01)
        # the closed form used by the eager-step test at integer h
        if float(e_h).is_integer():
            h = int(e_h)
            assert Fraction(k - h, h + 1) == Fraction(e_s).limit_denominator(1000)


def test_query_keys_are_in_their_own_namespace(small_graph):
    g, Q = small_graph
    p = O.Params(k=6, speedup=10)
    res = O.query(g, Q[:3], p, first_seq=4, record=True)
    for j, r in enumerate(res):
        again = O.ignns(g, Q[j], key=O.QUERY_KEY_BASE + 4 + j, p=p, record=True)
        assert again.sequence == r.sequence
