"""Pins of the exact rows by branch and bound over a grouping
(oracle.GroupedExactRows), the lazily built exact snapshot
(oracle.LazyExactGraph) and the batch phases run on it: each equals the
brute-force definition (Section 2.1's naive method, Section 8.5.2's ground
truth) whatever the grouping."""

import numpy as np
import pytest

import oracle as O
from oracle.online import merge_proposals, search_and_propose


def _float_points(seed, n, dim, clusters, sigma=0.2):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((clusters, dim))
    lab = rng.integers(0, clusters, n)
    return (c[lab] + rng.standard_normal((n, dim)) * sigma).astype(np.float32), lab


def _groupings(n, lab, seed):
    rng = np.random.default_rng(seed)
    return {
        "labels": lab,
        "one": np.zeros(n, dtype=np.int64),
        "singletons": np.arange(n),
        "random": rng.integers(0, 7, n),
        "by_id": np.arange(n) // 13,
    }


@pytest.mark.parametrize("which", ["labels", "one", "singletons", "random", "by_id"])
def test_grouped_rows_equal_brute_force_float(which):
    X, lab = _float_points(1, 400, 6, 5)
    grp = _groupings(400, lab, 2)[which]
    rows = O.GroupedExactRows(X, 7, grp)
    rng = np.random.default_rng(3)
    for u in range(0, 400, 9):
        assert rows.row(X[u], exclude=u) == O.exact_row(X, u, 7)
    for _ in range(20):
        q = (rng.standard_normal(6) * 1.5).astype(np.float32)
        assert rows.row(q) == O.exact_row(X, 0, 7, q=q, exclude=None)


@pytest.mark.parametrize("which", ["labels", "random", "by_id"])
def test_grouped_rows_equal_brute_force_with_ties(which):
    """uint8 points on 3 values per coordinate: many exact ties, which the
    lists must break by id."""
    rng = np.random.default_rng(4)
    X = rng.integers(0, 3, (300, 3)).astype(np.uint8) * 10
    lab = X[:, 0].astype(np.int64)
    grp = _groupings(300, lab, 5)[which]
    rows = O.GroupedExactRows(X, 9, grp)
    for u in range(300):
        assert rows.row(X[u], exclude=u) == O.exact_row(X, u, 9)


def test_lazy_graph_lists_equal_the_exact_graph():
    X, lab = _float_points(6, 500, 8, 6)
    ids, d = O.exact_graph(X, 5)
    g = O.LazyExactGraph(X, 5, lab)
    for u in range(0, 500, 7):
        assert g.neighbours(u) == ids[u].tolist()
        assert [p[0] for p in g.neighbour_pairs(u)] == d[u].tolist()
    assert g.cached() == len(range(0, 500, 7))


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_batch_phases_on_the_lazy_snapshot_equal_insert_batch(kind):
    if kind == "f32":
        X, lab = _float_points(7, 660, 8, 5)
    else:
        rng = np.random.default_rng(8)
        c = rng.uniform(40, 215, (5, 8))
        lab = rng.integers(0, 5, 660)
        X = np.clip(np.rint(c[lab] + rng.standard_normal((660, 8)) * 12), 0, 255).astype(np.uint8)
    k = 6
    p = O.Params(k=k, speedup=8, depth=2, e_num=3, e_den=2)
    ids, d = O.exact_graph(X[:600], k)
    full = O.OracleGraph(X[:600].copy(), ids, d, k)
    want = O.insert_batch(full, X[600:660], p)
    lazy = O.LazyExactGraph(X[:600], k, lab[:600])
    search, final, props, upd, sims = search_and_propose(lazy, X[600:660], p)
    assert sims == want.sims and upd == want.update_evals
    assert props == want.proposals
    assert final == want.final_lists
    merged = merge_proposals(lazy, props, k)
    for u, pairs in merged.items():
        assert want.graph.neighbour_pairs(u) == pairs
