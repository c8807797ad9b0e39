"""Pins of the oracle's online insertion (Algorithms 1 and 2 with batch
semantics): exhaustive special case, the literal sequential transcription,
update cost bound (Section 4), invariants and batch independence."""

import numpy as np
import pytest

import oracle as O


def _gmm(seed, n, dim, clusters, sigma, kind="u8"):
    rng = np.random.default_rng(seed)
    if kind == "u8":
        c = rng.uniform(40, 215, (clusters, dim))
        lab = rng.integers(0, clusters, n)
        x = c[lab] + rng.standard_normal((n, dim)) * sigma
        return np.clip(np.rint(x), 0, 255).astype(np.uint8)
    c = rng.standard_normal((clusters, dim))
    lab = rng.integers(0, clusters, n)
    return (c[lab] + rng.standard_normal((n, dim)) * sigma).astype(np.float32)


def _graph(X, k):
    ids, d = O.exact_graph(X, k)
    return O.OracleGraph(X.copy(), ids, d, k)


def check_invariants(g: O.OracleGraph):
    """Lists: min(k, n-1) distinct non-self ids < n, sorted by (d, id), and
    every stored distance equals the recomputed one."""
    n, k = g.n, g.k
    want_len = min(k, n - 1)
    for u in range(n):
        pairs = g.neighbour_pairs(u)
        assert len(pairs) == want_len, (u, pairs)
        vs = [v for _, v in pairs]
        assert len(set(vs)) == len(vs) and u not in vs
        assert all(0 <= v < n for v in vs)
        assert pairs == sorted(pairs)
        for d, v in pairs:
            assert d == O.sqdist(g.X[u], g.X[v])


@pytest.mark.parametrize("batch", [1, 3, 8])
@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_exhaustive_parameters_rebuild_the_exact_graph(batch, kind):
    """speedup = 1 (search is exhaustive) and DEPTH = 0 (every node is
    updated): the online graph must equal the brute-force graph of all the
    points, whatever the batch sizes."""
    X = _gmm(2, 90, 4, 3, 10.0 if kind == "u8" else 0.3, kind)
    k = 5
    g = _graph(X[:50], k)
    p = O.Params(k=k, speedup=1, depth=0)
    g2, _ = O.insert_stream(g, X[50:], batch, p)
    ids, d = O.exact_graph(X, k)
    assert np.array_equal(g2.ids, ids)
    assert np.array_equal(g2.dist, d)


def test_exhaustive_search_depth2_gives_exact_new_lists():
    X = _gmm(3, 120, 4, 3, 10.0)
    g = _graph(X[:80], 5)
    p = O.Params(k=5, speedup=1, depth=2)
    res = O.insert_batch(g, X[80:96], p)
    ids, d = O.exact_graph(X[:96], 5)
    # new nodes' lists: exact search + exact peers -> exact
    assert np.array_equal(res.graph.ids[80:96], ids[80:96])


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_batch_of_one_equals_literal_algorithms_1_and_2(depth):
    X = _gmm(4, 330, 8, 4, 12.0)
    k = 6
    g_batch = _graph(X[:300], k)
    g_lit = g_batch.copy()
    p = O.Params(k=k, speedup=6, depth=depth)
    for i in range(300, 330):
        g_batch = O.insert_batch(g_batch, X[i:i + 1], p).graph
        g_lit = O.insert_sequential_literal(g_lit, X[i], p)
        assert np.array_equal(g_batch.ids, g_lit.ids), i
        assert np.array_equal(g_batch.dist, g_lit.dist), i


def test_update_cost_bound_k_squared():
    """Section 4: the update needs at most k^DEPTH similarities; with level-1
    distances reused, level 2 holds at most k^2 nodes."""
    X = _gmm(5, 700, 8, 6, 12.0)
    k = 10
    g = _graph(X[:600], k)
    p = O.Params(k=k, speedup=10, depth=2)
    res = O.insert_batch(g, X[600:700], p)
    assert max(res.update_evals) <= k * k
    assert min(res.update_evals) > 0
    b = 100
    for i, s in enumerate(res.sims):
        assert s == res.search[i].evals + (b - 1) + res.update_evals[i]


def test_invariants_after_stream():
    X = _gmm(6, 500, 8, 5, 12.0)
    g = _graph(X[:400], 7)
    p = O.Params(k=7, speedup=8, depth=2)
    g2, _ = O.insert_stream(g, X[400:], 25, p)
    check_invariants(g2)


def test_invariants_float():
    X = _gmm(7, 260, 6, 4, 0.2, "f32")
    g = _graph(X[:200], 5)
    g2, _ = O.insert_stream(g, X[200:], 16, O.Params(k=5, speedup=5))
    check_invariants(g2)


def test_search_is_independent_of_batch_composition():
    X = _gmm(8, 350, 8, 4, 12.0)
    g = _graph(X[:300], 6)
    p = O.Params(k=6, speedup=8)
    res = O.insert_batch(g, X[300:340], p, record=True)
    for i in (0, 7, 39):
        alone = O.ignns(g, X[300 + i], key=300 + i, p=p, record=True)
        assert alone.sequence == res.search[i].sequence


def test_proposals_never_target_batch_points_and_merge_keeps_best():
    X = _gmm(9, 240, 6, 3, 12.0)
    g = _graph(X[:200], 5)
    p = O.Params(k=5, speedup=4)
    res = O.insert_batch(g, X[200:240], p)
    assert all(u < 200 for u, _, _ in res.proposals)
    by_u = {}
    for u, d, s in res.proposals:
        by_u.setdefault(u, []).append((d, s))
    for u, props in list(by_u.items())[:50]:
        want = sorted(g.neighbour_pairs(u) + props)[:5]
        assert res.graph.neighbour_pairs(u) == want


def test_small_graph_lists_grow_to_k():
    X = _gmm(10, 12, 3, 2, 12.0)
    g = _graph(X[:3], 5)                       # lists of length 2
    g2, _ = O.insert_stream(g, X[3:], 2, O.Params(k=5, speedup=1, depth=0))
    check_invariants(g2)
    ids, d = O.exact_graph(X, 5)
    assert np.array_equal(g2.ids, ids)
