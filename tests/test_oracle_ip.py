"""Pins of the oracle's inner-product similarity (Section 3: the method
applies to any similarity, metric or not).  The dissimilarity is the negated
inner product; the expansion test, stated for positive similarities, is
applied to exp(q . r), where the ratio s_r < s_max / e becomes the
difference (q . best) - (q . r) > ln e."""

import math

import numpy as np
import pytest

import oracle as O
from oracle.ignns import expansion_rejects


def ip_points(seed, n, d):
    rng = np.random.default_rng(seed)
    # norms spread over a factor of ~8: the inner product favours long rows
    return (rng.standard_normal((n, d)) * rng.uniform(0.25, 2.0, (n, 1))).astype(np.float32)


def test_inner_product_closed_forms():
    a = np.array([3.0, 4.0], dtype=np.float32)
    assert O.inner_product(a, np.array([4.0, -3.0], np.float32)) == 0.0      # orthogonal
    assert O.inner_product(a, 2 * a) == 50.0                                  # parallel
    assert O.inner_product(a, -a) == -25.0
    assert O.dissim(a, 2 * a, "ip") == -50.0 and O.dissim(a, -a, "ip") == 25.0
    assert O.dissim(a, 2 * a) == 25.0                                         # squared L2


def test_inner_product_graph_is_not_the_euclidean_one():
    # points 1, 2, 10 on a line: by inner product every node's most similar
    # other node is 10 (the longest), not its Euclidean nearest; 10's list
    # puts 2 before 1
    X = np.array([[1.0], [2.0], [10.0]], dtype=np.float32)
    ids, d = O.exact_graph_ip(X, 2)
    assert ids.tolist() == [[2, 1], [2, 0], [1, 0]]
    assert d.tolist() == [[-10.0, -2.0], [-20.0, -2.0], [-20.0, -10.0]]
    l2_ids, _ = O.exact_graph(X, 2)
    assert l2_ids[0, 0] == 1 and l2_ids[1, 0] == 0


def test_exact_graph_ip_against_nested_loops():
    X = ip_points(1, 40, 5)
    ids, d = O.exact_graph_ip(X, 6)
    for u in range(40):
        pairs = sorted((-sum(float(X[u, j]) * float(X[v, j]) for j in range(5)), v)
                       for v in range(40) if v != u)[:6]
        assert ids[u].tolist() == [v for _, v in pairs]
        assert np.allclose(d[u], [dd for dd, _ in pairs], rtol=1e-12, atol=1e-12)


def test_expansion_rule_on_inner_products():
    ln = math.log(3 / 2)
    assert ln == pytest.approx(0.4054651)
    assert expansion_rejects(-4.5, -5.0, 3, 2, "ip")          # 0.5 > ln 1.5
    assert not expansion_rejects(-4.7, -5.0, 3, 2, "ip")      # 0.3 <= ln 1.5
    assert not expansion_rejects(-5.0, -5.0, 3, 2, "ip")      # the best itself
    assert not expansion_rejects(7.0, 7.0, 3, 2, "ip")        # a first, dissimilar restart
    assert expansion_rejects(2.0, 1.5, 11, 10, "ip")          # 0.5 > ln 1.1
    # the squared-L2 rule is unchanged: (1 + d_r) e_den > e_num (1 + d_best)
    assert expansion_rejects(10, 5, 3, 2) and not expansion_rejects(8, 5, 3, 2)


def test_ip_exhaustive_search_is_exact():
    X = ip_points(2, 300, 8)
    base, Q = X[:260], X[260:]
    ids, d = O.exact_graph_ip(base, 7)
    g = O.OracleGraph(base, ids, d, 7)
    p = O.Params(k=7, speedup=1, e_num=3, e_den=2, seed=9, metric="ip")
    for j, q in enumerate(Q):
        r = O.ignns(g, q, 1000 + j, p)
        dq = O.dissim_many(q, base, "ip")
        want = sorted(zip(dq.tolist(), range(260)))[:7]
        assert r.evals == 260
        assert [v for _, v in r.pairs] == [v for _, v in want]
    ps = O.Params(k=7, speedup=10, e_num=3, e_den=2, seed=9, metric="ip")
    for j, q in enumerate(Q):
        assert O.ignns(g, q, 1000 + j, ps).evals == O.budget(260, 7, 10)


@pytest.mark.parametrize("batches", [[7, 1, 5], [13]])
def test_ip_exhaustive_insertion_gives_the_exact_graph(batches):
    total = 120 + sum(batches)
    X = ip_points(3, total, 6)
    ids, d = O.exact_graph_ip(X[:120], 5)
    g = O.OracleGraph(X[:120].copy(), ids, d, 5)
    p = O.Params(k=5, speedup=1, e_num=3, e_den=2, depth=0, seed=4, metric="ip")
    lo = 120
    for b in batches:
        g = O.insert_batch(g, X[lo:lo + b], p).graph
        lo += b
    want_ids, want_d = O.exact_graph_ip(X, 5)
    assert np.array_equal(g.ids, want_ids)
    assert np.array_equal(g.dist, want_d)


def test_ip_batch_of_one_equals_the_literal_algorithms():
    X = ip_points(5, 160, 6)
    ids, d = O.exact_graph_ip(X[:150], 6)
    p = O.Params(k=6, speedup=5, e_num=3, e_den=2, depth=2, seed=8, metric="ip")
    g1 = O.OracleGraph(X[:150].copy(), ids, d, 6)
    g2 = O.OracleGraph(X[:150].copy(), ids.copy(), d.copy(), 6)
    for i in range(150, 160):
        g1 = O.insert_batch(g1, X[i:i + 1], p).graph
        g2 = O.insert_sequential_literal(g2, X[i], p)
    assert np.array_equal(g1.ids, g2.ids)
    assert np.array_equal(g1.dist, g2.dist)
