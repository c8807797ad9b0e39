"""Pins of the oracle's building blocks: restart permutation, distances and
the exact k-nn graph (brute force), checked against definitions, number
theory and independent computations -- not against the oracle itself."""

import math

import numpy as np
import pytest

import oracle as O
from oracle.restart import modulus_for


# ---------------------------------------------------------------- restarts
@pytest.mark.parametrize("n", list(range(1, 70)) + [100, 257, 1000, 4096, 4097])
def test_restart_sequence_is_a_full_period_permutation(n):
    """Hull-Dobell: with c odd and a = 1 (mod 4) the LCG mod 2^w has full
    period, so x_0..x_{m-1} is a permutation of [0, m) and cycle-walking
    past values >= n visits every node exactly once."""
    for key in (0, 1, n, 12345, (1 << 62) + 7):
        order = O.RestartOrder(n, seed=99, key=key)
        seq = order.full_sequence()
        assert sorted(seq) == list(range(modulus_for(n)))
        drawn = []
        while True:
            r = order.next_unvisited(set())
            if r is None:
                break
            drawn.append(r)
        assert sorted(drawn) == list(range(n))


def test_restart_params_satisfy_hull_dobell():
    for n in (3, 5, 17, 1000, 100_000, 2_000_000):
        for key in range(20):
            m, a, c, x0 = O.restart_params(n, 7, key)
            assert m & (m - 1) == 0 and m >= n and m < 2 * n
            assert c % 2 == 1 and a % 4 == 1 and 0 <= x0 < m


def test_restart_skips_visited_without_consuming_them_twice():
    order = O.RestartOrder(50, seed=1, key=2)
    full = [x for x in order.full_sequence() if x < 50]
    visited = set(full[1::2])
    got = []
    while (r := order.next_unvisited(visited)) is not None:
        got.append(r)
    assert got == full[0::2]


def test_splitmix64_is_a_bijection_on_small_state_window():
    # the output function of SplitMix64 is a bijection of 64-bit words;
    # distinct consecutive states must give distinct outputs
    outs = set()
    s = 0
    for _ in range(5000):
        s, z = O.splitmix64_next(s)
        outs.add(z)
    assert len(outs) == 5000


# ---------------------------------------------------------------- distance
def test_sqdist_u8_exact_and_symmetric():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 256, 64).astype(np.uint8)
    b = rng.integers(0, 256, 64).astype(np.uint8)
    want = sum((int(x) - int(y)) ** 2 for x, y in zip(a, b))
    assert O.sqdist(a, b) == want == O.sqdist(b, a)
    # extremes: d * 255^2 fits int32
    z = np.zeros(64, np.uint8)
    f = np.full(64, 255, np.uint8)
    assert O.sqdist(z, f) == 64 * 255 * 255 < 2 ** 31


# ---------------------------------------------------------------- exact graph
def test_exact_graph_hand_example():
    # 1-D points 0, 1, 3, 7 (ids 0..3), k = 2, squared distances:
    # 0: to 1 ->1, to 3 ->9, to 7 ->49       list [1, 2]
    # 1: to 0 ->1, to 3 ->4, to 7 ->36       list [0, 2]
    # 2: to 1 ->4, to 0 ->9, to 7 ->16       list [1, 0]
    # 3: to 3 ->16, to 1 ->36, to 0 ->49     list [2, 1]
    X = np.array([[0], [1], [3], [7]], dtype=np.uint8)
    ids, d = O.exact_graph(X, 2)
    assert ids.tolist() == [[1, 2], [0, 2], [1, 0], [2, 1]]
    assert d.tolist() == [[1, 9], [1, 4], [4, 9], [16, 36]]


def test_exact_graph_tie_break_by_id():
    # all points equal: every distance is 0, lists are the smallest other ids
    X = np.full((6, 3), 9, dtype=np.uint8)
    ids, d = O.exact_graph(X, 3)
    for u in range(6):
        want = [v for v in range(6) if v != u][:3]
        assert ids[u].tolist() == want
        assert d[u].tolist() == [0, 0, 0]


@pytest.mark.parametrize("seed", range(4))
def test_exact_graph_blas_equals_nested_loops_u8(seed):
    rng = np.random.default_rng(seed)
    n, dim, k = 150, 5, 7
    # few distinct values -> many distance ties
    X = rng.integers(0, 4, (n, dim)).astype(np.uint8)
    a = O.exact_graph(X, k, chunk=37)
    b = O.exact_graph_loops(X, k)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_exact_graph_blas_equals_nested_loops_float():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((120, 6)).astype(np.float32)
    X[10] = X[11]                          # an exact tie
    a = O.exact_graph(X, 5, chunk=50)
    b = O.exact_graph_loops(X, 5)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])


def test_exact_graph_small_n_pads():
    X = np.array([[1, 2], [3, 4], [5, 7]], dtype=np.uint8)
    ids, d = O.exact_graph(X, 5)
    assert ids.shape == (3, 5)
    assert (ids[:, 2:] == -1).all() and (d[:, 2:] == O.INF_INT).all()
    assert ids[0, :2].tolist() == [1, 2]


def test_exact_row_matches_graph():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 256, (300, 8)).astype(np.uint8)
    ids, d = O.exact_graph(X, 6)
    for u in (0, 17, 299):
        pairs = O.exact_row(X, u, 6)
        assert [v for _, v in pairs] == ids[u].tolist()
        assert [dd for dd, _ in pairs] == d[u].tolist()


def test_budget_formula():
    # n / speedup rounded up, at least k, at most n
    assert O.budget(2000, 10, 8) == 250
    assert O.budget(2001, 10, 8) == 251
    assert O.budget(100, 10, 50) == 10
    assert O.budget(5, 10, 1) == 5
    assert O.budget(100_000, 10, 1) == 100_000
    assert all(O.budget(n, 3, s) <= n for n in range(1, 50) for s in range(1, 9))


def test_params_validation():
    with pytest.raises(ValueError):
        O.Params(k=0)
    with pytest.raises(ValueError):
        O.Params(k=3, e_num=1, e_den=1)
    with pytest.raises(ValueError):
        O.Params(k=3, speedup=0)
    assert math.isclose(O.Params(k=3, e_num=6, e_den=5).e_num / 5, 1.2)
