"""Pins of the oracle's GNNS baseline (fixed restarts, steepest climb)."""

import numpy as np
import pytest

import oracle as O
from tests.helpers import u8_points


def graph_of(X, k):
    ids, d = O.exact_graph(X, k)
    return O.OracleGraph(X, ids, d, k)


def test_all_restarts_reach_every_node_and_the_exact_result():
    X = u8_points(3, 300, 8, clusters=4)
    g = graph_of(X, 6)
    q = u8_points(4, 1, 8, clusters=4)[0]
    r = O.gnns(g, q, key=77, k=6, restarts=300, seed=1)
    assert r.evals == 300
    assert r.pairs == O.exact_row(X, 0, 6, q=q)


def test_one_dimensional_chain_reaches_the_nearest_point():
    # evenly spaced points on a line with 2-nn lists: every point's list is
    # its two sides, so the steepest climb from anywhere ends at the point
    # nearest to the query
    X = (np.arange(0, 200, 2, dtype=np.int64)[:, None] + 20).astype(np.uint8)
    g = graph_of(X, 2)
    for key in range(40):
        qv = np.array([int(20 + (key * 37) % 198)], dtype=np.uint8)
        r = O.gnns(g, qv, key=key, k=1, restarts=1, seed=5)
        want = min((int(O.sqdist(qv, X[v])), v) for v in range(len(X)))
        assert r.pairs[0] == want


@pytest.mark.parametrize("key", [1, 2, 3])
def test_trace_is_a_steepest_climb(key):
    """Replay the recorded evaluation order: after each restart, nodes come
    in groups = the unvisited entries of the current node's list, and the
    climb moves to each group's best only when it is strictly closer."""
    X = u8_points(5, 400, 16, clusters=5)
    g = graph_of(X, 8)
    q = u8_points(6, 1, 16, clusters=5)[0]
    R = 5
    r = O.gnns(g, q, key=key, k=8, restarts=R, seed=9, record=True)
    seq = r.sequence
    order = O.RestartOrder(len(X), 9, key)
    visited = set()
    i = 0
    for _ in range(R):
        start = order.next_unvisited(visited)
        if start is None:
            break
        assert seq[i] == start
        visited.add(start)
        i += 1
        c, dc = start, int(O.sqdist(q, X[start]))
        while True:
            group = [v for v in g.neighbours(c) if v not in visited]
            assert seq[i:i + len(group)] == group
            visited.update(group)
            i += len(group)
            if not group:
                break
            db, b = min((int(O.sqdist(q, X[v])), v) for v in group)
            if db < dc:
                c, dc = b, db
            else:
                break
    assert i == len(seq) == r.evals


def test_more_restarts_extend_the_sequence():
    X = u8_points(7, 500, 16, clusters=5)
    g = graph_of(X, 10)
    q = u8_points(8, 1, 16, clusters=5)[0]
    prev = []
    for R in range(1, 8):
        s = O.gnns(g, q, key=11, k=10, restarts=R, seed=3, record=True).sequence
        assert s[:len(prev)] == prev and len(s) >= len(prev)
        prev = s


def test_budget_stops_immediately():
    X = u8_points(9, 500, 16, clusters=5)
    g = graph_of(X, 10)
    q = u8_points(10, 1, 16, clusters=5)[0]
    full = O.gnns(g, q, key=4, k=10, restarts=50, seed=3, record=True)
    cut = O.gnns(g, q, key=4, k=10, restarts=50, seed=3, budget=37, record=True)
    assert cut.evals == min(37, full.evals)
    assert cut.sequence == full.sequence[:cut.evals]
