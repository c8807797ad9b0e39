"""Pins of the oracle's balanced k-medoids and partitioned search.

The update step's medoid follows Section 6: shortest paths in the graph
(here the k-nn graph taken as undirected, edge length = the stored distance
of the pair) within the cluster, by Dijkstra.  It is pinned by a hand-worked
graph on which the path median and the dissimilarity median differ, by the
all-pairs shortest paths of Floyd and Warshall (an independent algorithm) on
random graphs, and by a cluster that the graph splits in two."""

import numpy as np
import pytest

import oracle as O
from oracle import partition as Pt
from tests.helpers import u8_points


def kmedoids(X, p, iters, seed, k=8, **kw):
    ids, d = O.exact_graph(X, k)
    return Pt.balanced_kmedoids(X, ids, d, p, iters, seed, **kw)


def test_perfect_balance_with_imbalance_one():
    X = u8_points(1, 600, 8, clusters=3)
    for p in (2, 3, 4, 6):
        part, meds = kmedoids(X, p, iters=2, seed=5)
        sizes = np.bincount(part, minlength=p)
        assert sizes.tolist() == [600 // p] * p
        assert len(set(meds)) == p


def test_capacity_bounds_sizes_with_imbalance():
    X = u8_points(2, 500, 8, clusters=2)
    part, _ = kmedoids(X, 3, iters=2, seed=1, imb_num=6, imb_den=5)
    sizes = np.bincount(part, minlength=3)
    assert sizes.sum() == 500 and sizes.max() <= 500 * 6 / 15


def test_path_median_differs_from_dissimilarity_median():
    # five points on a line, 0 1 2 3 100, and their exact 2-nn lists:
    #   0: (1,1) (4,2)   1: (1,0) (1,2)   2: (1,1) (1,3)   3: (1,2) (4,1)
    #   4: (9409,3) (9604,2)
    # undirected path lengths: from 0 -> 1, 2, 3, 9412 (sum 9418); from 1 ->
    # 1, 1, 2, 9411 (9415); from 2 -> 2, 1, 1, 9410 (9414); from 3 -> 3, 2, 1,
    # 9409 (9415); from 4 -> 9412, 9411, 9410, 9409 (37642): the path median
    # is 2.  Sums of squared distances: 10014, 9807, 9610, 9423, 38814: the
    # dissimilarity median is 3.
    X = np.array([[0], [1], [2], [3], [100]], dtype=np.uint8)
    ids, d = O.exact_graph(X, 2)
    assert ids.tolist() == [[1, 2], [0, 2], [1, 3], [2, 1], [3, 2]]
    assert d.tolist() == [[1, 4], [1, 1], [1, 1], [1, 4], [9409, 9604]]
    adj = Pt.undirected_edges(ids, d)
    members = [0, 1, 2, 3, 4]
    keys = [Pt.member_path_key(adj, u, members) for u in members]
    assert [kk[1] for kk in keys] == [9418, 9415, 9414, 9415, 37642]
    assert all(kk[0] == 0 for kk in keys)
    assert Pt.update(ids, d, np.zeros(5, np.int64), [0]) == [2]
    sq = [sum(int(O.sqdist(X[u], X[v])) for v in range(5)) for u in range(5)]
    assert sq == [10014, 9807, 9610, 9423, 38814]
    assert int(np.argmin(sq)) == 3


def floyd_warshall(ids, d, members):
    """All-pairs shortest path lengths within `members` (float64 matrix,
    inf where unreachable), from the undirected edge list."""
    idx = {u: i for i, u in enumerate(members)}
    m = len(members)
    D = np.full((m, m), np.inf)
    np.fill_diagonal(D, 0.0)
    n, k = ids.shape
    for u in range(n):
        for j in range(k):
            v = int(ids[u, j])
            if v >= 0 and u in idx and v in idx:
                w = float(d[u, j])
                D[idx[u], idx[v]] = min(D[idx[u], idx[v]], w)
                D[idx[v], idx[u]] = min(D[idx[v], idx[u]], w)
    for t in range(m):
        D = np.minimum(D, D[:, t:t + 1] + D[t:t + 1, :])
    return D


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_update_matches_all_pairs_shortest_paths(seed):
    X = u8_points(20 + seed, 120, 6, clusters=3)
    ids, d = O.exact_graph(X, 4)
    part = np.random.default_rng(seed).integers(0, 3, 120)
    meds = Pt.update(ids, d, part, [0, 1, 2])
    for m in range(3):
        members = [int(u) for u in np.nonzero(part == m)[0]]
        D = floyd_warshall(ids, d, members)
        unreach = np.isinf(D).sum(axis=1)
        tot = np.where(np.isinf(D), 0.0, D).sum(axis=1)
        want = min(zip(unreach.tolist(), tot.tolist(), members))[2]
        assert meds[m] == want
        adj = Pt.undirected_edges(ids, d)
        for i, u in enumerate(members):
            key = Pt.member_path_key(adj, u, members)
            assert key[0] == unreach[i] and key[1] == tot[i]


def test_unreachable_members_decide_first():
    # one cluster whose graph has two components {0, 1, 2} and {3, 4}: every
    # member of the larger component misses 2 members, of the smaller 3
    ids = np.array([[1, 2], [0, 2], [0, 1], [4, -1], [3, -1]])
    d = np.array([[5, 9], [5, 1], [9, 1], [1, 0], [1, 0]])
    keys = [Pt.member_path_key(Pt.undirected_edges(ids, d), u, [0, 1, 2, 3, 4])
            for u in range(5)]
    assert [kk[0] for kk in keys] == [2, 2, 2, 3, 3]
    # paths: 0 -> 5, 6 (11); 1 -> 5, 1 (6); 2 -> 6, 1 (7); 3 -> 1; 4 -> 1
    assert [kk[1] for kk in keys] == [11, 6, 7, 1, 1]
    assert Pt.update(ids, d, np.zeros(5, np.int64), [3]) == [1]


def test_separated_blobs_are_recovered():
    # four far-apart blobs of 50 points; one initial medoid in each blob
    rng = np.random.default_rng(4)
    centres = np.array([[30] * 4, [220] * 4, [30, 30, 220, 220], [220, 220, 30, 30]])
    X = np.concatenate([np.clip(c + rng.normal(0, 4, (50, 4)), 0, 255) for c in centres])
    X = np.rint(X).astype(np.uint8)
    part, meds = kmedoids(X, 4, iters=3, seed=0, medoids=[0, 50, 100, 150])
    for b in range(4):
        assert np.all(part[50 * b:50 * b + 50] == b)
        assert 50 * b <= meds[b] < 50 * b + 50


def test_partitioned_search_special_cases():
    X = u8_points(5, 800, 16, clusters=4)
    ids, d = O.exact_graph(X, 8)
    g = O.OracleGraph(X, ids, d, 8)
    q = u8_points(6, 1, 16, clusters=4)[0]
    # one partition: the plain search
    p1 = O.Params(k=8, speedup=6, seed=3)
    r, ev = Pt.partitioned_search(g, np.zeros(800, np.int64), 1, q, 99, p1)
    base = O.ignns(g, q, 99, p1)
    assert r.pairs == base.pairs and ev == [base.evals]
    # exhaustive per partition: the union covers every node -> exact result
    part, _ = Pt.balanced_kmedoids(X, ids, d, 4, iters=2, seed=7)
    pe = O.Params(k=8, speedup=1, seed=3)
    r, ev = Pt.partitioned_search(g, part, 4, q, 5, pe)
    assert ev == np.bincount(part, minlength=4).tolist()
    assert r.pairs == O.exact_row(X, 0, 8, q=q)
    # budgets per partition
    ps = O.Params(k=8, speedup=8, seed=3)
    _, ev = Pt.partitioned_search(g, part, 4, q, 5, ps)
    assert ev == [O.budget(int(c), 8, 8) for c in np.bincount(part, minlength=4)]
