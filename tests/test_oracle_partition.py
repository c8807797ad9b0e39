"""Pins of the oracle's balanced k-medoids and partitioned search."""

import numpy as np
import pytest

import oracle as O
from oracle import partition as Pt
from tests.helpers import u8_points


def test_perfect_balance_with_imbalance_one():
    X = u8_points(1, 600, 8, clusters=3)
    for p in (2, 3, 4, 6):
        part, meds = Pt.balanced_kmedoids(X, p, iters=2, seed=5)
        sizes = np.bincount(part, minlength=p)
        assert sizes.tolist() == [600 // p] * p
        assert len(set(meds)) == p


def test_capacity_bounds_sizes_with_imbalance():
    X = u8_points(2, 500, 8, clusters=2)
    part, _ = Pt.balanced_kmedoids(X, 3, iters=2, seed=1, imb_num=6, imb_den=5)
    sizes = np.bincount(part, minlength=3)
    assert sizes.sum() == 500 and sizes.max() <= 500 * 6 / 15


def test_one_cluster_medoid_is_the_brute_force_median():
    X = u8_points(3, 150, 6, clusters=2)
    part, meds = Pt.balanced_kmedoids(X, 1, iters=1, seed=2)
    assert np.all(part == 0)
    D = np.array([[O.sqdist(X[u], X[v]) for v in range(150)] for u in range(150)])
    tot = D.sum(axis=1)
    want = min(range(150), key=lambda u: (tot[u], u))
    assert meds == [want]


def test_separated_blobs_are_recovered():
    # four far-apart blobs of 50 points; one initial medoid in each blob
    rng = np.random.default_rng(4)
    centres = np.array([[30] * 4, [220] * 4, [30, 30, 220, 220], [220, 220, 30, 30]])
    X = np.concatenate([np.clip(c + rng.normal(0, 4, (50, 4)), 0, 255) for c in centres])
    X = np.rint(X).astype(np.uint8)
    part, meds = Pt.balanced_kmedoids(X, 4, iters=3, seed=0, medoids=[0, 50, 100, 150])
    for b in range(4):
        assert np.all(part[50 * b:50 * b + 50] == b)


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
    part, _ = Pt.balanced_kmedoids(X, 4, iters=2, seed=7)
    pe = O.Params(k=8, speedup=1, seed=3)
    r, ev = Pt.partitioned_search(g, part, 4, q, 5, pe)
    assert ev == np.bincount(part, minlength=4).tolist()
    assert r.pairs == O.exact_row(X, 0, 8, q=q)
    # budgets per partition
    ps = O.Params(k=8, speedup=8, seed=3)
    _, ev = Pt.partitioned_search(g, part, 4, q, 5, ps)
    assert ev == [O.budget(int(c), 8, 8) for c in np.bincount(part, minlength=4)]
