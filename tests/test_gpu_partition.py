"""Balanced k-medoids partitioning and partitioned search on the GPU
against the oracle (uint8: bit-exact parts, medoids and search results)."""

import sys

import numpy as np
import pytest

import oracle as O
from oracle import partition as Pt
from tests.helpers import ensure_library, to_oracle_lists, u8_points

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    ensure_library()
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_1602_06819_amd import graph
    return graph


def tensor(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n,dim,p,iters,imb", [(2000, 16, 4, 3, (1, 1)), (1500, 64, 7, 2, (6, 5)),
                                               (700, 32, 1, 1, (1, 1)), (3000, 16, 16, 2, (1, 1))])
def test_partition_bit_exact(G, n, dim, p, iters, imb):
    X = u8_points(91 + p, n, dim, clusters=6, sigma=12.0)
    cfg = G.GraphConfig(dim=dim, k=10, capacity=n, max_batch=16)
    g = G.KnnGraph.build_exact(cfg, tensor(X))
    say(f"partition n={n} p={p} iters={iters} imbalance={imb}")
    part, med = g.partition(p, iters=iters, imbalance=imb, seed=77)
    oi, od = O.exact_graph(X, 10)
    o_part, o_med = Pt.balanced_kmedoids(X, oi, od, p, iters, seed=77, imb_num=imb[0],
                                         imb_den=imb[1])
    assert np.array_equal(part.cpu().numpy(), o_part)
    assert med.cpu().numpy().tolist() == o_med


def test_partition_float_agrees(G):
    from datagen import float_mixture
    n, dim, p = 2000, 24, 5
    X = float_mixture(95, 8, dim).sample(n, 1095).astype(np.float32)
    cfg = G.GraphConfig(dim=dim, k=10, capacity=n, max_batch=16, dtype="f32", score="exact")
    g = G.KnnGraph.build_exact(cfg, tensor(X))
    part, med = g.partition(p, iters=3, seed=5)
    # the oracle on the graph's own stored lists (float32 lengths): its
    # assignments may differ at near ties of the float64 distances
    gi, gd = (t.cpu().numpy() for t in g.lists())
    o_part, o_med = Pt.balanced_kmedoids(X, gi, gd, p, 3, seed=5)
    agree = float(np.mean(part.cpu().numpy() == o_part))
    say(f"  float partition agreement {agree:.4f}")
    assert agree > 0.98
    assert np.bincount(part.cpu().numpy(), minlength=p).tolist() == [n // p] * p


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_medoid_update_by_graph_paths(G, kind):
    """One iteration from given medoids: the assignment, then the medoids the
    update step computes from shortest paths in the graph, against the
    oracle's Dijkstra on the same stored lists (the float32 lengths summed in
    float64 in the same order: equal bits)."""
    from datagen import float_mixture
    n, dim, k, p = 1800, 12, 8, 5
    if kind == "u8":
        X = u8_points(93, n, dim, clusters=5, sigma=14.0)
        cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=16)
    else:
        X = float_mixture(94, 5, dim).sample(n, 1094).astype(np.float32)
        cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=16, dtype="f32",
                            score="exact")
    g = G.KnnGraph.build_exact(cfg, tensor(X))
    part, med = g.partition(p, iters=1, seed=21)
    gi, gd = (t.cpu().numpy() for t in g.lists())
    pn = part.cpu().numpy()
    o_med = Pt.update(gi, gd, pn, Pt.initial_medoids(n, p, 21))
    say(f"medoids by graph paths {kind}: {med.cpu().numpy().tolist()}")
    assert med.cpu().numpy().tolist() == o_med


@pytest.mark.parametrize("p,speedup", [(4, 6), (1, 8), (8, 3), (4, 1)])
def test_partitioned_search_bit_exact(G, p, speedup):
    import torch
    n, dim, k = 3000, 32, 10
    X = u8_points(97, n, dim, clusters=6, sigma=10.0)
    Q = u8_points(98, 80, dim, clusters=6, sigma=10.0)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, speedup=speedup, seed=31)
    g = G.KnnGraph.build_exact(cfg, tensor(X))
    part, _ = g.partition(p, iters=2, seed=3)
    keys = torch.arange(50_000, 50_080, dtype=torch.int64)
    say(f"partitioned search p={p} speedup={speedup}")
    ids, d, ev = g.search_partitioned(tensor(Q), keys, part, p)
    ids, d = to_oracle_lists(ids.cpu().numpy(), d.cpu().numpy())
    ev = ev.cpu().numpy()
    pn = part.cpu().numpy()
    oi, od = O.exact_graph(X, k)
    og = O.OracleGraph(X, oi, od, k)
    prm = O.Params(k=k, speedup=speedup, seed=31)
    for j in range(len(Q)):
        r, evs = Pt.partitioned_search(og, pn, p, Q[j], 50_000 + j, prm)
        assert ev[j] == sum(evs), j
        assert ids[j, :len(r.pairs)].tolist() == [v for _, v in r.pairs], j
        assert d[j, :len(r.pairs)].tolist() == [dd for dd, _ in r.pairs], j


def test_partitioned_search_float_exhaustive(G):
    """float32 scoring: with speedup 1 every part is searched exhaustively,
    so the merged result is the exact top-k."""
    import torch
    from datagen import float_mixture
    n, dim, k, p = 2000, 3, 10, 4
    X = float_mixture(99, 10, dim).sample(n + 40, 1099).astype(np.float32)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, speedup=1, dtype="f32",
                        score="exact")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n]))
    part, _ = g.partition(p, iters=3, seed=1)
    keys = torch.arange(0, 40, dtype=torch.int64)
    ids, d, ev = g.search_partitioned(tensor(X[n:]), keys, part, p)
    assert np.all(ev.cpu().numpy() == n)
    rows = O.ExactRows(X[:n], k)
    ref = np.array([[dd for dd, _ in rows.row(q)] for q in X[n:]])
    assert np.isclose(d.cpu().numpy().astype(np.float64), ref, rtol=2e-5, atol=1e-12).all()
