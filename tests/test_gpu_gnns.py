"""Parity of the GNNS baseline mode of the search kernel with the oracle's
GNNS (uint8 points: bit-exact ids, distances, evaluation counts and order)."""

import sys

import numpy as np
import pytest

import oracle as O
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


@pytest.mark.parametrize("dim,k,restarts,speedup", [(16, 10, 1, 1), (16, 10, 5, 1),
                                                    (64, 10, 20, 1), (64, 10, 200, 8),
                                                    (32, 20, 7, 1), (64, 10, 0, 1)])
def test_gnns_bit_exact(G, dim, k, restarts, speedup):
    import torch
    n = 3000
    X = u8_points(81 + dim, n, dim, clusters=6, sigma=10.0)
    Q = u8_points(82 + dim, 60, dim, clusters=6, sigma=10.0)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, speedup=speedup, seed=4321)
    say(f"gnns d={dim} k={k} R={restarts} speedup={speedup}")
    g = G.KnnGraph.build_exact(cfg, tensor(X))
    keys = torch.arange(10_000, 10_000 + len(Q), dtype=torch.int64)
    ids, d, ev, tr = g.search_gnns(tensor(Q), keys, restarts, trace=True)
    ids, d = to_oracle_lists(ids.cpu().numpy(), d.cpu().numpy())
    ev = ev.cpu().numpy()
    tr = tr.cpu().numpy()
    oi, od = O.exact_graph(X, k)
    og = O.OracleGraph(X, oi, od, k)
    B = g.budget()
    for j in range(len(Q)):
        r = O.gnns(og, Q[j], key=10_000 + j, k=k, restarts=restarts, seed=4321, budget=B,
                   record=True)
        assert ev[j] == r.evals, j
        assert tr[j, :r.evals].tolist() == r.sequence, j
        assert ids[j, :len(r.pairs)].tolist() == [v for _, v in r.pairs], j
        assert d[j, :len(r.pairs)].tolist() == [dd for dd, _ in r.pairs], j


def test_gnns_float32_follows_oracle(G):
    """float32 scoring decides like the float64 oracle except at near ties."""
    import torch
    from datagen import float_mixture
    n, dim, k, R = 3000, 3, 10, 6
    X = float_mixture(83, 10, dim).sample(n + 100, 1083).astype(np.float32)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=100, speedup=1, seed=99,
                        dtype="f32", score="exact")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n]))
    keys = torch.arange(500, 600, dtype=torch.int64)
    ids, d, ev, tr = (t.cpu().numpy() for t in g.search_gnns(tensor(X[n:]), keys, R, trace=True))
    oi, od = O.exact_graph(X[:n], k)
    og = O.OracleGraph(X[:n], oi, od, k)
    same = 0
    for j in range(100):
        r = O.gnns(og, X[n + j], key=500 + j, k=k, restarts=R, seed=99, record=True)
        if tr[j, :ev[j]].tolist() == r.sequence:
            same += 1
    say(f"  float GNNS identical evaluation order: {same}/100")
    assert same >= 95
