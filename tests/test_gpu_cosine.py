"""The cosine metric on the GPU against the oracle (float64 normalization,
float64 distances): the graph and search results of cosine similarity equal
the squared-L2 results on normalized points, up to float32 near-ties."""

import sys

import numpy as np
import pytest

import oracle as O
from datagen import float_mixture
from oracle import cosine as C
from tests.helpers import ensure_library

pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 1e-6


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


def points(seed, n, dim):
    X = float_mixture(seed, 12, dim).sample(n, seed + 1000).astype(np.float32)
    # random positive row scales: cosine ignores them
    scale = np.random.default_rng(seed).uniform(0.2, 5.0, size=(n, 1)).astype(np.float32)
    return (X * scale).astype(np.float32)


def cfg(G, dim, k, cap, mb, score="bf16", speedup=6):
    return G.GraphConfig(dim=dim, k=k, capacity=cap, max_batch=mb, speedup=speedup, dtype="f32",
                         score=score, metric="cosine")


def check_error(Xn, Qn, ids, d):
    have = ids >= 0
    safe = np.where(have, ids, 0)
    diff = Xn[safe] - Qn[:, None, :]
    ref = np.einsum("ijk,ijk->ij", diff, diff)
    err = np.abs(d.astype(np.float64) - ref)
    assert np.all(err[have] <= REL * ref[have] + ABS), float(np.max(err[have]))


def test_stored_points_are_normalized(G):
    X = points(1, 500, 40)
    X[7] = 0.0
    g = G.KnnGraph.build_exact(cfg(G, 40, 8, 500, 16), tensor(X))
    P = g.points().cpu().numpy().astype(np.float64)
    assert np.allclose(P, C.normalize(X), rtol=0, atol=2e-7)
    assert np.all(P[7] == 0)


@pytest.mark.parametrize("score", ["bf16", "exact"])
def test_exact_graph_and_exhaustive_search(G, score):
    import torch
    n, dim, k = 2500, 64, 10
    X = points(2, n + 60, dim)
    Xn = C.normalize(X)
    say(f"cosine exact graph + exhaustive search score={score}")
    g = G.KnnGraph.build_exact(cfg(G, dim, k, n, 64, score=score, speedup=1), tensor(X[:n]))
    ids, d = (t.cpu().numpy() for t in g.lists())
    check_error(Xn[:n], Xn[:n], ids, d)
    o_ids, o_d = O.exact_graph(Xn[:n], k)
    agree = float(np.mean(ids == o_ids))
    seq = np.isclose(d.astype(np.float64), o_d, rtol=2 * REL, atol=2 * ABS).all(axis=1)
    say(f"  exact graph id agreement {agree:.5f}, equal distance rows {seq.mean():.4f}")
    assert agree > 0.999 and seq.all()
    keys = torch.arange(n, n + 60, dtype=torch.int64)
    si, sd, ev, _ = g.search(tensor(X[n:]), keys)
    si, sd = si.cpu().numpy(), sd.cpu().numpy()
    assert np.all(ev.cpu().numpy() == n)
    check_error(Xn[:n], Xn[n:], si, sd)
    rows = O.ExactRows(Xn[:n], k)
    ref = np.array([[dd for dd, _ in rows.row(q)] for q in Xn[n:]])
    assert np.isclose(sd.astype(np.float64), ref, rtol=2 * REL, atol=2 * ABS).all()


def test_inserts_follow_oracle_on_normalized_points(G):
    n0, dim, k = 2000, 48, 10
    X = points(3, n0 + 300, dim)
    Xn = C.normalize(X)
    g = G.KnnGraph.build_exact(cfg(G, dim, k, n0 + 300, 256, score="exact", speedup=8),
                               tensor(X[:n0]))
    o_ids, o_d = O.exact_graph(Xn[:n0], k)
    og = O.OracleGraph(Xn[:n0].copy(), o_ids, o_d, k)
    p = O.Params(k=k, speedup=8, e_num=5, e_den=1, depth=2, seed=0x5EED)
    for lo, hi in ((n0, n0 + 256), (n0 + 256, n0 + 300)):
        g.insert(tensor(X[lo:hi]))
        og = O.insert_batch(og, Xn[lo:hi], p).graph
    ids, d = (t.cpu().numpy() for t in g.lists())
    check_error(Xn, Xn, ids, d)
    agree = float(np.mean(ids == og.ids))
    say(f"  cosine inserts: agreement with the oracle graph {agree:.4f}")
    assert agree > 0.98


def test_query_ignores_query_scale(G):
    n, dim, k = 2000, 32, 10
    X = points(4, n + 50, dim)
    g = G.KnnGraph.build_exact(cfg(G, dim, k, n, 64, score="exact", speedup=1), tensor(X[:n]))
    a_ids, _, _ = g.query(tensor(X[n:]))
    b_ids, _, _ = g.query(tensor(X[n:] * np.float32(3.5)))
    assert float(np.mean(a_ids.cpu().numpy() == b_ids.cpu().numpy())) > 0.99
