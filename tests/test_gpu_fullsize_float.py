"""The float workload at its full size (1,000,000 points, d = 128, k = 20,
BF16 scoring): sampled rows of the exact initial graph against the float64
oracle, and one insert batch of 1,024 points in the benchmark's launch
configuration, checked by list invariants and distance error on sampled
rows."""

import sys

import numpy as np
import pytest

import oracle as O
from datagen import get_workload
from tests.helpers import ensure_library

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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


def exact_row64(X64, q, k, exclude=None):
    """k nearest rows of X64 to q by float64 squared distance, (d, id) order."""
    d = np.einsum("ij,ij->i", X64 - q, X64 - q)
    if exclude is not None:
        d[exclude] = np.inf
    idx = np.argpartition(d, k + 8)[:k + 8]
    pairs = sorted((float(d[i]), int(i)) for i in idx)
    return pairs[:k]


def test_full_size_float_graph_and_first_batch(G):
    import torch
    w = get_workload("f32-d128-n1m-b1024")
    n0, b, k = w.n_initial, w.batch, w.k
    say(f"generating {w.name}")
    X = w.mixture().sample(n0 + b, w.stream_seed).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    cfg = G.GraphConfig(dim=w.dim, k=k, capacity=n0 + b, max_batch=b, speedup=w.speedup,
                        expansion_num=w.expansion_num, expansion_den=w.expansion_den,
                        depth=w.depth, seed=w.algo_seed, dtype="f32", score=w.score)
    say("exact graph of 1,000,000 points")
    g = G.KnnGraph.build_exact(cfg, Xd[:n0])
    rng = np.random.default_rng(0)
    sample = rng.choice(n0, size=12, replace=False)
    ids, d = (t.cpu().numpy() for t in g.lists(0, n0))
    X64 = X[:n0].astype(np.float64)
    for u in sample:
        want = exact_row64(X64, X64[u], k, exclude=u)
        got_d = d[u].astype(np.float64)
        ref_d = np.array([dd for dd, _ in want])
        assert np.allclose(got_d, ref_d, rtol=2e-5, atol=1e-9), u
        agree = np.mean(ids[u] == np.array([v for _, v in want]))
        assert agree >= 0.95, (u, agree)
    say("first insert batch of 1,024 points (BF16 scoring, float32 re-rank)")
    first, sims = g.insert(Xd[n0:n0 + b])
    assert first == n0
    ids, d = (t.cpu().numpy() for t in g.lists(0, n0 + b))
    X64 = X.astype(np.float64)
    rows = np.concatenate([n0 + rng.choice(b, size=24, replace=False), sample])
    for u in rows:
        have = ids[u] >= 0
        row = ids[u][have]
        assert len(set(row.tolist())) == len(row) and u not in row and np.all(row < n0 + b)
        keys = list(zip(d[u][have].tolist(), row.tolist()))
        assert keys == sorted(keys)
        diff = X64[row] - X64[u]
        ref = np.einsum("ij,ij->i", diff, diff)
        assert np.all(np.abs(d[u][have] - ref) <= 1e-5 * ref + 1e-12), u
    B = g.budget(n0)
    assert np.all(sims.cpu().numpy() >= B + b - 1)
