"""The naive insertion of Section 2.1 (knng_insert_exact): from an exact
graph, inserting batches by comparing every new point with every node gives
the exact graph of all points -- bit for bit against the oracle's brute
force for uint8 points, and the float64 exact graph's distance sequence
(within the float tolerance) for float32 points."""

import sys

import numpy as np
import pytest

import oracle as O
from tests.helpers import ensure_library, to_oracle_lists, u8_points
from tests.test_gpu_parity_f32 import check_error, check_lists, f32_points, same_sequence

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


# (n0, dim, k, batches): small and ragged batches, k_pad 16 / 32 / 64, a
# batch of one, and a graph of more than 32,768 pre-batch nodes (the
# pre-batch nodes are merged in several chunks)
@pytest.mark.parametrize("n0,dim,k,batches", [
    (3000, 64, 10, [500, 37, 1, 300]),
    (2000, 32, 20, [129, 64]),
    (1500, 16, 40, [200, 3]),
    (40000, 16, 10, [256, 1000]),
])
def test_insert_exact_u8_bit_exact(G, n0, dim, k, batches):
    total = n0 + sum(batches)
    X = u8_points(141 + k, total, dim, clusters=7, sigma=12.0)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=total, max_batch=max(batches))
    say(f"naive insertion u8 n0={n0} d={dim} k={k} batches={batches}")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    lo = n0
    for b in batches:
        assert g.insert_exact(tensor(X[lo:lo + b])) == lo
        lo += b
    assert g.n == total
    got_ids, got_d = to_oracle_lists(*(t.cpu().numpy() for t in g.lists()))
    want_ids, want_d = O.exact_graph(X, k)
    assert np.array_equal(got_ids, want_ids)
    assert np.array_equal(got_d, want_d)


@pytest.mark.parametrize("score", ["exact", "bf16"])
def test_insert_exact_float(G, score):
    import torch
    n0, dim, k, batches = 5000, 96, 10, [700, 1, 333]
    total = n0 + sum(batches)
    X = f32_points(151, total, dim)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=total, max_batch=700, dtype="f32", score=score)
    say(f"naive insertion float score={score}")
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(X[:n0]).cuda())
    lo = n0
    for b in batches:
        g.insert_exact(torch.from_numpy(X[lo:lo + b]).cuda())
        lo += b
    ids, d = (t.cpu().numpy() for t in g.lists())
    check_lists(X, ids, d, self_ids=np.arange(total))
    worst = check_error(X, X, ids, d)
    o_ids, o_d = O.exact_graph(X, k)
    seq = same_sequence(o_d, d.astype(np.float64))
    agree = float(np.mean(ids == o_ids))
    say(f"  worst rel err {worst:.2e}  rows with the exact distance sequence {seq.mean():.4f}  "
        f"id agreement {agree:.5f}")
    assert seq.all()
    assert agree > 0.999


def test_insert_exact_limits(G):
    from paper_1602_06819_amd import _lib
    X = u8_points(161, 600, 16)
    cfg = G.GraphConfig(dim=16, k=5, capacity=520, max_batch=64)
    g = G.KnnGraph.build_exact(cfg, tensor(X[:500]))
    assert g.insert_exact(tensor(X[:0])) == 500          # empty batch: nothing to do
    with pytest.raises(_lib.KnngError):
        g.insert_exact(tensor(X[500:565]))               # above max_batch
    with pytest.raises(_lib.KnngError):
        g.insert_exact(tensor(X[500:530]))               # above capacity
    assert g.n == 500
