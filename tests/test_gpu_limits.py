"""Limits and edge cases of the HIP path against the oracle: empty calls,
the largest list length and row size of the integer path, graphs filled to
exactly their capacity with batches of exactly max_batch, and the float
search kernels at the top of every row-size range they are chosen for."""

import sys

import numpy as np
import pytest

import oracle as O
from datagen import float_mixture
from tests.helpers import ensure_library, to_oracle_lists, u8_points

pytestmark = pytest.mark.gpu

REL = 1e-5


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


def test_empty_calls_change_nothing(G):
    import torch
    X = u8_points(81, 600, 16)
    cfg = G.GraphConfig(dim=16, k=10, capacity=600, max_batch=64, speedup=5)
    g = G.KnnGraph.build_exact(cfg, tensor(X[:500]))
    before = [a.cpu().numpy() for a in g.lists()]
    first, sims = g.insert(tensor(X[:0]))
    assert first == 500 and sims.numel() == 0 and g.n == 500
    ids, d, ev = g.query(tensor(X[:0]))
    assert ids.shape == (0, 10) and d.shape == (0, 10) and ev.numel() == 0
    assert g.query_count == 0
    ids, d, ev, _ = g.search(tensor(X[:0]), torch.zeros(0, dtype=torch.int64))
    assert ids.shape == (0, 10)
    first, _, qi, _, _ = g.epoch(None, None)
    assert first == 500 and qi is None
    after = [a.cpu().numpy() for a in g.lists()]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    # the next non-empty call behaves as if the empty ones never happened
    og = O.OracleGraph(X[:500].copy(), *O.exact_graph(X[:500], 10), 10)
    p = O.Params(k=10, speedup=5, seed=cfg.seed)
    g.insert(tensor(X[500:540]))
    og = O.insert_batch(og, X[500:540], p).graph
    ids, d = (t.cpu().numpy() for t in g.lists())
    ids, d = to_oracle_lists(ids, d)
    assert np.array_equal(ids, og.ids) and np.array_equal(d, og.dist)


def test_u8_largest_rows_and_lists_to_exact_capacity(G):
    """d = 256 (the longest integer row) and k = 64 (the longest list), with
    batches of exactly max_batch filling the graph to exactly its capacity;
    bit-exact against the oracle, then one more point is refused."""
    from paper_1602_06819_amd._lib import KNNG_ECAPACITY, KnngError
    n0, dim, k, mb = 300, 256, 64, 48
    batches = [mb, 1, mb, 23]
    cap = n0 + sum(batches)
    X = u8_points(82, cap + 1, dim, clusters=4, sigma=14.0)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=cap, max_batch=mb, speedup=4, depth=2)
    say(f"u8 d={dim} k={k} batches={batches} capacity={cap}")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    og = O.OracleGraph(X[:n0].copy(), *O.exact_graph(X[:n0], k), k)
    ids, d = to_oracle_lists(*(t.cpu().numpy() for t in g.lists()))
    assert np.array_equal(ids, og.ids) and np.array_equal(d, og.dist)
    p = O.Params(k=k, speedup=4, depth=2, seed=cfg.seed)
    lo = n0
    for b in batches:
        first, sims = g.insert(tensor(X[lo:lo + b]))
        res = O.insert_batch(og, X[lo:lo + b], p)
        og = res.graph
        assert first == lo
        assert sims.cpu().numpy().tolist() == res.sims
        ids, d = to_oracle_lists(*(t.cpu().numpy() for t in g.lists()))
        assert np.array_equal(ids, og.ids), lo
        assert np.array_equal(d, og.dist), lo
        lo += b
    assert g.n == cap
    with pytest.raises(KnngError) as ei:
        g.insert(tensor(X[cap:cap + 1]))
    assert ei.value.status == KNNG_ECAPACITY
    # queries on the full graph
    Q = u8_points(83, 20, dim, clusters=4, sigma=14.0)
    qi, qd, qe = (t.cpu().numpy() for t in g.query(tensor(Q)))
    for j, r in enumerate(O.query(og, Q, p, first_seq=0)):
        assert qi[j, :len(r.pairs)].tolist() == [v for _, v in r.pairs]
        assert qd[j, :len(r.pairs)].tolist() == [dd for dd, _ in r.pairs]
        assert qe[j] == r.evals


def _d64(X, Q, ids):
    safe = np.where(ids >= 0, ids, 0)
    diff = X.astype(np.float64)[safe] - Q.astype(np.float64)[:, None, :]
    return np.where(ids >= 0, np.einsum("ijk,ijk->ij", diff, diff), np.nan)


# the float search kernels are chosen by row size and list stride; each case
# sits at the top of its row-size range
@pytest.mark.parametrize("score,dim,k", [
    ("exact", 64, 50), ("exact", 128, 50), ("exact", 256, 20), ("exact", 256, 50),
    ("bf16", 128, 50), ("bf16", 256, 10), ("bf16", 512, 20),
    ("fp8", 256, 50), ("fp8", 512, 10), ("fp8", 1024, 20),
    ("bf16m", 32, 20), ("bf16m", 64, 10), ("bf16m", 96, 10), ("bf16m", 128, 50),
])
def test_float_search_at_row_size_limits(G, score, dim, k):
    import torch
    n, m = 1500, 32
    X = float_mixture(84, 8, dim, lognormal_dim_scale=0.5).sample(n + m, 1084).astype(np.float32)
    base, Q = X[:n], X[n:]
    say(f"float search limits score={score} d={dim} k={k}")
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, dtype="f32", score=score,
                        speedup=4)
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(base).cuda())
    keys = torch.arange(700, 700 + m, dtype=torch.int64)
    ids, d, ev, tr = (t.cpu().numpy() for t in g.search(torch.from_numpy(Q).cuda(), keys,
                                                         trace=True))
    B = g.budget()
    assert np.all(ev == B)
    for i in range(m):
        seq = tr[i][tr[i] >= 0]
        assert len(seq) == B and len(set(seq.tolist())) == B
        row = ids[i][ids[i] >= 0]
        assert len(row) == k and set(row.tolist()) <= set(seq.tolist())
        keys_i = list(zip(d[i].tolist(), row.tolist()))
        assert keys_i == sorted(keys_i)
    ref = _d64(base, Q, ids)
    assert np.all(np.abs(d - ref) <= REL * ref + 1e-12)
    # exhaustive limit: every node evaluated, the exact k nearest found
    g1 = G.KnnGraph.build_exact(
        G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, dtype="f32", score=score,
                      speedup=1), torch.from_numpy(base).cuda())
    ids1, _, ev1, _ = g1.search(torch.from_numpy(Q).cuda(), keys)
    assert np.all(ev1.cpu().numpy() == n)
    rows = O.ExactRows(base, k)
    ids1 = ids1.cpu().numpy()
    rec = np.mean([len(set(ids1[i].tolist()) & {v for _, v in rows.row(Q[i])}) / k
                   for i in range(m)])
    say(f"  exhaustive recall {rec:.4f}")
    assert rec >= (0.95 if score == "fp8" else 0.99)
