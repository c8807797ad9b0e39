"""Parity of the HIP path with the oracle on uint8 data: bit-exact ids,
distances, evaluation counts, evaluation order and final graphs.

Every test calls the library through its C ABI (via the Python binding)
and compares with the oracle on the same seeded inputs."""

import sys

import numpy as np
import pytest

import oracle as O
from datagen import get_workload
from tests.helpers import LazyExactGraph, ensure_library, to_oracle_lists, u8_points

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


def cfg_for(G, dim, k, capacity, max_batch, speedup=10, e=(5, 1), depth=2, seed=0x5EED):
    return G.GraphConfig(dim=dim, k=k, capacity=capacity, max_batch=max_batch, speedup=speedup,
                         expansion_num=e[0], expansion_den=e[1], depth=depth, seed=seed)


def gpu_lists(g):
    ids, d = g.lists()
    return to_oracle_lists(ids.cpu().numpy(), d.cpu().numpy())


def oracle_graph(X, k):
    ids, d = O.exact_graph(X, k)
    return O.OracleGraph(X.copy(), ids, d, k)


def tensor(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# ------------------------------------------------------------------ exact graph
@pytest.mark.parametrize("n,dim,k,vals", [
    (2, 16, 10, 256), (5, 16, 10, 256), (40, 16, 10, 3), (300, 64, 10, 4),
    (3000, 16, 10, 256), (2500, 64, 10, 256), (1000, 100, 20, 256), (700, 64, 50, 256),
    (1337, 48, 7, 256), (5000, 64, 1, 2),
])
def test_exact_graph_bit_exact(G, n, dim, k, vals):
    say(f"exact graph n={n} dim={dim} k={k} vals={vals}")
    rng = np.random.default_rng(n + dim + k)
    X = rng.integers(0, vals, (n, dim)).astype(np.uint8)
    g = G.KnnGraph.build_exact(cfg_for(G, dim, k, n + 8, min(64, n + 8)), tensor(X))
    ids, d = gpu_lists(g)
    want_ids, want_d = O.exact_graph(X, k)
    assert np.array_equal(ids, want_ids)
    assert np.array_equal(d, want_d)
    # points round trip
    assert np.array_equal(g.points().cpu().numpy(), X)


def test_exact_graph_full_size_sampled_rows(G):
    """100,000 uint8 points, d = 64, k = 10 (the integer workload's initial
    graph, same launch as the benchmark): sampled rows against brute force."""
    w = get_workload("u8-d64-n100k-b256")
    X = w.points()[: w.n_initial]
    say("exact graph 100k build")
    g = G.KnnGraph.build_exact(cfg_for(G, 64, 10, w.n_initial + w.n_insert, w.batch), tensor(X))
    ids, d = gpu_lists(g)
    rows = O.ExactRows(X, 10)
    rng = np.random.default_rng(0)
    sample = np.concatenate([[0, 1, w.n_initial - 1], rng.integers(0, w.n_initial, 200)])
    for u in sample:
        pairs = rows.row(X[u], exclude=int(u))
        assert ids[u].tolist() == [v for _, v in pairs], u
        assert d[u].tolist() == [dd for dd, _ in pairs], u


# ------------------------------------------------------------------ search
@pytest.mark.parametrize("dim", [16, 64])
@pytest.mark.parametrize("speedup,e", [(1, (5, 1)), (3, (5, 1)), (10, (5, 1)), (10, (6, 5)),
                                       (50, (2, 1)), (1000, (5, 1))])
def test_search_bit_exact_with_trace(G, dim, speedup, e):
    say(f"search dim={dim} speedup={speedup} e={e}")
    X = u8_points(7, 3000, dim, clusters=6)
    k = 10
    og = oracle_graph(X[:2900], k)
    cfg = cfg_for(G, dim, k, 3000, 100, speedup=speedup, e=e, seed=1234)
    import torch
    g = G.KnnGraph.load(cfg, tensor(og.X), torch.from_numpy(og.ids), torch.from_numpy(
        np.where(og.ids < 0, 0x7fffffff, og.dist)))
    Q = X[2900:]
    keys = np.arange(100, dtype=np.int64) * 7919 + 5
    ids, d, ev, tr = g.search(tensor(Q), torch.from_numpy(keys), trace=True)
    ids, d = to_oracle_lists(ids.cpu().numpy(), d.cpu().numpy())
    ev = ev.cpu().numpy()
    tr = tr.cpu().numpy()
    p = O.Params(k=k, speedup=speedup, e_num=e[0], e_den=e[1], seed=1234)
    for j in range(100):
        r = O.ignns(og, Q[j], key=int(keys[j]), p=p, record=True)
        assert ev[j] == r.evals, j
        assert tr[j, : r.evals].tolist() == r.sequence, j
        assert ids[j, : len(r.pairs)].tolist() == [v for _, v in r.pairs], j
        assert d[j, : len(r.pairs)].tolist() == [dd for dd, _ in r.pairs], j


def test_query_uses_query_namespace_and_counter(G):
    X = u8_points(9, 1500, 16)
    og = oracle_graph(X[:1400], 10)
    g = G.KnnGraph.build_exact(cfg_for(G, 16, 10, 1500, 100, speedup=5), tensor(X[:1400]))
    p = O.Params(k=10, speedup=5, seed=0x5EED)
    first = g.query(tensor(X[1400:1430]))
    second = g.query(tensor(X[1430:1500]))
    assert g.query_count == 100
    want = O.query(og, X[1400:1500], p, first_seq=0)
    got_ids = np.concatenate([first[0].cpu().numpy(), second[0].cpu().numpy()])
    got_ev = np.concatenate([first[2].cpu().numpy(), second[2].cpu().numpy()])
    for j, r in enumerate(want):
        assert got_ids[j, : len(r.pairs)].tolist() == [v for _, v in r.pairs]
        assert got_ev[j] == r.evals


# ------------------------------------------------------------------ insertion
def _run_inserts(G, X, n0, batches, k, speedup, e=(5, 1), depth=2, from_gpu_build=True):
    cfg = cfg_for(G, X.shape[1], k, X.shape[0], max(batches), speedup=speedup, e=e, depth=depth)
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    og = oracle_graph(X[:n0], k)
    p = O.Params(k=k, speedup=speedup, e_num=e[0], e_den=e[1], depth=depth, seed=cfg.seed)
    lo = n0
    for b in batches:
        say(f"  batch n={lo} b={b}")
        first, sims = g.insert(tensor(X[lo:lo + b]))
        res = O.insert_batch(og, X[lo:lo + b], p)
        og = res.graph
        assert first == lo
        assert sims.cpu().numpy().tolist() == res.sims
        ids, d = gpu_lists(g)
        assert np.array_equal(ids, og.ids), lo
        assert np.array_equal(d, og.dist), lo
        lo += b
    return g, og


def test_small_workload_sequential_inserts_bit_exact(G):
    """The small integer workload: 2,000 points, d = 16, k = 10, then 200
    points inserted one at a time (batch = 1, the paper's sequential
    insertion)."""
    w = get_workload("u8-d16-n2k-b1")
    X = w.points()
    say("small workload, 200 sequential inserts")
    _run_inserts(G, X, w.n_initial, [1] * w.n_insert, w.k, w.speedup,
                 (w.expansion_num, w.expansion_den), w.depth)


@pytest.mark.parametrize("batches,depth", [([256, 100], 2), ([64, 1, 33], 1), ([17, 200], 2),
                                           ([256, 77], 3), ([1, 5, 1], 3), ([256, 130], 4)])
def test_batched_inserts_bit_exact(G, batches, depth):
    X = u8_points(11, 6000 + sum(batches), 64, clusters=8, sigma=10.0)
    say(f"batched inserts {batches} depth={depth}")
    _run_inserts(G, X, 6000, batches, 10, 12, depth=depth)


def test_large_batch_peers_on_tiles_bit_exact(G):
    """Batches of 1,024 points or more score their peers with the exact
    graph's tiles instead of one wavefront per point: same graph, bit for
    bit."""
    X = u8_points(14, 3000 + 1100, 16, clusters=6, sigma=12.0)
    say("large batch: peers on the exact tiles")
    _run_inserts(G, X, 3000, [1100], 10, 12, depth=2)


def test_batched_inserts_then_queries_k20(G):
    X = u8_points(12, 3200, 32, clusters=4)
    g, og = _run_inserts(G, X, 3000, [128, 72], 20, 6)
    Q = u8_points(13, 40, 32, clusters=4)
    ids, d, ev = g.query(tensor(Q))
    want = O.query(og, Q, O.Params(k=20, speedup=6), first_seq=0)
    ids = ids.cpu().numpy()
    for j, r in enumerate(want):
        assert ids[j].tolist() == [v for _, v in r.pairs]


def test_exhaustive_search_gives_exact_new_lists(G):
    X = u8_points(14, 2300, 16)
    g, _ = _run_inserts(G, X, 2000, [300], 10, 1)
    ids, _ = gpu_lists(g)
    want, _ = O.exact_graph(X, 10)
    assert np.array_equal(ids[2000:], want[2000:])


def test_insert_is_deterministic(G):
    X = u8_points(15, 5300, 64, clusters=8, sigma=10.0)
    outs = []
    for _ in range(2):
        cfg = cfg_for(G, 64, 10, 5300, 300, speedup=10)
        g = G.KnnGraph.build_exact(cfg, tensor(X[:5000]))
        g.insert(tensor(X[5000:5300]))
        outs.append([a.cpu().numpy() for a in g.lists()])
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_full_size_first_batch_sampled_searches(G):
    """The integer workload at full size in the benchmark's launch
    configuration (100,000 points, batch of 256): sampled searches of the
    first batch against the oracle's iGNNS on the exact graph (lists
    computed on demand), and the new nodes' lists of those points."""
    import torch
    w = get_workload("u8-d64-n100k-b256")
    X = w.points()
    n0 = w.n_initial
    cfg = cfg_for(G, 64, w.k, n0 + w.n_insert, w.batch, speedup=w.speedup,
                  e=(w.expansion_num, w.expansion_den), depth=w.depth, seed=w.algo_seed)
    say("full size: build 100k")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    Y = X[n0:n0 + w.batch]
    keys = torch.arange(n0, n0 + w.batch, dtype=torch.int64)
    say("full size: GPU search of the first batch")
    ids, d, ev, tr = g.search(tensor(Y), keys, trace=True)
    ids = ids.cpu().numpy()
    d = d.cpu().numpy()
    ev = ev.cpu().numpy()
    tr = tr.cpu().numpy()
    _, sims = g.insert(tensor(Y))
    new_ids, new_d = gpu_lists(g)
    lazy = LazyExactGraph(X[:n0], w.k)
    p = O.Params(k=w.k, speedup=w.speedup, e_num=w.expansion_num, e_den=w.expansion_den,
                 depth=w.depth, seed=w.algo_seed)
    for i in (0, 101, 255):
        say(f"full size: oracle search of batch point {i}")
        r = O.ignns(lazy, Y[i], key=n0 + i, p=p, record=True)
        assert ev[i] == r.evals
        assert tr[i, : r.evals].tolist() == r.sequence
        assert ids[i].tolist() == [v for _, v in r.pairs]
        assert d[i].tolist() == [dd for dd, _ in r.pairs]
        # the new node's list: search result plus the other batch points
        cand = list(r.pairs) + [(O.sqdist(Y[i], Y[j]), n0 + j) for j in range(w.batch) if j != i]
        cand.sort()
        assert new_ids[n0 + i].tolist() == [v for _, v in cand[: w.k]]
        assert new_d[n0 + i].tolist() == [dd for dd, _ in cand[: w.k]]


def test_errors_leave_graph_unchanged(G):
    from paper_1602_06819_amd._lib import KNNG_ECAPACITY, KnngError
    X = u8_points(16, 600, 16)
    g = G.KnnGraph.build_exact(cfg_for(G, 16, 10, 520, 64), tensor(X[:500]))
    before = [a.cpu().numpy() for a in g.lists()]
    with pytest.raises(KnngError) as ei:
        g.insert(tensor(X[500:530]))          # 500 + 30 > capacity 520
    assert ei.value.status == KNNG_ECAPACITY
    with pytest.raises(KnngError):
        g.insert(tensor(X[500:600]))          # batch above max_batch
    assert g.n == 500
    after = [a.cpu().numpy() for a in g.lists()]
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])


@pytest.mark.parametrize("depth", [5, 6])
def test_deep_update_level_arrays_in_workspace(G, depth):
    """Depths whose level arrays exceed LDS (k^(depth-1) slots) keep them in
    the workspace; results stay bit-exact."""
    X = u8_points(15, 1500 + 40, 16, clusters=3, sigma=14.0)
    say(f"deep update depth={depth}")
    _run_inserts(G, X, 1500, [24, 1, 15], 10, 8, depth=depth)
