"""The serving loop (continuous batching of inserts and queries).

Contract: an epoch's queries answer as knng_query on the snapshot before
the epoch, and its inserts leave the graph as knng_insert_batch of the same
points on that snapshot -- bit for bit; the whole served stream replays in
the oracle, epoch by epoch, to the same lists and query answers."""

import sys

import numpy as np
import pytest

import oracle as O
from datagen import float_mixture
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


def u8_cfg(G, dim, k, cap, mb, speedup=10, depth=2):
    return G.GraphConfig(dim=dim, k=k, capacity=cap, max_batch=mb, speedup=speedup, depth=depth)


@pytest.mark.parametrize("b,m", [(100, 37), (0, 20), (64, 0), (1, 1)])
def test_epoch_equals_alone_u8(G, b, m):
    n0, dim, k = 3000, 64, 10
    X = u8_points(61, n0 + b + m, dim, clusters=6, sigma=10.0)
    cfg = u8_cfg(G, dim, k, n0 + b, 128)
    say(f"epoch vs alone u8 b={b} m={m}")
    ga = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    gb = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    xi = tensor(X[n0:n0 + b]) if b else None
    xq = tensor(X[n0 + b:]) if m else None
    first, _, qi, qd, qe = ga.epoch(xi, xq)
    assert first == n0
    if m:
        bi, bd, be = gb.query(xq)
        assert np.array_equal(qi.cpu().numpy(), bi.cpu().numpy())
        assert np.array_equal(qd.cpu().numpy(), bd.cpu().numpy())
        assert np.array_equal(qe.cpu().numpy(), be.cpu().numpy())
    if b:
        gb.insert(xi)
    assert ga.n == gb.n == n0 + b and ga.query_count == gb.query_count == m
    for a, c in zip(ga.lists(), gb.lists()):
        assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())


def test_epoch_equals_alone_float(G):
    n0, dim, k, b, m = 3000, 96, 10, 200, 50
    X = float_mixture(62, 10, dim).sample(n0 + b + m, 1062).astype(np.float32)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n0 + b, max_batch=256, speedup=8, dtype="f32",
                        score="bf16")
    say("epoch vs alone float")
    ga = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    gb = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    _, _, qi, qd, _ = ga.epoch(tensor(X[n0:n0 + b]), tensor(X[n0 + b:]))
    bi, bd, _ = gb.query(tensor(X[n0 + b:]))
    gb.insert(tensor(X[n0:n0 + b]))
    assert np.array_equal(qi.cpu().numpy(), bi.cpu().numpy())
    assert np.array_equal(qd.cpu().numpy(), bd.cpu().numpy())
    for a, c in zip(ga.lists(), gb.lists()):
        assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())


def test_served_stream_replays_in_oracle(G):
    """Poisson stream of small inserts and queries through the serving loop;
    the epoch log replayed in the oracle gives the same answers and graph."""
    from paper_1602_06819_amd import serve as S
    n0, dim, k = 2000, 16, 10
    reqs = S.make_requests(5, rate=2000.0, count=60, max_insert=40, max_query=12)
    ins_total, q_total = S.stream_totals(reqs)
    X = u8_points(63, n0 + ins_total, dim, clusters=5)
    Q = u8_points(64, q_total, dim, clusters=5)
    cfg = u8_cfg(G, dim, k, n0 + ins_total, 64, speedup=8)
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    say(f"served stream: {len(reqs)} requests, {ins_total} insert / {q_total} query points")
    res = S.serve(g, reqs, tensor(X[n0:]), tensor(Q), max_query_points=24, keep_queries=True)
    summary = res.summary(reqs)
    say(f"  epochs {summary['epochs']} p50 {summary['p50_ms']:.2f} ms p99 {summary['p99_ms']:.2f} ms")
    assert sum(len(e.requests) for e in res.epochs) == len(reqs)
    ids, d = O.exact_graph(X[:n0], k)
    og = O.OracleGraph(X[:n0].copy(), ids, d, k)
    p = O.Params(k=k, speedup=8, e_num=5, e_den=1, depth=2, seed=0x5EED)
    qseq = 0
    for e, out in zip(res.epochs, res.query_out):
        assert e.n_before == og.n
        if e.q_hi > e.q_lo:
            want = O.query(og, Q[e.q_lo:e.q_hi], p, first_seq=qseq)
            qseq += e.q_hi - e.q_lo
            got_ids, got_d = to_oracle_lists(*out)
            for j, r in enumerate(want):
                assert got_ids[j, :len(r.pairs)].tolist() == [v for _, v in r.pairs]
                assert got_d[j, :len(r.pairs)].tolist() == [dd for dd, _ in r.pairs]
        if e.ins_hi > e.ins_lo:
            og = O.insert_batch(og, X[n0 + e.ins_lo:n0 + e.ins_hi], p).graph
    gi, gd = (t.cpu().numpy() for t in g.lists())
    gi, gd = to_oracle_lists(gi, gd)
    assert np.array_equal(gi, og.ids) and np.array_equal(gd, og.dist)
