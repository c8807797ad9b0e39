"""Parity of the HIP float path with the oracle (float32 points).

The search decides with bfloat16 / FP8 / float32 scores and stores float32
distances re-computed in one fixed order; the oracle works in float64.
Acceptance, following the method's float reading:
  * every stored distance is within 1e-5 (relative) of the float64 distance
    of its pair (absolute floor for coincident points);
  * list invariants: sorted by (distance, id), distinct, no self, ids in
    range, padding only at the end;
  * results that the method fixes up to near-ties (exact graph, exhaustive
    search) have the same sorted distance sequence as the oracle within
    that tolerance;
  * decisions taken on float32 scores follow the oracle's float64 ones except
    at near-ties: high agreement rates, stated in each test.
Stored scoring rows match the oracle's quantizers bit for bit."""

import sys

import numpy as np
import pytest

import oracle as O
from datagen import float_mixture
from tests.helpers import ensure_library

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


def f32_points(seed, n, dim, clusters=20):
    return float_mixture(seed, clusters, dim).sample(n, seed + 1000).astype(np.float32)


def cfg_for(G, dim, k, capacity, max_batch, score="bf16", speedup=8, e=(5, 1), depth=2,
            seed=0x5EED):
    return G.GraphConfig(dim=dim, k=k, capacity=capacity, max_batch=max_batch, speedup=speedup,
                         expansion_num=e[0], expansion_den=e[1], depth=depth, seed=seed,
                         dtype="f32", score=score)


def d64(X, Q, ids):
    """float64 distances of query rows Q to the rows ids of X (-1: nan)."""
    Xd = X.astype(np.float64)
    Qd = Q.astype(np.float64)
    safe = np.where(ids >= 0, ids, 0)
    diff = Xd[safe] - Qd[:, None, :]
    out = np.einsum("ijk,ijk->ij", diff, diff)
    return np.where(ids >= 0, out, np.nan)


def check_lists(X, ids, d, self_ids=None, n_limit=None):
    """List invariants and the stored-distance error bound."""
    n_limit = X.shape[0] if n_limit is None else n_limit
    m, k = ids.shape
    have = ids >= 0
    # padding only at the end
    assert np.all(have[:, :-1] | ~have[:, 1:])
    assert np.all(ids < n_limit)
    assert np.all(np.isinf(d[~have]))
    for i in range(m):
        row = ids[i][have[i]]
        assert len(set(row.tolist())) == len(row), f"duplicate id in row {i}"
        if self_ids is not None:
            assert self_ids[i] not in row, f"self in row {i}"
        keys = list(zip(d[i][have[i]].tolist(), row.tolist()))
        assert keys == sorted(keys), f"row {i} not sorted by (distance, id)"
    Q = X[self_ids] if self_ids is not None else None
    return Q


def check_error(X, Q, ids, d):
    ref = d64(X, Q, ids)
    have = ids >= 0
    err = np.abs(d.astype(np.float64) - ref)
    bound = REL * ref + 1e-12
    worst = float(np.max(np.where(have, err / np.maximum(ref, 1e-30), 0.0)))
    assert np.all(err[have] <= bound[have]), f"stored distance error above 1e-5 (worst {worst})"
    return worst


def same_sequence(ref_d, got_d):
    """Sorted distance sequences equal within the tolerance, row by row."""
    ok = np.isclose(got_d, ref_d, rtol=2 * REL, atol=1e-12) | (np.isinf(ref_d) & np.isinf(got_d))
    return ok.all(axis=1)


@pytest.mark.parametrize("score,dim", [("bf16", 40), ("fp8", 40), ("exact", 40),
                                       ("bf16", 300), ("fp8", 960), ("bf16m", 40),
                                       ("bf16m", 128)])
def test_ingest_rows_match_quantizers(G, score, dim):
    import torch
    X = f32_points(3, 300, dim) * 7.0
    X[5] = 0.0                                      # a zero row (FP8 scale 0)
    X[6, :4] = [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2 ** -11]   # rounding ties
    say(f"ingest rows score={score} n=300 d={dim}")
    g = G.KnnGraph.build_exact(cfg_for(G, dim, 5, 300, 8, score=score), torch.from_numpy(X).cuda())
    rows, scale = g.rows()
    rows = rows.cpu().numpy()
    if score in ("bf16", "bf16m"):
        coord = -(-2 * dim // 16) * 16
        # rows scored on the matrix cores carry the float32 squared norm of
        # the stored row in a 16-byte chunk
        packed = score == "bf16m"
        assert rows.shape[1] == coord + (16 if packed else 0)
        got = rows[:, :coord].view(np.uint16)[:, :dim]
        bits = O.quantize.bf16_bits(X)
        assert np.array_equal(got, bits)
        assert not rows[:, :coord].view(np.uint16)[:, dim:].any()
        if packed:
            tail = rows[:, coord:].view(np.float32)
            vals = O.quantize.bf16_value(bits).astype(np.float64)
            want = (vals * vals).sum(axis=1)
            assert np.allclose(tail[:, 0], want, rtol=dim * 2.0 ** -23, atol=0)
            assert not tail[:, 1:].any()
    elif score == "fp8":
        codes, s = O.quantize.fp8_rows(X)
        assert rows.shape[1] == -(-dim // 16) * 16
        assert np.array_equal(scale.cpu().numpy(), s)
        assert np.array_equal(rows[:, :dim], codes)
        assert not rows[:, dim:].any()
    else:
        assert np.array_equal(rows.view(np.float32)[:, :dim], X)
    assert np.array_equal(g.points().cpu().numpy(), X)


@pytest.mark.parametrize("n,dim,k,score", [(2500, 128, 20, "bf16"), (1100, 96, 10, "bf16"),
                                           (700, 37, 7, "bf16"), (300, 200, 50, "bf16"),
                                           (600, 960, 50, "fp8"), (900, 300, 20, "bf16"),
                                           (1100, 96, 10, "bf16m")])
def test_exact_graph_float(G, n, dim, k, score):
    import torch
    X = f32_points(11 + dim, n, dim)
    say(f"float exact graph n={n} d={dim} k={k}")
    g = G.KnnGraph.build_exact(cfg_for(G, dim, k, n, 16, score=score), torch.from_numpy(X).cuda())
    ids, d = (t.cpu().numpy() for t in g.lists())
    check_lists(X, ids, d, self_ids=np.arange(n))
    worst = check_error(X, X, ids, d)
    o_ids, o_d = O.exact_graph(X, k)
    seq = same_sequence(o_d, d.astype(np.float64))
    agree = float(np.mean(ids == o_ids))
    say(f"  worst rel err {worst:.2e}  rows with equal distance sequence {seq.mean():.4f}  "
        f"id agreement {agree:.5f}")
    assert seq.all()
    assert agree > 0.999


@pytest.mark.parametrize("score", ["bf16", "fp8", "exact", "bf16m"])
def test_search_float_invariants_and_exhaustive(G, score):
    import torch
    n, dim, k = 3000, 128, 20
    X = f32_points(21, n + 64, dim)
    base, Q = X[:n], X[n:]
    cfg = cfg_for(G, dim, k, n + 64, 64, score=score, speedup=6)
    say(f"float search score={score} n={n}")
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(base).cuda())
    keys = torch.arange(500, 500 + len(Q), dtype=torch.int64)
    ids, d, ev, tr = (t.cpu().numpy() if t is not None else None
                      for t in g.search(torch.from_numpy(Q).cuda(), keys, trace=True))
    B = g.budget()
    assert np.all(ev == B)
    for i in range(len(Q)):
        seq = tr[i][tr[i] >= 0]
        assert len(seq) == B and len(set(seq.tolist())) == B
        assert set(ids[i][ids[i] >= 0].tolist()) <= set(seq.tolist())
    check_lists(np.concatenate([base, Q]), ids, d, n_limit=n)
    check_error(base, Q, ids, d)
    # exhaustive limit: speedup 1 evaluates every node; the re-ranked result
    # is the exact top-k (up to near ties)
    g1 = G.KnnGraph.build_exact(cfg_for(G, dim, k, n + 64, 64, score=score, speedup=1),
                                torch.from_numpy(base).cuda())
    ids1, d1, ev1, _ = g1.search(torch.from_numpy(Q).cuda(), keys)
    ids1, d1 = ids1.cpu().numpy(), d1.cpu().numpy()
    assert np.all(ev1.cpu().numpy() == n)
    rows = O.ExactRows(base, k)
    exact = [rows.row(q) for q in Q]
    ref = np.array([[dd for dd, _ in r] for r in exact])
    seq = same_sequence(ref, d1.astype(np.float64))
    rec = np.mean([len(set(ids1[i].tolist()) & {v for _, v in exact[i]}) / k
                   for i in range(len(Q))])
    say(f"  exhaustive rows equal to exact: {seq.mean():.4f}  recall {rec:.4f}")
    # the kept candidates (2k for bfloat16, 4k for FP8's 3-bit mantissas)
    # contain the exact k nearest
    assert seq.all()


def test_search_float32_scores_follow_oracle(G):
    """float32 scoring decides like the float64 oracle except at near ties."""
    import torch
    n, dim, k = 3000, 64, 10
    X = f32_points(31, n + 200, dim)
    base, Q = X[:n], X[n:]
    cfg = cfg_for(G, dim, k, n + 200, 200, score="exact", speedup=8)
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(base).cuda())
    keys = torch.arange(n, n + len(Q), dtype=torch.int64)
    say("float32 search vs oracle traces")
    ids, d, ev, tr = (t.cpu().numpy() for t in g.search(torch.from_numpy(Q).cuda(), keys, trace=True))
    o_ids, o_d = O.exact_graph(base, k)
    og = O.OracleGraph(base, o_ids, o_d, k)
    p = O.Params(k=k, speedup=8, e_num=5, e_den=1, depth=2, seed=0x5EED)
    same = 0
    for i in range(len(Q)):
        r = O.ignns(og, Q[i], n + i, p, record=True)
        if list(tr[i][tr[i] >= 0]) == r.sequence:
            same += 1
            assert ids[i][ids[i] >= 0].tolist() == [v for _, v in r.pairs]
    say(f"  identical evaluation order: {same}/{len(Q)}")
    assert same >= 0.95 * len(Q)


@pytest.mark.parametrize("score,batches", [("bf16", [256, 100, 1]), ("bf16m", [256, 100, 1]),
                                            ("exact", [256, 77]), ("exact", [1100]),
                                           ("fp8", [128])])
def test_insert_float(G, score, batches):
    import torch
    n0, dim, k = 2000, 96, 10
    total = n0 + sum(batches)
    X = f32_points(41, total, dim)
    cfg = cfg_for(G, dim, k, total, max(batches), score=score, speedup=8)
    say(f"float inserts score={score} batches={batches}")
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(X[:n0]).cuda())
    o_ids, o_d = O.exact_graph(X[:n0], k)
    og = O.OracleGraph(X[:n0].copy(), o_ids, o_d, k)
    p = O.Params(k=k, speedup=8, e_num=5, e_den=1, depth=2, seed=0x5EED)
    at = n0
    for b in batches:
        first, sims = g.insert(torch.from_numpy(X[at:at + b]).cuda())
        assert first == at
        res = O.insert_batch(og, X[at:at + b], p)
        og = res.graph
        at += b
    ids, d = (t.cpu().numpy() for t in g.lists())
    check_lists(X, ids, d, self_ids=np.arange(total))
    worst = check_error(X, X, ids, d)
    agree = float(np.mean(ids == og.ids))
    ex_ids, _ = O.exact_graph(X, k)
    rec = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(ids, ex_ids)]))
    orec = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(og.ids, ex_ids)]))
    say(f"  worst rel err {worst:.2e}  agreement with oracle graph {agree:.4f}  "
        f"recall gpu {rec:.4f} oracle {orec:.4f}")
    if score == "exact":
        assert agree > 0.99
    assert rec > orec - 0.02


def test_query_float(G):
    import torch
    n, dim, k = 2000, 128, 20
    X = f32_points(51, n + 100, dim)
    g = G.KnnGraph.build_exact(cfg_for(G, dim, k, n, 100, speedup=1), torch.from_numpy(X[:n]).cuda())
    say("float query exhaustive")
    ids, d, ev = (t.cpu().numpy() for t in g.query(torch.from_numpy(X[n:]).cuda()))
    assert np.all(ev == n)
    assert g.query_count == 100
    check_lists(X, ids, d, n_limit=n)
    check_error(X[:n], X[n:], ids, d)
    rows = O.ExactRows(X[:n], k)
    ref = np.array([[dd for dd, _ in rows.row(q)] for q in X[n:]])
    assert same_sequence(ref, d.astype(np.float64)).all()


@pytest.mark.parametrize("score,dim,k", [("fp8", 960, 50), ("bf16", 300, 20)])
def test_long_rows_search_and_insert(G, score, dim, k):
    """Rows longer than the register file holds for a whole step (pass
    groups with double-buffered gathers): search invariants, the exhaustive
    limit and batched inserts."""
    import torch
    n, m = 2000, 48
    X = float_mixture(71, 10, dim, lognormal_dim_scale=1.0).sample(n + m + 200, 1071)
    X = X.astype(np.float32)
    base, Q, ins = X[:n], X[n:n + m], X[n + m:]
    say(f"long rows score={score} d={dim} k={k}")
    cfg = cfg_for(G, dim, k, n + 200, 128, score=score, speedup=4)
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(base).cuda())
    keys = torch.arange(900, 900 + m, dtype=torch.int64)
    ids, d, ev, tr = (t.cpu().numpy() for t in g.search(torch.from_numpy(Q).cuda(), keys, trace=True))
    B = g.budget()
    assert np.all(ev == B)
    for i in range(m):
        seq = tr[i][tr[i] >= 0]
        assert len(seq) == B and len(set(seq.tolist())) == B
    check_lists(np.concatenate([base, Q]), ids, d, n_limit=n)
    check_error(base, Q, ids, d)
    g1 = G.KnnGraph.build_exact(cfg_for(G, dim, k, n, 64, score=score, speedup=1),
                                torch.from_numpy(base).cuda())
    ids1, d1, ev1, _ = g1.search(torch.from_numpy(Q).cuda(), keys)
    rows = O.ExactRows(base, k)
    exact = [rows.row(q) for q in Q]
    rec = np.mean([len(set(ids1[i].cpu().numpy().tolist()) & {v for _, v in exact[i]}) / k
                   for i in range(m)])
    say(f"  exhaustive recall {rec:.4f}")
    assert rec >= 0.97
    g.insert(torch.from_numpy(ins[:128]).cuda())
    g.insert(torch.from_numpy(ins[128:]).cuda())
    Xall = np.concatenate([base, ins])
    # the graph's node order is base then the inserted points
    gi, gd = (t.cpu().numpy() for t in g.lists())
    check_lists(Xall, gi, gd, self_ids=np.arange(len(Xall)))
    check_error(Xall, Xall, gi, gd)


@pytest.mark.parametrize("n,dim,speedup,e", [(6000, 96, 6, (3, 2)), (400_000, 16, 100, (5, 4))])
def test_large_launch_equals_small_launches(G, n, dim, speedup, e):
    """Launches of 2,048 searches or more keep the scored positions of a
    restart window across the climb it starts (rows of up to 96 coordinates,
    lists of up to 16 ids), and on graphs whose visited sets live in global
    memory (above ~327k nodes) skip the visited probe of restart candidates
    that an LDS filter of the climbs' evaluations clears; smaller launches
    do neither.  Both must give the same results, evaluation order
    included."""
    import torch
    k, m = 10, 2304
    X = f32_points(81, n + m, dim)
    base, Q = X[:n], X[n:]
    cfg = cfg_for(G, dim, k, n, m, speedup=speedup, e=e)
    say(f"large vs small search launches n={n} m={m}")
    g = G.KnnGraph.build_exact(cfg, torch.from_numpy(base).cuda())
    keys = torch.arange(77, 77 + m, dtype=torch.int64)
    Qd = torch.from_numpy(Q).cuda()
    big = [t.cpu().numpy() for t in g.search(Qd, keys, trace=True)]
    parts = [[t.cpu().numpy() for t in g.search(Qd[i:i + 1000], keys[i:i + 1000], trace=True)]
             for i in range(0, m, 1000)]
    for j in range(4):
        assert np.array_equal(big[j], np.concatenate([p[j] for p in parts])), j
