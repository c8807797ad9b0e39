"""Parity at the workloads' own sizes, in the launch configurations the
benchmark uses.

* Integer workload (100,000 uint8 points, d = 64, k = 10, depth 4): the whole
  graph after the first four 256-point batches (search, peers, update and
  merge at full size) and 1,000 read-only queries, bit for bit against the
  oracle (its per-point steps run in worker processes).
* FP8 workload (500,000 points, d = 960, k = 50): the first 512-point batch
  through the global-visited-set FP8 matrix-core search; list invariants and
  stored-distance error of the new and the updated lists, and recall of
  sampled searches against the float64 exact lists.
* Serving workload (1,000,000 points, d = 96): the first two epochs of the
  request stream served together equal their queries and inserts run alone
  on each snapshot, bit for bit."""

import math
import multiprocessing as mp
import os
import sys
from collections import deque

import numpy as np
import pytest

import oracle as O
from datagen import get_workload
from datagen.workloads import query_points
from tests.helpers import ensure_library, to_oracle_lists
from tests.test_gpu_parity_f32 import check_error, check_lists

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


def tensor(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


_STATE = {}


def _point(i):
    return O.point_search_and_proposals(_STATE["g"], _STATE["Y"], i, _STATE["p"])


def _query(j):
    return O.ignns(_STATE["g"], _STATE["Y"][j], O.QUERY_KEY_BASE + j, _STATE["p"])


def _pool_map(fn, items, g, Y, p):
    """fn over items in worker processes forked with (g, Y, p) in place."""
    _STATE.update(g=g, Y=Y, p=p)
    procs = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (4 * procs)))


def test_integer_workload_four_batches_whole_graph(G):
    w = get_workload("u8-d64-n100k-b256")
    n0, b, k = w.n_initial, w.batch, w.k
    X = w.points()[:n0 + 4 * b]
    Q = query_points(w, 1000)
    p = O.Params(k=k, speedup=w.speedup, e_num=w.expansion_num, e_den=w.expansion_den,
                 depth=w.depth, seed=w.algo_seed)
    cfg = G.GraphConfig(dim=w.dim, k=k, capacity=n0 + 4 * b, max_batch=max(b, 1000),
                        speedup=w.speedup, expansion_num=w.expansion_num,
                        expansion_den=w.expansion_den, depth=w.depth, seed=w.algo_seed)
    say("integer workload: 100k exact graph, four batches of 256, 1,000 queries on the GPU")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n0]))
    sims = []
    for s in range(4):
        _, sm = g.insert(tensor(X[n0 + s * b:n0 + (s + 1) * b]))
        sims.append(sm.cpu().numpy())
    qi, qd, qe = (t.cpu().numpy() for t in g.query(tensor(Q)))
    gi, gd = to_oracle_lists(*(t.cpu().numpy() for t in g.lists()))
    say("  oracle: exact graph, then the four batches")
    oi, od = O.exact_graph(X[:n0], k)
    og = O.OracleGraph(X[:n0].copy(), oi, od, k)
    for s in range(4):
        Y = X[n0 + s * b:n0 + (s + 1) * b]
        res = O.insert_batch(og, Y, p, run_points=lambda idx: _pool_map(_point, idx, og, Y, p))
        assert res.sims == sims[s].tolist(), f"similarity counts differ in batch {s}"
        og = res.graph
        say(f"  batch {s}: lists of {og.n} nodes")
    assert np.array_equal(gi, og.ids), "graph ids differ from the oracle"
    assert np.array_equal(gd, og.dist), "graph distances differ from the oracle"
    say("  oracle: 1,000 queries")
    want = _pool_map(_query, list(range(len(Q))), og, Q, p)
    for j, r in enumerate(want):
        assert qi[j].tolist() == [v for _, v in r.pairs], f"query {j} differs"
        assert qd[j].tolist() == [d for d, _ in r.pairs]
        assert int(qe[j]) == r.evals


def test_fp8_workload_first_batch(G):
    import torch
    w = get_workload("f32-d960-n500k-b512-fp8")
    n0, b, k = w.n_initial, w.batch, w.k
    say("FP8 workload: generating 500k x 960 points")
    X = w.mixture().sample(n0 + b, w.stream_seed)
    cfg = G.GraphConfig(dim=w.dim, k=k, capacity=n0 + b, max_batch=b, speedup=w.speedup,
                        expansion_num=w.expansion_num, expansion_den=w.expansion_den,
                        depth=w.depth, seed=w.algo_seed, dtype="f32", score="fp8")
    Xd = torch.from_numpy(X).cuda()
    g = G.KnnGraph.build_exact(cfg, Xd[:n0])
    ids0 = g.lists()[0].cpu().numpy()
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(b, 32, replace=False))
    keys = torch.from_numpy((n0 + sample).astype(np.int64))
    say("  sampled searches on the pre-batch graph")
    si, sd, sev, _ = (t.cpu().numpy() if t is not None else None
                      for t in g.search(Xd[n0 + sample], keys))
    assert np.all(sev == g.budget())
    check_lists(X, si, sd, n_limit=n0)
    check_error(X, X[n0 + sample], si, sd)
    say("  the first batch")
    g.insert(Xd[n0:])
    ids, d = (t.cpu().numpy() for t in g.lists())
    check_lists(X, ids[n0:], d[n0:], self_ids=np.arange(n0, n0 + b))
    worst = check_error(X, X[n0:], ids[n0:], d[n0:])
    # pre-batch lists that the batch changed
    changed = np.nonzero((ids[:n0] != ids0).any(axis=1))[0]
    pick = changed[rng.choice(len(changed), min(300, len(changed)), replace=False)]
    check_lists(X, ids[pick], d[pick], self_ids=pick)
    check_error(X, X[pick], ids[pick], d[pick])
    # recall of the sampled searches against the float64 exact lists
    X64 = X[:n0].astype(np.float64)
    hits = 0
    for j, i in enumerate(sample):
        q = X[n0 + i].astype(np.float64)
        dist = np.einsum("ij,ij->i", X64 - q, X64 - q)
        exact = set(np.argpartition(dist, k)[:k].tolist())
        hits += len(exact & set(si[j].tolist()))
    rec = hits / (len(sample) * k)
    say(f"  {len(changed)} pre-batch lists changed; worst new-list error {worst:.2e}; "
        f"search recall@{k} of the sample {rec:.3f}")
    assert len(changed) > 0
    assert rec >= 0.8


def test_serving_workload_two_epochs_alone_vs_mix(G):
    import torch
    import bench
    from paper_1602_06819_amd.serve import Admission, plan_epoch
    w = get_workload("serve-f32-d96-1m-2m")
    n0 = w.n_initial
    steps = bench.serving_steps(1, 50_000)
    adm = Admission(w.batch, 4096)
    pending = deque(steps[0])
    epochs = [plan_epoch(adm.take(pending, math.inf)) for _ in range(2)]
    ins = epochs[-1].ins_hi
    nq = epochs[-1].q_hi
    say(f"serving workload: 1M exact graph, epochs of {[e.ins_hi - e.ins_lo for e in epochs]} "
        f"inserts and {[e.q_hi - e.q_lo for e in epochs]} queries")
    X = w.mixture().sample(n0 + ins, w.stream_seed)
    Q = w.mixture().sample(max(nq, 1), w.query_seed)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    cfg = G.GraphConfig(dim=w.dim, k=w.k, capacity=n0 + ins, max_batch=w.batch,
                        speedup=w.speedup, expansion_num=w.expansion_num,
                        expansion_den=w.expansion_den, depth=w.depth, seed=w.algo_seed,
                        dtype="f32", score=w.score)
    ga = G.KnnGraph.build_exact(cfg, Xd[:n0])
    ids0, d0 = ga.lists()
    gb = G.KnnGraph.load(cfg, Xd[:n0], ids0, d0)
    for e in epochs:
        x = Xd[n0 + e.ins_lo:n0 + e.ins_hi] if e.ins_hi > e.ins_lo else None
        q = Qd[e.q_lo:e.q_hi] if e.q_hi > e.q_lo else None
        _, _, qi, qd, qe = ga.epoch(x, q)
        if q is not None:
            bi, bd, be = gb.query(q)
            assert torch.equal(qi, bi) and torch.equal(qd, bd) and torch.equal(qe, be)
        if x is not None:
            gb.insert(x, sims=False)
    assert ga.n == gb.n == n0 + ins
    for a, c in zip(ga.lists(), gb.lists()):
        assert torch.equal(a, c)
    ids, d = (t.cpu().numpy() for t in ga.lists(n0))
    check_lists(X, ids, d, self_ids=np.arange(n0, n0 + ins))
    worst = check_error(X, X[n0:], ids, d)
    say(f"  served = alone for {len(epochs)} epochs; worst new-list error {worst:.2e}")
