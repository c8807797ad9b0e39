"""Parameter sweeps of the paper's evaluation (Section 8), run through the
library on the synthetic stand-ins:

  expansion  recall of iGNNS against the expansion coefficient e at a fixed
             speedup (Section 8.2.1: graph of 5,000 points, speedup 50,
             100 queries, 10 repetitions)
  gnns       recall against the number of computed similarities, iGNNS
             (speedup swept) beside GNNS (restarts swept) (Section 8.2.2:
             graph of 5,000 points, e = 5)
  depth      correct edges and similarities of sequential online building
             against the update depth 1..5 (Section 8.3: n = 1,000 initial
             points, n_a = 1,000 added, speedup 20)
  partitions recall of the partitioned search (balanced k-medoids parts,
             each searched with its own budget, k best of the union) against
             the number of parts, beside the plain search (Section 8.4:
             graph of 8,000 points, speedup 4, 100 queries, 10 repetitions)
  quality    the quality Q of the online graph over the insertion of
             n_a = 16,000 points into n = 8,000 (Section 8.5.2, speedup 4;
             one partition)

Each prints one JSON object per measured point.  Ground truth comes from
the library's exhaustive search (speedup 1 evaluates every node) or exact
graph, both pinned against the oracle by the test suite.

    python -m paper_1602_06819_amd.experiments expansion [--workload W]
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _graph_cfg(w, n_cap, max_batch, **kw):
    from .graph import GraphConfig
    is_float = w.kind != "u8"
    base = dict(dim=w.dim, k=w.k, capacity=n_cap, max_batch=max_batch, speedup=w.speedup,
                expansion_num=w.expansion_num, expansion_den=w.expansion_den, depth=w.depth,
                seed=w.algo_seed, dtype="f32" if is_float else "u8",
                score=w.score if is_float else "exact")
    base.update(kw)
    return GraphConfig(**base)


def _e_pair(e: float) -> tuple[int, int]:
    den = 100
    return int(round(e * den)), den


def _recall(ids, gt, k) -> float:
    return float(np.mean([len(set(a[a >= 0].tolist()) & set(b[b >= 0].tolist())) / k
                          for a, b in zip(ids, gt)]))


def _setup_search(w, n, m, rep):
    """Graph of n points and m held-out queries for repetition rep."""
    import torch
    from .graph import KnnGraph
    X = w.mixture().sample(n + m, w.stream_seed + 1000 * rep)
    Xd = torch.from_numpy(X).cuda()
    cfg1 = _graph_cfg(w, n, m, speedup=1)
    g1 = KnnGraph.build_exact(cfg1, Xd[:n])
    keys = torch.arange(n, n + m, dtype=torch.int64)
    gt, _, _, _ = g1.search(Xd[n:], keys)
    ids, d = g1.lists()
    return Xd, ids, d, keys, gt.cpu().numpy()


def run_expansion(w, n, m, speedup, es, reps):
    from .graph import KnnGraph
    for e in es:
        rec = []
        for rep in range(reps):
            Xd, ids, d, keys, gt = _setup_search(w, n, m, rep)
            num, den = _e_pair(e)
            g = KnnGraph.load(_graph_cfg(w, n, m, speedup=speedup, expansion_num=num,
                                         expansion_den=den), Xd[:n], ids, d)
            r, _, ev, _ = g.search(Xd[n:], keys)
            rec.append(_recall(r.cpu().numpy(), gt, w.k))
        yield {"experiment": "expansion", "workload": w.name, "n": n, "queries": m,
               "speedup": speedup, "e": e, "recall": float(np.mean(rec)),
               "recall_std": float(np.std(rec)), "reps": reps}


def run_gnns(w, n, m, e, speedups, restarts, reps):
    from .graph import KnnGraph
    setups = [_setup_search(w, n, m, rep) for rep in range(reps)]
    num, den = _e_pair(e)
    for sp in speedups:
        rec, ev_all = [], []
        for Xd, ids, d, keys, gt in setups:
            g = KnnGraph.load(_graph_cfg(w, n, m, speedup=sp, expansion_num=num,
                                         expansion_den=den), Xd[:n], ids, d)
            r, _, ev, _ = g.search(Xd[n:], keys)
            rec.append(_recall(r.cpu().numpy(), gt, w.k))
            ev_all.append(float(ev.float().mean()))
        yield {"experiment": "gnns", "method": "iGNNS", "workload": w.name, "n": n,
               "speedup": sp, "e": e, "similarities": float(np.mean(ev_all)),
               "recall": float(np.mean(rec))}
    for R in restarts:
        rec, ev_all = [], []
        for Xd, ids, d, keys, gt in setups:
            g = KnnGraph.load(_graph_cfg(w, n, m, speedup=1), Xd[:n], ids, d)
            r, _, ev, _ = g.search_gnns(Xd[n:], keys, R)
            rec.append(_recall(r.cpu().numpy(), gt, w.k))
            ev_all.append(float(ev.float().mean()))
        yield {"experiment": "gnns", "method": "GNNS", "workload": w.name, "n": n,
               "restarts": R, "similarities": float(np.mean(ev_all)),
               "recall": float(np.mean(rec))}


def run_partitions(w, n, m, speedup, parts, reps):
    from .graph import KnnGraph
    for p in parts:
        rec, seq_rec, ev_all = [], [], []
        for rep in range(reps):
            Xd, ids, d, keys, gt = _setup_search(w, n, m, rep)
            g = KnnGraph.load(_graph_cfg(w, n, m, speedup=speedup), Xd[:n], ids, d)
            if p == 1:
                r, _, ev, _ = g.search(Xd[n:], keys)
            else:
                part, _ = g.partition(p, iters=5, seed=rep)
                r, _, ev = g.search_partitioned(Xd[n:], keys, part, p)
            rec.append(_recall(r.cpu().numpy(), gt, w.k))
            ev_all.append(float(ev.float().mean()))
        yield {"experiment": "partitions", "workload": w.name, "n": n, "speedup": speedup,
               "parts": p, "recall": float(np.mean(rec)), "similarities": float(np.mean(ev_all)),
               "reps": reps}


def run_depth(w, n, n_a, speedup, depths):
    import torch
    from . import metrics
    from .graph import KnnGraph
    X = w.mixture().sample(n + n_a, w.stream_seed)
    Xd = torch.from_numpy(X).cuda()
    gx = KnnGraph.build_exact(_graph_cfg(w, n + n_a, 1, speedup=1), Xd)
    exact, _ = gx.lists()
    exact = exact.cpu().numpy()
    for depth in depths:
        g = KnnGraph.build_exact(_graph_cfg(w, n + n_a, 1, speedup=speedup, depth=depth), Xd[:n])
        sims = 0
        for i in range(n_a):
            _, s = g.insert(Xd[n + i:n + i + 1])
            sims += int(s[0])
        ids, _ = g.lists()
        e_c = metrics.correct_edges(ids.cpu().numpy(), exact)
        yield {"experiment": "depth", "workload": w.name, "n": n, "n_a": n_a,
               "speedup": speedup, "depth": depth, "similarities": sims, "correct_edges": e_c,
               "edges": (n + n_a) * w.k, "quality_Q": metrics.quality(e_c, n, n_a, w.k)}


def run_quality(w, n, n_a, speedup, checkpoints, batch):
    import torch
    from . import metrics
    from .graph import KnnGraph
    X = w.mixture().sample(n + n_a, w.stream_seed)
    Xd = torch.from_numpy(X).cuda()
    g = KnnGraph.build_exact(_graph_cfg(w, n + n_a, batch, speedup=speedup), Xd[:n])
    added = 0
    t0 = time.perf_counter()
    for cp in checkpoints:
        while added < cp:
            b = min(batch, cp - added)
            g.insert(Xd[n + added:n + added + b])
            added += b
        gx = KnnGraph.build_exact(_graph_cfg(w, n + added, 1, speedup=1), Xd[:n + added])
        exact, _ = gx.lists()
        ids, _ = g.lists()
        e_c = metrics.correct_edges(ids.cpu().numpy(), exact.cpu().numpy())
        yield {"experiment": "quality", "workload": w.name, "n": n, "n_a": added,
               "speedup": speedup, "batch": batch, "correct_edges": e_c,
               "recall": e_c / ((n + added) * w.k),
               "quality_Q": metrics.quality(e_c, n, added, w.k),
               "seconds": time.perf_counter() - t0}
        gx.close()


def main(argv=None):
    from datagen import get_workload
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["expansion", "gnns", "depth", "quality", "partitions"])
    ap.add_argument("--workload", default="f32-d3-gmm")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--n-add", type=int, default=None)
    ap.add_argument("--queries", type=int, default=100)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--speedup", type=int, default=None)
    ap.add_argument("--parts", default="1,2,4,8,16,32", help="partitions experiment: part counts")
    ap.add_argument("--e", type=float, default=5.0)
    ap.add_argument("--batch", type=int, default=1)
    args = ap.parse_args(argv)
    w = get_workload(args.workload)
    if args.experiment == "expansion":
        it = run_expansion(w, args.n or 5000, args.queries, args.speedup or 50,
                           [1.05, 1.1, 1.2, 1.5, 2.0, 3.0, 5.0, 8.0, 12.0], args.reps)
    elif args.experiment == "gnns":
        it = run_gnns(w, args.n or 5000, args.queries, args.e, [2, 4, 8, 16, 32, 64, 128],
                      [1, 2, 4, 8, 16, 32, 64, 128], args.reps)
    elif args.experiment == "partitions":
        it = run_partitions(w, args.n or 8000, args.queries, args.speedup or 4,
                            [int(v) for v in args.parts.split(",")], args.reps)
    elif args.experiment == "depth":
        it = run_depth(w, args.n or 1000, args.n_add or 1000, args.speedup or 20, [1, 2, 3, 4, 5])
    else:
        n_a = args.n_add or 16000
        it = run_quality(w, args.n or 8000, n_a, args.speedup or 4,
                         [n_a * i // 8 for i in range(1, 9)], args.batch)
    for rec in it:
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    sys.exit(main())
