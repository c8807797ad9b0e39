"""Benchmark of online k-nn graph building on one MI355X.

Default workload (``serve-f32-d96-1m-2m``): a served k-nn graph that grows
from 1,000,000 to 2,000,000 float32 points (d = 96, 2,000 mixture
components, k = 10, bfloat16 candidate scoring with a float32 re-rank).
The exact initial graph is built by brute force; then a request stream --
Poisson arrivals, three insert requests of 1..4,096 points to one query
request of 1..512 points, log-uniform sizes -- is served in epochs: each
epoch admits the waiting requests first come, first served within the
epoch limits (insert points, query points), searches its inserts and
queries in one launch on the snapshot before the epoch, then runs the
inserts' update and merge (Algorithms 1-2 in batch form).  Epochs are
enqueued back to back on one stream with no host synchronisation between
them.

A step admits 50,000 inserted points (with the queries that arrive among
them; a request that crosses a step boundary is split there), so the
default 20 steps grow the graph to exactly 2,000,000 nodes.  Every input is
resident in GPU memory before the timed region.  `value` is inserted points
per second over the K timed steps (bracketed by device synchronisation);
p50/p99 are the epochs' (batches') GPU latencies.  The report also carries
recall@k of the final graph against its exact graph (all edges, new nodes,
old nodes), query throughput inside the mix, similarity evaluations per
insert, the search kernel's fraction of the HBM roofline (algorithmic bytes
over its measured time), the plain per-point (batch = 1) insertion rate on
the same GPU, the naive exact insertion of Section 2.1 (every new point
compared with every node, brute-force tiles) on the same inserts, a
search-only comparison of bfloat16 and float32 ("FP32 plain") scoring, and
the CPU oracle timed on a bounded sample with one process and with one
process per host core.

The other workloads (``--workload u8-d64-n100k-b256``, ``f32-d128-n1m-b1024``,
``f32-d960-n500k-b512-fp8``) time fixed-size insert batches (one batch per
step) the same way.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 2] [--workload NAME]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "inserts/sec at recall@k>=0.95 vs exact graph; p50/p99 batch latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="serve-f32-d96-1m-2m")
    ap.add_argument("--speedup", type=int, default=None, help="override the search speedup")
    ap.add_argument("--depth", type=int, default=None, help="override the update depth")
    ap.add_argument("--expansion", default=None, help="override e as num/den, e.g. 5/1")
    ap.add_argument("--score", default=None, choices=["exact", "bf16", "bf16m", "fp8"],
                    help="override the scoring rows of a float workload")
    ap.add_argument("--step-inserts", type=int, default=50_000,
                    help="serving: inserted points admitted per step")
    ap.add_argument("--epoch-inserts", type=int, default=None,
                    help="serving: insert points per epoch (default: the workload's batch)")
    ap.add_argument("--epoch-queries", type=int, default=4096,
                    help="serving: query points per epoch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="points of the first batch the CPU oracle inserts (batch workloads)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="serving: CPU time per oracle leg (one process; one per core)")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="serving: oracle worker processes (at most the host's cores)")
    ap.add_argument("--per-point", type=int, default=256,
                    help="points inserted one at a time for the batch=1 baseline")
    ap.add_argument("--no-naive", action="store_true",
                    help="skip the naive exact insertion baseline (Section 2.1)")
    ap.add_argument("--plain-compare", type=int, default=4096,
                    help="serving: points searched with bfloat16 and float32 scoring")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


def search_algorithmic_bytes(score: str, dim: int, k: int, points: int, evals: float,
                             lists: float) -> float:
    """Bytes the searches of `points` points must move: every evaluated
    point's scoring row (int8: d; bfloat16: 2d, plus the 4-byte row norm
    when scored on the matrix cores; FP8: d codes + a 4-byte scale; float32:
    4d), every adjacency list read by the climb (k ids), the
    query row and the k (id, distance) output; float graphs also read the
    float32 rows of the kept candidates for the re-rank.  `score` is "u8"
    for integer graphs, else the float scoring format."""
    is_float = score != "u8"
    v_bytes = {"u8": dim, "bf16": 2 * dim, "bf16m": 2 * dim + 4, "fp8": dim + 4,
               "exact": 4 * dim}[score]
    q_bytes = 4 * dim if is_float else dim
    # candidates the reduced-precision scores keep for the float32 re-rank
    mult = {"bf16": 2, "bf16m": 2, "fp8": 4}.get(score, 1)
    keep = min(mult * k, 128 if k > 16 else 64) if mult > 1 else k
    total = evals * v_bytes + lists * k * 4 + points * (q_bytes + k * 8)
    if is_float:
        total += points * keep * 4 * dim
    return total


def recorded_traffic(grid_threads: int):
    """HBM bytes per search launch (int8 rows) from the committed counter
    record, or None if there is none or it was taken on a different kernel
    source."""
    from paper_1602_06819_amd import profsum
    path = os.path.join(ROOT, "profiles", "traffic_k_search_i8.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != profsum.search_kernel_hash():
        return None
    rows = rec.get("per_grid_kib_per_dispatch", {})
    fetch = rows.get("FETCH_SIZE", {}).get(str(grid_threads))
    write = rows.get("WRITE_SIZE", {}).get(str(grid_threads))
    if fetch is None or write is None or not rec.get("fetch_scale") or not rec.get("write_scale"):
        return None
    return 1024.0 * (fetch * rec["fetch_scale"] + write * rec["write_scale"])


def cpu_baseline(w, X, params, sample: int):
    """The oracle as it stands, on the host cores: its exact initial graph,
    then insert_batch of the first `sample` points of the first batch."""
    import oracle as O
    n0 = w.n_initial
    t0 = time.perf_counter()
    ids, d = O.exact_graph(X[:n0], w.k)
    t_exact = time.perf_counter() - t0
    g = O.OracleGraph(X[:n0].copy(), ids, d, w.k)
    Y = X[n0:n0 + sample]
    t0 = time.perf_counter()
    O.insert_batch(g, Y, params)
    t_ins = time.perf_counter() - t0
    import torch
    return {
        "value": sample / t_ins,
        "unit": "inserts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle insert_batch of the first {sample} points of the first batch "
                   f"(batch semantics, b={sample}) on the {n0}-point snapshot; the oracle's "
                   f"exact initial graph took {t_exact:.1f} s on {torch.get_num_threads()} "
                   f"threads (not counted)"),
        "seconds": t_ins,
        "exact_graph_seconds": t_exact,
        "host_cpus": os.cpu_count(),
    }


def load_workload(args):
    from datagen import get_workload
    w = get_workload(args.workload)
    if args.depth is not None:
        w = w.scaled(depth=args.depth)
    if args.expansion is not None:
        num, den = (int(v) for v in args.expansion.split("/"))
        w = w.scaled(expansion_num=num, expansion_den=den)
    if args.score is not None:
        w = w.scaled(score=args.score)
    if args.speedup is not None:
        w = w.scaled(speedup=args.speedup)
    return w


def bench_batches(args, w) -> dict:
    """Fixed-size insert batches (one per step), then read-only queries."""
    import torch

    from paper_1602_06819_amd import metrics
    from paper_1602_06819_amd.graph import GraphConfig, KnnGraph

    speedup = w.speedup
    n0, b = w.n_initial, w.batch
    max_steps = len(w.batches())
    K = min(args.steps, max_steps)
    W = args.warmup
    dev = torch.device("cuda:0")

    log(f"[bench] generating {w.name}")
    X = w.points()
    Qpts = w.queries() if w.n_query else None
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Qpts).to(dev) if Qpts is not None else None
    is_float = w.kind != "u8"
    gdt = "f32" if is_float else "u8"
    cfg = GraphConfig(dim=w.dim, k=w.k, capacity=n0 + K * b, max_batch=max(b, w.n_query or 0),
                      speedup=speedup, expansion_num=w.expansion_num,
                      expansion_den=w.expansion_den, depth=w.depth, seed=w.algo_seed,
                      dtype=gdt, score=w.score if is_float else "exact")

    # ---- exact initial graph (timed on its own) ----------------------------
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g = KnnGraph.build_exact(cfg, Xd[:n0])
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    log(f"[bench] exact initial graph of {n0} points: {build_ms:.1f} ms")

    # ---- warmup on a separate graph -------------------------------------------
    if W > 0:
        gw = KnnGraph.build_exact(cfg, Xd[:n0])
        for s in range(min(W, K)):
            gw.insert(Xd[n0 + s * b:n0 + (s + 1) * b])
        torch.cuda.synchronize()
        gw.close()
        del gw
        log(f"[bench] {W} warmup steps done")
    if is_float:
        log("[bench] float batch workload: the CPU oracle leg is not run (its float64 exact "
            "initial graph of this size does not fit a bounded sample)")

    # ---- timed steps ---------------------------------------------------------
    stats = []
    lat_events = []
    g.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        _, sims, st = g.insert(Xd[n0 + s * b:n0 + (s + 1) * b], stats=True)
        z.record()
        lat_events.append((a, z))
        stats.append((sims, st))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage = g.timing_read()
    g.timing(False)
    elapsed = t1 - t0
    inserts = K * b
    value = inserts / elapsed
    lat = np.array([a.elapsed_time(z) for a, z in lat_events])
    sims = np.concatenate([x[0].cpu().numpy() for x in stats]).astype(np.float64)
    st = np.concatenate([x[1].cpu().numpy() for x in stats]).astype(np.float64)
    log(f"[bench] {K} steps: {value:.0f} inserts/s, {1000 * elapsed / K:.3f} ms/step")

    # ---- roofline of the search kernel (dominant) ----------------------------
    search_ms, search_launches = stage["search"]
    search_bytes = search_algorithmic_bytes("u8" if not is_float else w.score, w.dim, w.k,
                                            inserts, st[:, 0].sum(), st[:, 1].sum())
    search_avg_ms = search_ms / max(search_launches, 1)
    bytes_per_launch = search_bytes / max(search_launches, 1)
    achieved = bytes_per_launch / (search_avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": None if is_float else recorded_traffic(b * 64),
                "kernel": f"k_search ({'int8' if not is_float else w.score} rows)",
                "avg_launch_ms": search_avg_ms,
                "algorithmic_bytes_per_launch": bytes_per_launch}

    # ---- queries on the final graph -------------------------------------------
    qps = None
    q_stats = {}
    if Qd is not None:
        g.timing(True)
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        qids, qd, qev, qlr = g.query(Qd, list_reads=True)
        torch.cuda.synchronize()
        tq = time.perf_counter() - tq0
        qstage = g.timing_read()
        g.timing(False)
        qps = Qd.shape[0] / tq
        q_stats = {"queries": int(Qd.shape[0]), "queries_per_s": qps,
                   "query_kernel_ms": qstage["query"][0],
                   "evals_per_query": float(qev.float().mean())}
        log(f"[bench] {Qd.shape[0]} queries: {qps:.0f} queries/s")

    # ---- recall of the final graph against its exact graph ---------------------
    rec = {}
    if not args.no_recall:
        n_final = n0 + inserts
        ids_online, _ = g.lists()
        # the exact graph is built from the float32 rows whatever the scoring
        # format; float32 scoring rows exist up to d = 256
        gt_score = "exact" if not is_float or w.dim <= 256 else w.score
        cfg_x = GraphConfig(dim=w.dim, k=w.k, capacity=n_final, max_batch=b, speedup=speedup,
                            dtype=gdt, score=gt_score)
        gx = KnnGraph.build_exact(cfg_x, Xd[:n_final])
        ids_exact, _ = gx.lists()
        io = ids_online.cpu().numpy()
        ie = ids_exact.cpu().numpy()
        gx.close()
        del gx
        e_c = metrics.correct_edges(io, ie)
        rec = {"recall_at_k": e_c / (n_final * w.k),
               "recall_new_nodes": metrics.recall(io[n0:], ie[n0:]),
               "quality_Q": metrics.quality(e_c, n0, inserts, w.k)}
        log(f"[bench] recall@{w.k} {rec['recall_at_k']:.4f} (new nodes "
            f"{rec['recall_new_nodes']:.4f}), Q {rec['quality_Q']:.4f}")

    # ---- plain per-point insertion (b = 1) on the same GPU -------------------------
    per_point = None
    if args.per_point > 0:
        gp = KnnGraph.build_exact(cfg, Xd[:n0])
        P = min(args.per_point, inserts)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for i in range(P):
            gp.insert(Xd[n0 + i:n0 + i + 1], sims=False)
        torch.cuda.synchronize()
        per_point = P / (time.perf_counter() - tp0)
        gp.close()
        del gp
        log(f"[bench] per-point insertion (b=1): {per_point:.0f} inserts/s")

    # ---- the naive method (Section 2.1) on the same GPU: the same batches -----------
    naive = None
    if not args.no_naive:
        gw = KnnGraph.build_exact(cfg, Xd[:n0])      # untimed warmup batch
        gw.insert_exact(Xd[n0:n0 + b])
        gw.close()
        del gw
        gn = KnnGraph.build_exact(cfg, Xd[:n0])
        torch.cuda.synchronize()
        tn0 = time.perf_counter()
        for s in range(K):
            gn.insert_exact(Xd[n0 + s * b:n0 + (s + 1) * b])
        torch.cuda.synchronize()
        naive = inserts / (time.perf_counter() - tn0)
        gn.close()
        del gn
        log(f"[bench] naive exact insertion (brute force, batches of {b}): {naive:.0f} inserts/s")

    # ---- calibration copy for the HBM byte counters ----------------------------------
    if args.calibrate_copy > 0:
        calibration_copy(args.calibrate_copy, dev)

    # ---- CPU oracle baseline -----------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline and not is_float:
        import oracle as O
        params = O.Params(k=w.k, speedup=speedup, e_num=w.expansion_num, e_den=w.expansion_den,
                          depth=w.depth, seed=w.algo_seed)
        log("[bench] timing the CPU oracle (exact initial graph, then a sample of inserts)")
        cpu = cpu_baseline(w, X, params, args.cpu_sample)
        log(f"[bench] CPU oracle: {cpu['value']:.2f} inserts/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "inserts/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if not is_float else {"bf16": "bf16", "bf16m": "bf16", "fp8": "fp8",
                                               "exact": "f32"}[w.score],
        "data": "synthetic",
        "config": {"workload": w.name, "n_initial": n0, "dim": w.dim, "k": w.k, "batch": b,
                   "inserts": inserts, "speedup": speedup,
                   "expansion": f"{w.expansion_num}/{w.expansion_den}", "depth": w.depth,
                   "mixture_clusters": w.n_clusters},
        "p50_batch_ms": float(np.percentile(lat, 50)),
        "p99_batch_ms": float(np.percentile(lat, 99)),
        **rec,
        **q_stats,
        "sims_per_insert": float(sims.mean()),
        "search_evals_per_insert": float(st[:, 0].mean()),
        "lists_read_per_insert": float(st[:, 1].mean()),
        "update_evals_per_insert": float(st[:, 2].mean()),
        "budget": g.budget(n0),
        "build_exact_ms": build_ms,
        "stage_ms": {k: round(v[0], 3) for k, v in stage.items() if v[1]},
        "per_point_inserts_per_s": per_point,
        "naive_exact_inserts_per_s": naive,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    return out


# ---- serving workload ----------------------------------------------------------------

SERVE_REQUEST_SEED = 2024


def serving_steps(steps: int, step_inserts: int, seed: int = SERVE_REQUEST_SEED) -> list:
    """The request stream cut into `steps` steps of exactly `step_inserts`
    insert points each (an insert request crossing a boundary is split
    there; query requests stay where they arrive)."""
    from paper_1602_06819_amd.serve import Request, make_requests
    need = steps * step_inserts
    count = 1024
    while True:
        reqs = make_requests(seed, rate=1.0, count=count)
        if sum(r.size for r in reqs if r.kind == "insert") >= need:
            break
        count *= 2
    out = [[] for _ in range(steps)]
    s = filled = 0
    for r in reqs:
        if s >= steps:
            break
        if r.kind == "query":
            out[s].append(r)
            continue
        size, off = r.size, r.offset
        while size > 0 and s < steps:
            take = min(size, step_inserts - filled)
            out[s].append(Request(r.rid, "insert", take, r.arrival, off))
            off += take
            size -= take
            filled += take
            if filled == step_inserts:
                s += 1
                filled = 0
    return out


def run_steps(g, steps, Xins, Qd, adm, with_events: bool, with_stats: bool):
    """Serve the steps' requests on g: epochs admitted FIFO within the limits,
    enqueued back to back (no host synchronisation).  Returns per-epoch
    records (events, inserts, queries, stats)."""
    import math
    from collections import deque

    import torch

    from paper_1602_06819_amd.serve import plan_epoch
    recs = []
    for reqs in steps:
        pending = deque(reqs)
        while pending:
            ep = plan_epoch(adm.take(pending, math.inf))
            x = Xins[ep.ins_lo:ep.ins_hi] if ep.ins_hi > ep.ins_lo else None
            q = Qd[ep.q_lo:ep.q_hi] if ep.q_hi > ep.q_lo else None
            a = z = None
            if with_events:
                a = torch.cuda.Event(enable_timing=True)
                a.record()
            res = g.epoch(x, q, stats=with_stats)
            if with_events:
                z = torch.cuda.Event(enable_timing=True)
                z.record()
            recs.append((a, z, ep.ins_hi - ep.ins_lo, ep.q_hi - ep.q_lo, res))
    return recs


def exact_topk_f64(Q, D, k: int) -> np.ndarray:
    """Exact k nearest rows of D for every row of Q (float64 on the GPU, for
    measuring search recall)."""
    import torch
    Dd = D.double()
    dn = (Dd * Dd).sum(1)
    out = []
    for i in range(0, Q.shape[0], 256):
        q = Q[i:i + 256].double()
        dist = (q * q).sum(1, keepdim=True) - 2.0 * (q @ Dd.T) + dn[None]
        out.append(torch.topk(dist, k, largest=False).indices.cpu())
    return torch.cat(out).numpy()


_CPU = {}


def _oracle_points(lo_hi):
    """Worker: steps (i) and (iii) of the oracle for batch points [lo, hi)
    until the time budget is spent; returns (points done, proposals)."""
    import oracle as O
    lo, hi = lo_hi
    g, Y, p, budget_s = _CPU["g"], _CPU["Y"], _CPU["p"], _CPU["seconds"]
    t0 = time.perf_counter()
    done, props = 0, []
    for i in range(lo, hi):
        _, pr, _ = O.point_search_and_proposals(g, Y, i, p)
        props.extend(pr)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    return done, props


def _oracle_finish(g, Y, n0: int, k: int, idx: list, props: list, t_start: float):
    """Steps (ii) peers among the points done and (iv) merge of their
    proposals; returns (points, seconds since t_start)."""
    import oracle as O
    for i in idx:
        sorted([(O.sqdist(Y[i], Y[j]), n0 + j) for j in idx if j != i])[:k]
    O.merge_proposals(g, props, k)
    return len(idx), time.perf_counter() - t_start


def cpu_baseline_serving(w, X, labels, seconds: float, procs: int) -> dict:
    """The oracle as it stands inserting the first points of the first epoch
    as one batch (batch semantics) into the exact initial graph, whose lists
    it computes on first use (LazyExactGraph, grouped by mixture component).
    Timed with one process and with `procs` processes (one per core), each
    for about `seconds` of work: steps (i) search and (iii) update proposals
    run per point in the workers, (ii) peers and (iv) merge in the parent."""
    import multiprocessing as mp

    import oracle as O
    n0 = w.n_initial
    procs = max(1, min(procs, os.cpu_count() or 1))
    t0 = time.perf_counter()
    g = O.LazyExactGraph(X[:n0], w.k, labels[:n0])
    t_setup = time.perf_counter() - t0
    p = O.Params(k=w.k, speedup=w.speedup, e_num=w.expansion_num, e_den=w.expansion_den,
                 depth=w.depth, seed=w.algo_seed)
    Y = X[n0:n0 + 64 * procs]
    _CPU.update(g=g, Y=Y, p=p, seconds=seconds)
    shares = [(64 * j, 64 * j + 64) for j in range(procs)]
    # the workers are forked before the parent computes any list
    pool = mp.get_context("fork").Pool(procs)
    try:
        t1 = time.perf_counter()
        d1, pr1 = _oracle_points((0, 64))
        m1, s1 = _oracle_finish(g, Y, n0, w.k, list(range(d1)), pr1, t1)
        t2 = time.perf_counter()
        res = pool.map(_oracle_points, shares)
        idx = [lo + i for (lo, _), (d, _) in zip(shares, res) for i in range(d)]
        props = [pr for _, prs in res for pr in prs]
        m2, s2 = _oracle_finish(g, Y, n0, w.k, idx, props, t2)
    finally:
        pool.close()
        pool.join()
    return {
        "value": m2 / s2,
        "unit": "inserts/s",
        "cores": procs,
        "kind": "oracle",
        "sample": (f"oracle steps (i)-(iv) for the first points of the first epoch as one batch "
                   f"on the exact {n0}-point snapshot (lists computed on first use): {procs} "
                   f"processes x ~{seconds:.0f} s inserted {m2} points in {s2:.1f} s; one "
                   f"process inserted {m1} in {s1:.1f} s ({m1 / s1:.2f} inserts/s); snapshot "
                   f"set-up {t_setup:.1f} s not counted"),
        "single_process_value": m1 / s1,
        "seconds": s2,
        "host_cpus": os.cpu_count(),
    }


def bench_serving(args, w) -> dict:
    """The serving workload: the graph grows by K steps of inserted points."""
    import torch

    from paper_1602_06819_amd import metrics
    from paper_1602_06819_amd.graph import GraphConfig, KnnGraph
    from paper_1602_06819_amd.serve import Admission, stream_totals

    n0 = w.n_initial
    K, W = args.steps, args.warmup
    step_ins = args.step_inserts
    if K * step_ins > w.n_insert:
        raise SystemExit(f"bench.py: {K} steps of {step_ins} points exceed the workload's "
                         f"{w.n_insert} inserts")
    ep_ins = args.epoch_inserts or w.batch
    ep_q = args.epoch_queries
    dev = torch.device("cuda:0")
    steps = serving_steps(max(K, W), step_ins)
    total_q = sum(stream_totals(st)[1] for st in steps)

    log(f"[bench] generating {w.name}")
    t = time.perf_counter()
    X, labels = w.mixture().sample(n0 + w.n_insert, w.stream_seed, with_labels=True)
    Q = w.mixture().sample(total_q, w.query_seed)
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    Xins = Xd[n0:]
    log(f"[bench] {n0 + w.n_insert} points and {total_q} query points in "
        f"{time.perf_counter() - t:.1f} s")
    n_final = n0 + K * step_ins
    cfg = GraphConfig(dim=w.dim, k=w.k, capacity=n0 + max(K, W) * step_ins, max_batch=ep_ins,
                      speedup=w.speedup, expansion_num=w.expansion_num,
                      expansion_den=w.expansion_den, depth=w.depth, seed=w.algo_seed,
                      dtype="f32", score=w.score)
    adm = Admission(ep_ins, ep_q)

    # ---- exact initial graph (timed on its own) ----------------------------
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g = KnnGraph.build_exact(cfg, Xd[:n0])
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    ids0, d0 = g.lists()
    log(f"[bench] exact initial graph of {n0} points: {build_ms:.1f} ms")

    # ---- warmup: the first W steps on a copy of the initial graph ----------------
    if W > 0:
        gw = KnnGraph.load(cfg, Xd[:n0], ids0, d0)
        run_steps(gw, steps[:W], Xins, Qd, adm, False, False)
        torch.cuda.synchronize()
        gw.close()
        del gw
        torch.cuda.empty_cache()
        log(f"[bench] {W} warmup steps done")

    # ---- timed steps ---------------------------------------------------------
    g.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = run_steps(g, steps[:K], Xins, Qd, adm, True, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage = g.timing_read()
    g.timing(False)
    elapsed = t1 - t0
    inserts = K * step_ins
    assert g.n == n_final
    budgets = [g.budget(n0), g.budget(n_final - step_ins)]
    value = inserts / elapsed
    lat = np.array([a.elapsed_time(z) for a, z, _, _, _ in recs])
    ins_st = np.concatenate([r[4][5].cpu().numpy() for r in recs if r[2] > 0]).astype(np.float64)
    qrecs = [r for r in recs if r[3] > 0]
    q_ev = np.concatenate([r[4][4].cpu().numpy() for r in qrecs]).astype(np.float64)
    q_lr = np.concatenate([r[4][6].cpu().numpy() for r in qrecs]).astype(np.float64)
    n_q = int(q_ev.size)
    epochs = len(recs)
    log(f"[bench] {K} steps: {value:.0f} inserts/s, {1000 * elapsed / K:.1f} ms/step, "
        f"{epochs} epochs, p50/p99 epoch {np.percentile(lat, 50):.1f}/"
        f"{np.percentile(lat, 99):.1f} ms")

    # ---- roofline of the search kernel (dominant) ----------------------------
    search_ms, search_launches = stage["search"]
    evals = ins_st[:, 0].sum() + q_ev.sum()
    lists = ins_st[:, 1].sum() + q_lr.sum()
    search_bytes = search_algorithmic_bytes(w.score, w.dim, w.k, inserts + n_q, evals, lists)
    search_avg_ms = search_ms / max(search_launches, 1)
    bytes_per_launch = search_bytes / max(search_launches, 1)
    achieved = bytes_per_launch / (search_avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": recorded_serving_traffic(
                    w.name, serving_run_shape(w, K, step_ins, ep_ins, ep_q)),
                "kernel": f"k_search ({w.score} rows)",
                "avg_launch_ms": search_avg_ms,
                "algorithmic_bytes_per_launch": bytes_per_launch}

    # ---- recall of the final graph against its exact graph ---------------------
    rec = {}
    if not args.no_recall:
        ids_online, _ = g.lists()
        cfg_x = GraphConfig(dim=w.dim, k=w.k, capacity=n_final, max_batch=1024,
                            speedup=w.speedup, dtype="f32", score="exact")
        te = time.perf_counter()
        gx = KnnGraph.build_exact(cfg_x, Xd[:n_final])
        ids_exact, _ = gx.lists()
        torch.cuda.synchronize()
        t_gt = time.perf_counter() - te
        io = ids_online.cpu().numpy()
        ie = ids_exact.cpu().numpy()
        gx.close()
        del gx
        torch.cuda.empty_cache()
        e_c = metrics.correct_edges(io, ie)
        rec = {"recall_at_k": e_c / (n_final * w.k),
               "recall_new_nodes": metrics.recall(io[n0:], ie[n0:]),
               "recall_old_nodes": metrics.recall(io[:n0], ie[:n0]),
               "quality_Q": metrics.quality(e_c, n0, inserts, w.k),
               "exact_graph_s": t_gt}
        log(f"[bench] recall@{w.k} {rec['recall_at_k']:.4f} (new nodes "
            f"{rec['recall_new_nodes']:.4f}, old {rec['recall_old_nodes']:.4f}), "
            f"Q {rec['quality_Q']:.4f}; exact {n_final}-point graph in {t_gt:.1f} s")
    g.close()
    del g
    torch.cuda.empty_cache()

    # ---- search alone: bfloat16 scoring against float32 scoring ("FP32 plain") ----
    plain = None
    if args.plain_compare > 0:
        m = args.plain_compare
        Qs = Xins[:m]
        keys = torch.arange(n0, n0 + m, dtype=torch.int64, device=dev)
        gt = exact_topk_f64(Qs, Xd[:n0], w.k)
        plain = {"points": m, "n": n0}
        for score in (w.score, "exact"):
            cs = GraphConfig(dim=w.dim, k=w.k, capacity=n0, max_batch=m, speedup=w.speedup,
                             expansion_num=w.expansion_num, expansion_den=w.expansion_den,
                             depth=w.depth, seed=w.algo_seed, dtype="f32", score=score)
            gs = KnnGraph.load(cs, Xd[:n0], ids0, d0)
            gs.search(Qs, keys)              # first launch of this instantiation
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ri, _, _, _ = gs.search(Qs, keys)
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - ts)
            name = "f32" if score == "exact" else score
            plain[name] = {"ms": ms, "recall": metrics.recall(ri.cpu().numpy(), gt)}
            gs.close()
            del gs
        torch.cuda.empty_cache()
        log(f"[bench] search alone, {m} points: " + ", ".join(
            f"{k} {v['ms']:.1f} ms recall {v['recall']:.4f}"
            for k, v in plain.items() if isinstance(v, dict)))

    # ---- plain per-point insertion (b = 1) on the same GPU -------------------------
    per_point = None
    if args.per_point > 0:
        gp = KnnGraph.load(cfg, Xd[:n0], ids0, d0)
        P = min(args.per_point, inserts)
        gp.insert(Xins[:1], sims=False)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for i in range(1, P + 1):
            gp.insert(Xins[i:i + 1], sims=False)
        torch.cuda.synchronize()
        per_point = P / (time.perf_counter() - tp0)
        gp.close()
        del gp
        log(f"[bench] per-point insertion (b=1): {per_point:.0f} inserts/s")

    # ---- the naive method (Section 2.1) on the same GPU: the same inserts -----------
    naive = None
    if not args.no_naive:
        gn = KnnGraph.load(cfg, Xd[:n0], ids0, d0)
        sizes = [sum(r.size for r in reqs if r.kind == "insert") for reqs in steps[:K]]
        torch.cuda.synchronize()
        tn0 = time.perf_counter()
        lo = 0
        for total in sizes:
            end = lo + total
            while lo < end:
                hi = min(end, lo + ep_ins)
                gn.insert_exact(Xins[lo:hi])
                lo = hi
        torch.cuda.synchronize()
        naive = inserts / (time.perf_counter() - tn0)
        assert gn.n == n_final
        gn.close()
        del gn
        torch.cuda.empty_cache()
        log(f"[bench] naive exact insertion (brute force, batches of {ep_ins}): "
            f"{naive:.0f} inserts/s")

    # ---- calibration copy for the HBM byte counters ----------------------------------
    if args.calibrate_copy > 0:
        calibration_copy(args.calibrate_copy, dev)

    # ---- CPU oracle baseline -----------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample of the first epoch's inserts")
        cpu = cpu_baseline_serving(w, X, labels, args.cpu_seconds, args.cpu_procs)
        log(f"[bench] CPU oracle: {cpu['value']:.2f} inserts/s on {cpu['cores']} processes "
            f"({cpu['single_process_value']:.2f} on one)")

    return {
        "metric": METRIC,
        "value": value,
        "unit": "inserts/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "bf16m": "bf16", "fp8": "fp8", "exact": "f32"}[w.score],
        "data": "synthetic",
        "config": {"workload": w.name, "n_initial": n0, "n_final": n_final, "dim": w.dim,
                   "k": w.k, "step_inserts": step_ins, "epoch_max_inserts": ep_ins,
                   "epoch_max_queries": ep_q, "speedup": w.speedup,
                   "expansion": f"{w.expansion_num}/{w.expansion_den}", "depth": w.depth,
                   "mixture_components": w.n_clusters,
                   "component_rank": w.subspace_rank, "requests": "poisson 3:1 insert:query"},
        "p50_batch_ms": float(np.percentile(lat, 50)),
        "p99_batch_ms": float(np.percentile(lat, 99)),
        "epochs": epochs,
        "mean_epoch_inserts": inserts / max(sum(1 for r in recs if r[2] > 0), 1),
        **rec,
        "queries": n_q,
        "queries_per_s_in_mix": n_q / elapsed,
        "search_evals_per_insert": float(ins_st[:, 0].mean()),
        "lists_read_per_insert": float(ins_st[:, 1].mean()),
        "update_evals_per_insert": float(ins_st[:, 2].mean()),
        "evals_per_query": float(q_ev.mean()) if n_q else None,
        "budget_first_last": budgets,
        "build_exact_ms": build_ms,
        "stage_ms": {k: round(v[0], 3) for k, v in stage.items() if v[1]},
        "search_alone": plain,
        "per_point_inserts_per_s": per_point,
        "naive_exact_inserts_per_s": naive,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def calibration_copy(mib: int, dev) -> None:
    """A plain device copy of `mib` MiB (calibrates the HBM byte counters)."""
    import torch
    nbytes = mib << 20
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def serving_run_shape(w, steps: int, step_ins: int, ep_ins: int, ep_q: int) -> dict:
    """What a counter record of the serving run must match to be reported."""
    return {"steps": steps, "step_inserts": step_ins, "epoch_inserts": ep_ins,
            "epoch_queries": ep_q, "speedup": w.speedup,
            "expansion": f"{w.expansion_num}/{w.expansion_den}", "depth": w.depth}


def recorded_serving_traffic(workload: str, run_shape: dict):
    """HBM bytes per search launch of the serving run from the committed
    counter record, or None if there is none, it was taken on another
    kernel source or flags, or on another run shape."""
    from paper_1602_06819_amd import profsum
    path = os.path.join(ROOT, "profiles", f"traffic_k_search_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != profsum.search_kernel_hash("bf16"):
        return None
    if rec.get("run") != run_shape:
        return None
    return rec.get("bytes_per_dispatch")


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU only (one GPU holds one graph at its "
              "real shape; sharding across GPUs is not built). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    w = load_workload(args)
    out = bench_serving(args, w) if w.name.startswith("serve-") else bench_batches(args, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
