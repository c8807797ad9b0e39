"""Benchmark of online k-nn graph building on one MI355X.

Default workload (the integer workload at scale): 100,000 uint8 points,
d = 64, drawn from a 100-cluster Gaussian mixture (sigma 10); exact initial
graph by brute force (int8 MFMA); then 10,000 points inserted in batches of
256 (iGNNS search + batch peers + depth-2 update + merge), then 10,000
read-only k-nn queries on the final graph.

A step is one insert batch: every stage of the insertion path over 256
points, all inputs already resident in GPU memory.  `value` is inserts per
second over the K timed steps (bracketed by device synchronisation).  The
report also carries recall@k of the final graph against its exact graph
(the metric is quoted at recall@k >= 0.95), p50/p99 batch latency, query
throughput, similarity evaluations per insert, the search kernel's achieved
fraction of the HBM roofline (algorithmic bytes / measured kernel time),
the plain per-point (batch = 1) insertion rate on the same GPU, and the
CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 40] [--warmup 2]
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
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="u8-d64-n100k-b256")
    ap.add_argument("--speedup", type=int, default=None, help="override the search speedup")
    ap.add_argument("--depth", type=int, default=None, help="override the update depth")
    ap.add_argument("--expansion", default=None, help="override e as num/den, e.g. 5/1")
    ap.add_argument("--score", default=None, choices=["exact", "bf16", "fp8"],
                    help="override the scoring rows of a float workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="points of the first batch the CPU oracle inserts")
    ap.add_argument("--per-point", type=int, default=256,
                    help="points inserted one at a time for the batch=1 baseline")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


def search_algorithmic_bytes(score: str, dim: int, k: int, points: int, evals: float,
                             lists: float) -> float:
    """Bytes the searches of `points` points must move: every evaluated
    point's scoring row (int8: d; bfloat16: 2d; FP8: d codes + a 4-byte
    scale; float32: 4d), every adjacency list read by the climb (k ids), the
    query row and the k (id, distance) output; float graphs also read the
    float32 rows of the kept candidates for the re-rank.  `score` is "u8"
    for integer graphs, else the float scoring format."""
    is_float = score != "u8"
    v_bytes = {"u8": dim, "bf16": 2 * dim, "fp8": dim + 4, "exact": 4 * dim}[score]
    q_bytes = 4 * dim if is_float else dim
    keep = min(64, 2 * k) if score in ("bf16", "fp8") else k
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


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU only (one GPU holds one graph at its "
              "real shape; sharding across GPUs is not built). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from datagen import get_workload
    from paper_1602_06819_amd import metrics
    from paper_1602_06819_amd.graph import GraphConfig, KnnGraph

    w = get_workload(args.workload)
    if args.depth is not None:
        w = w.scaled(depth=args.depth)
    if args.expansion is not None:
        num, den = (int(v) for v in args.expansion.split("/"))
        w = w.scaled(expansion_num=num, expansion_den=den)
    if args.score is not None:
        w = w.scaled(score=args.score)
    speedup = args.speedup or w.speedup
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
        log("[bench] float workload: the CPU oracle leg is not run (its float64 exact "
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

    # ---- calibration copy for the HBM byte counters ----------------------------------
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

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
        "dtype": "int8" if not is_float else {"bf16": "bf16", "fp8": "fp8",
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
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
