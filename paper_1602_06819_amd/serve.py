"""Continuous-batching serving loop over one graph.

Requests arrive as a Poisson process.  Each is an insert of 1..4096 points
or a read-only query of 1..512 points (three inserts to one query; sizes
floor(exp(U[0, ln(max + 1)))), i.e. log-uniform, means about 492 and 82).
The server runs epochs back to back.  An epoch admits the arrived requests
first come, first served, while its insert points fit the graph's
max_batch and its query points fit the query limit (admission by free
workspace: a request that does not fit waits for the next epoch, and no
later request overtakes it).  The epoch's queries and inserts then run as
one ``knng_epoch`` against the snapshot before the epoch, so a query's
answer and an insert's effect are those of running the epoch's requests
alone on that snapshot.  A request completes when its epoch completes.

Time is the server's wall clock, except that idle gaps (no request has
arrived) are skipped instead of slept: GPU work is unaffected by them, and
the latencies are those of a server that waits for the next arrival.

This module is host-side scheduling only; every step of insertion and
search runs in the library's kernels.
"""

from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Request:
    rid: int
    kind: str          # "insert" | "query"
    size: int          # points
    arrival: float     # seconds from the start
    offset: int        # first point in the insert or query stream


def log_uniform_sizes(rng: np.random.Generator, count: int, max_size: int) -> np.ndarray:
    """floor(exp(U[0, ln(max_size + 1)))): 1 .. max_size, log-uniform."""
    u = rng.uniform(0.0, math.log(max_size + 1), size=count)
    return np.minimum(np.floor(np.exp(u)).astype(np.int64), max_size)


def make_requests(seed: int, rate: float, count: int, p_insert: float = 0.75,
                  max_insert: int = 4096, max_query: int = 512) -> list[Request]:
    """`count` requests with Poisson arrivals at `rate` requests per second."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    is_ins = rng.uniform(size=count) < p_insert
    ins_sizes = log_uniform_sizes(rng, count, max_insert)
    q_sizes = log_uniform_sizes(rng, count, max_query)
    out = []
    ins_off = q_off = 0
    for i in range(count):
        if is_ins[i]:
            out.append(Request(i, "insert", int(ins_sizes[i]), float(arrivals[i]), ins_off))
            ins_off += int(ins_sizes[i])
        else:
            out.append(Request(i, "query", int(q_sizes[i]), float(arrivals[i]), q_off))
            q_off += int(q_sizes[i])
    return out


def stream_totals(reqs: list[Request]) -> tuple[int, int]:
    """Insert and query points the requests consume."""
    ins = sum(r.size for r in reqs if r.kind == "insert")
    q = sum(r.size for r in reqs if r.kind == "query")
    return ins, q


@dataclass
class Epoch:
    requests: list
    ins_lo: int
    ins_hi: int
    q_lo: int
    q_hi: int
    n_before: int = 0
    start: float = 0.0
    end: float = 0.0


class Admission:
    """First come, first served admission within the workspace limits."""

    def __init__(self, max_insert_points: int, max_query_points: int):
        self.max_ins = max_insert_points
        self.max_q = max_query_points

    def fits_alone(self, r: Request) -> bool:
        return r.size <= (self.max_ins if r.kind == "insert" else self.max_q)

    def take(self, pending: deque, now: float) -> list:
        """Pop the arrived requests of the next epoch from the queue head."""
        ins = q = 0
        taken = []
        while pending and pending[0].arrival <= now:
            r = pending[0]
            if r.kind == "insert":
                if ins + r.size > self.max_ins:
                    break
                ins += r.size
            else:
                if q + r.size > self.max_q:
                    break
                q += r.size
            taken.append(pending.popleft())
        return taken


def plan_epoch(taken: list) -> Epoch:
    """The epoch's slices of the insert and query streams (FIFO admission
    keeps each kind's requests contiguous in its stream)."""
    ins = [r for r in taken if r.kind == "insert"]
    qs = [r for r in taken if r.kind == "query"]
    for a, b in zip(ins, ins[1:]):
        assert b.offset == a.offset + a.size
    for a, b in zip(qs, qs[1:]):
        assert b.offset == a.offset + a.size
    ins_lo = ins[0].offset if ins else 0
    ins_hi = ins[-1].offset + ins[-1].size if ins else ins_lo
    q_lo = qs[0].offset if qs else 0
    q_hi = qs[-1].offset + qs[-1].size if qs else q_lo
    return Epoch(taken, ins_lo, ins_hi, q_lo, q_hi)


@dataclass
class ServeResult:
    epochs: list = field(default_factory=list)
    latency: dict = field(default_factory=dict)    # rid -> seconds
    busy: float = 0.0                              # seconds spent in epochs
    span: float = 0.0                              # first arrival .. last completion
    query_out: list = field(default_factory=list)  # per epoch (ids, d) on the host, if kept

    def summary(self, reqs: list[Request]) -> dict:
        lat = np.array([self.latency[r.rid] for r in reqs])
        kinds = np.array([r.kind for r in reqs])
        ins_pts, q_pts = stream_totals(reqs)
        out = {
            "requests": len(reqs), "epochs": len(self.epochs),
            "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "utilization": self.busy / self.span if self.span > 0 else 0.0,
            "inserted_points_per_s": ins_pts / self.span if self.span > 0 else 0.0,
            "query_points_per_s": q_pts / self.span if self.span > 0 else 0.0,
            "mean_epoch_ms": 1e3 * self.busy / max(len(self.epochs), 1),
        }
        for kind in ("insert", "query"):
            sel = lat[kinds == kind]
            if len(sel):
                out[f"{kind}_p50_ms"] = 1e3 * float(np.percentile(sel, 50))
                out[f"{kind}_p99_ms"] = 1e3 * float(np.percentile(sel, 99))
        return out


def serve(graph, reqs: list[Request], ins_points, q_points, max_query_points: int,
          keep_queries: bool = False, sync=None) -> ServeResult:
    """Run the requests through `graph` (a KnnGraph).  `ins_points` and
    `q_points` are device tensors holding the insert and query streams."""
    import torch
    sync = sync or torch.cuda.synchronize
    adm = Admission(graph.cfg.max_batch, max_query_points)
    for r in reqs:
        if not adm.fits_alone(r):
            raise ValueError(f"request {r.rid} ({r.kind}, {r.size} points) exceeds the limits")
    pending = deque(sorted(reqs, key=lambda r: r.arrival))
    res = ServeResult()
    skipped = 0.0                 # idle time jumped over
    sync()
    t0 = time.perf_counter()

    def now() -> float:
        return time.perf_counter() - t0 + skipped

    while pending:
        t = now()
        if pending[0].arrival > t:
            skipped += pending[0].arrival - t        # idle: jump to the next arrival
            t = now()
        ep = plan_epoch(adm.take(pending, t))
        ep.start = t
        ep.n_before = graph.n
        x = ins_points[ep.ins_lo:ep.ins_hi] if ep.ins_hi > ep.ins_lo else None
        q = q_points[ep.q_lo:ep.q_hi] if ep.q_hi > ep.q_lo else None
        _, _, qi, qd, _ = graph.epoch(x, q)
        sync()
        ep.end = now()
        res.busy += ep.end - ep.start
        for r in ep.requests:
            res.latency[r.rid] = ep.end - r.arrival
        if keep_queries:
            res.query_out.append(None if qi is None else (qi.cpu().numpy(), qd.cpu().numpy()))
        res.epochs.append(ep)
    first = min(r.arrival for r in reqs)
    res.span = max(ep.end for ep in res.epochs) - first
    return res


def main(argv=None) -> None:
    """Offered-load sweep of the serving workload: one JSON line per rate."""
    import argparse
    import json
    import sys

    import torch

    from datagen import get_workload
    from .graph import GraphConfig, KnnGraph

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="serve-f32-d96-1m-2m")
    ap.add_argument("--rates", default="100,200,400", help="requests per second")
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--max-batch", type=int, default=16384)
    ap.add_argument("--max-query", type=int, default=4096)
    ap.add_argument("--speedup", type=int, default=None)
    ap.add_argument("--expansion", default=None)
    ap.add_argument("--seed", type=int, default=2024)
    args = ap.parse_args(argv)
    w = get_workload(args.workload)
    if args.expansion:
        num, den = (int(v) for v in args.expansion.split("/"))
        w = w.scaled(expansion_num=num, expansion_den=den)
    speedup = args.speedup or w.speedup
    rates = [float(r) for r in args.rates.split(",")]
    plans = {r: make_requests(args.seed, r, args.requests) for r in rates}
    need_ins = max(stream_totals(p)[0] for p in plans.values())
    need_q = max(stream_totals(p)[1] for p in plans.values())
    n0 = w.n_initial
    X = w.mixture().sample(n0 + need_ins, w.stream_seed)
    Q = w.mixture().sample(need_q, w.query_seed)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    is_float = w.kind != "u8"
    cfg = GraphConfig(dim=w.dim, k=w.k, capacity=n0 + need_ins, max_batch=args.max_batch,
                      speedup=speedup, expansion_num=w.expansion_num,
                      expansion_den=w.expansion_den, depth=w.depth, seed=w.algo_seed,
                      dtype="f32" if is_float else "u8", score=w.score if is_float else "exact")
    t = time.perf_counter()
    g0 = KnnGraph.build_exact(cfg, Xd[:n0])
    ids, d = g0.lists()
    torch.cuda.synchronize()
    print(f"[serve] exact graph of {n0} points: {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    g0.close()
    del g0
    for r in rates:
        g = KnnGraph.load(cfg, Xd[:n0], ids, d)
        res = serve(g, plans[r], Xd[n0:], Qd, args.max_query)
        out = {"workload": w.name, "offered_rate_req_s": r, "speedup": speedup,
               "expansion": f"{w.expansion_num}/{w.expansion_den}", "n_final": g.n,
               **res.summary(plans[r])}
        print(json.dumps(out), flush=True)
        g.close()
        del g
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
