"""Step counts of the iGNNS search kernel on a workload's graph, from the
profiling build of the library (libknng_counters.so: the same sources with
the search's step counters compiled in; build it with
``python -m paper_1602_06819_amd.build --counters``).

    python -m paper_1602_06819_amd.stepstats [--workload NAME] [--points M] [--out FILE.md]

Serving workloads: M inserted points of the stream are searched at once on
the exact graph of the initial points (the first epoch's search).  Batch
workloads: the first M inserted points are searched on the exact initial
graph.  The output is a markdown table of totals and per-search means.
"""

from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="serve-f32-d96-1m-2m")
    ap.add_argument("--points", type=int, default=4096)
    ap.add_argument("--out", default=None, help="write the markdown summary here")
    args = ap.parse_args(argv)

    from paper_1602_06819_amd.build import COUNTERS_LIB_PATH
    os.environ.setdefault("KNNG_LIB", COUNTERS_LIB_PATH)
    if not os.path.exists(os.environ["KNNG_LIB"]):
        raise SystemExit(f"{os.environ['KNNG_LIB']} is missing: build it with "
                         "`python -m paper_1602_06819_amd.build --counters`")
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch

    from datagen import get_workload
    from paper_1602_06819_amd.graph import GraphConfig, KnnGraph

    w = get_workload(args.workload)
    n0, m = w.n_initial, args.points
    X = w.mixture().sample(n0 + m, w.stream_seed)
    dtype = w.kind
    Xd = torch.from_numpy(X).cuda()
    cfg = GraphConfig(dim=w.dim, k=w.k, capacity=n0 + m, max_batch=max(m, 1), speedup=w.speedup,
                      expansion_num=w.expansion_num, expansion_den=w.expansion_den,
                      depth=w.depth, seed=w.algo_seed, dtype=dtype,
                      score=w.score if dtype == "f32" else "exact")
    if dtype == "f32":
        cx = GraphConfig(dim=w.dim, k=w.k, capacity=n0, max_batch=1024, dtype="f32",
                         score="exact")
        gx = KnnGraph.build_exact(cx, Xd[:n0])
        ids, d = gx.lists()
        gx.close()
        g = KnnGraph.load(cfg, Xd[:n0], ids, d)
    else:
        g = KnnGraph.build_exact(cfg, Xd[:n0])
    keys = torch.arange(n0, n0 + m, dtype=torch.int64, device="cuda")
    g.step_counters(reset=True)
    g.search(Xd[n0:n0 + m], keys)
    c = g.step_counters(reset=True)

    s = max(c["searches"], 1)
    gathered = c["window_cands"] - c["window_kept"] + c["scan_cands"]
    rows = [
        ("searches", c["searches"], None),
        ("evaluations", c["evaluations"], c["evaluations"] / s),
        ("steps", c["window_steps"] + c["scan_steps"], (c["window_steps"] + c["scan_steps"]) / s),
        ("restart-window steps", c["window_steps"], c["window_steps"] / s),
        ("list-scan steps", c["scan_steps"], c["scan_steps"] / s),
        ("window candidates", c["window_cands"], c["window_cands"] / s),
        ("  of which scores kept from the window before", c["window_kept"], c["window_kept"] / s),
        ("  of which visited", c["window_visited"], c["window_visited"] / s),
        ("  of which committed (evaluations)", c["window_committed"], c["window_committed"] / s),
        ("list-scan candidates", c["scan_cands"], c["scan_cands"] / s),
        ("  of which visited", c["scan_visited"], c["scan_visited"] / s),
        ("  of which committed (evaluations)", c["scan_committed"], c["scan_committed"] / s),
        ("restarts that started a climb", c["restarts_taken"], c["restarts_taken"] / s),
        ("climb moves", c["moves"], c["moves"] / s),
        ("rows gathered", gathered, gathered / s),
    ]
    lines = [f"# Search step counts: {w.name}, {m} searches on the exact {n0}-point graph", "",
             "Command:", "", "```",
             "python -m paper_1602_06819_amd.build --counters && "
             f"python -m paper_1602_06819_amd.stepstats --workload {w.name} --points {m}"
             + (f" --out {args.out}" if args.out else ""), "```", "",
             f"Score {cfg.score}, k = {w.k}, speedup {w.speedup}, expansion "
             f"{w.expansion_num}/{w.expansion_den}; budget {g.budget(n0)} evaluations per search.",
             "", "| quantity | total | per search |", "|---|---|---|"]
    for name, tot, per in rows:
        lines.append(f"| {name} | {tot:,} | {'' if per is None else f'{per:,.1f}'} |")
    lines += ["", f"Rows gathered per evaluation: {gathered / max(c['evaluations'], 1):.2f}."]
    text = "\n".join(lines) + "\n"
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()
