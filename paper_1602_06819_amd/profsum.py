"""Summaries of rocprofv3 CSV output for the committed profile records.

    python -m paper_1602_06819_amd.profsum trace  <dir> <out.md> "<command>"
    python -m paper_1602_06819_amd.profsum pmc    <fetch_dir> <write_dir> <out.json> \
        "<fetch command>" "<write command>" <copy_bytes>
    python -m paper_1602_06819_amd.profsum pmc-serve <fetch_dir> <write_dir> <out.json> \
        "<fetch command>" "<write command>" <copy_bytes> '<run shape json>'

`trace` reads a `--kernel-trace --stats -f csv` run and writes per-kernel
statistics, split by grid size (one kernel serves batches, single points
and query sets), and per kernel over all its grids.  `pmc-serve` writes the
record of the serving run: the bfloat16 search's scaled HBM bytes averaged
over all its dispatches (epochs differ in size), with the run shape they
were taken on.  `pmc` reads one `--pmc FETCH_SIZE` and one
`--pmc WRITE_SIZE` run, scales both by what the counters read for the
calibration copy of `copy_bytes` bytes, and writes the bytes per dispatch
of the search kernel together with the hash of its source, so that a stale
record is never reported for a changed kernel.
"""

from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
SEARCH_SOURCES = ["csrc/search.h", "csrc/device.h", "csrc/common.h", "csrc/internal.h"]
# the instantiation unit and the kernel-name prefix of each scoring format
SEARCH_UNITS = {"i8": ("search_u8.hip", "k_search<knng::ScoreI8"),
                "bf16": ("search_bf16.hip", "k_search<knng::ScoreBF16")}
SEARCH_KERNEL = SEARCH_UNITS["i8"][1]
MAX_GRID_ROWS = 16        # rows of the per-grid table (the per-kernel table covers all)


def search_kernel_hash(fmt: str = "i8") -> str:
    """Hash of the search kernel's sources for one scoring format and of the
    flags it is compiled with (a record taken for other code or flags is
    stale)."""
    from . import build as _build
    unit = SEARCH_UNITS[fmt][0]
    h = hashlib.sha256()
    for rel in SEARCH_SOURCES[:1] + ["csrc/" + unit] + SEARCH_SOURCES[1:]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    flags = _build.HIP_FLAGS + _build.SOURCE_FLAGS.get(unit, [])
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def _rows(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    for path in files:
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def _short(name: str) -> str:
    name = name.strip('"')
    return name if len(name) < 150 else name[:147] + "..."


def _base(name: str) -> str:
    """The kernel function's name without its template arguments."""
    name = name.strip('"')
    if name.startswith("void "):
        name = name[5:]
    cut = [i for i in (name.find("<"), name.find("(")) if i >= 0]
    return name[:min(cut)] if cut else name


def kernel_table(directory: str):
    stats = defaultdict(list)
    for r in _rows(directory, "kernel_trace.csv"):
        name = r.get("Kernel_Name") or r.get("KernelName") or "?"
        start = int(r.get("Start_Timestamp") or r.get("BeginNs") or 0)
        end = int(r.get("End_Timestamp") or r.get("EndNs") or 0)
        grid = r.get("Grid_Size_X") or r.get("Grid_Size") or r.get("grd") or "?"
        wg = r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or r.get("wgr") or "?"
        stats[(name, grid, wg)].append((end - start) / 1000.0)
    return stats


def write_trace(directory: str, out: str, command: str) -> None:
    stats = kernel_table(directory)
    total = sum(sum(v) for v in stats.values())
    lines = ["# rocprofv3 kernel trace summary", "", "Command:", "", "```", command, "```", "",
             "Durations in microseconds, per kernel and grid (threads in x).", "",
             "| kernel | grid x | wg | calls | avg us | min us | max us | total us | % |",
             "|---|---|---|---|---|---|---|---|---|"]
    rows = sorted(stats.items(), key=lambda kv: -sum(kv[1]))
    for (name, grid, wg), v in rows[:MAX_GRID_ROWS]:
        lines.append(f"| `{_short(name)}` | {grid} | {wg} | {len(v)} | {sum(v) / len(v):.1f} | "
                     f"{min(v):.1f} | {max(v):.1f} | {sum(v):.1f} | {100 * sum(v) / total:.1f} |")
    if len(rows) > MAX_GRID_ROWS:
        rest = rows[MAX_GRID_ROWS:]
        lines.append(f"| ({len(rest)} more kernel/grid rows, {sum(len(v) for _, v in rest)} "
                     f"calls) | | | | | | | {sum(sum(v) for _, v in rest):.1f} | "
                     f"{100 * sum(sum(v) for _, v in rest) / total:.1f} |")
    by_kernel = defaultdict(list)
    for (name, _grid, _wg), v in stats.items():
        by_kernel[name].extend(v)
    lines += ["", "Per kernel, all grids:", "",
              "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
    for name, v in sorted(by_kernel.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{_short(name)}` | {len(v)} | {sum(v) / len(v):.1f} | {sum(v):.1f} | "
                     f"{100 * sum(v) / total:.1f} |")
    by_base = defaultdict(list)
    for name, v in by_kernel.items():
        by_base[_base(name)].extend(v)
    lines += ["", "Per kernel function, all instantiations and grids:", "",
              "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
    for name, v in sorted(by_base.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name}` | {len(v)} | {sum(v) / len(v):.1f} | {sum(v):.1f} | "
                     f"{100 * sum(v) / total:.1f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counter_table(directory: str):
    vals = defaultdict(list)
    for r in _rows(directory, "counter_collection.csv"):
        name = r.get("Kernel_Name", "?")
        grid = r.get("Grid_Size_X") or r.get("Grid_Size") or "?"
        cname = r.get("Counter_Name", "?")
        vals[(name, grid, cname)].append(float(r.get("Counter_Value", "nan")))
    return vals


def write_pmc(fetch_dir: str, write_dir: str, out: str, fetch_cmd: str, write_cmd: str,
              copy_bytes: int) -> None:
    fetch = counter_table(fetch_dir)
    write = counter_table(write_dir)

    def pick(table, kernel_part, counter):
        # the calibration copy is the largest copy dispatch of the run
        best = None
        for (name, grid, cname), v in table.items():
            if kernel_part in name and cname == counter:
                if best is None or max(v) > max(best[2]):
                    best = (name, grid, v)
        return best

    copy_f = pick(fetch, "copy", "FETCH_SIZE")
    copy_w = pick(write, "copy", "WRITE_SIZE")
    # the largest-grid dispatches of the search kernel are the insert batches
    rows = {}
    for table, counter in ((fetch, "FETCH_SIZE"), (write, "WRITE_SIZE")):
        for (name, grid, cname), v in table.items():
            if SEARCH_KERNEL in name and cname == counter:
                rows.setdefault(counter, {})[grid] = sum(v) / len(v)
    kib = 1024.0
    scale_f = copy_bytes / (max(copy_f[2]) * kib) if copy_f else None
    scale_w = copy_bytes / (max(copy_w[2]) * kib) if copy_w else None
    rec = {
        "kernel": "k_search (int8 rows)",
        "source_hash": search_kernel_hash(),
        "fetch_command": fetch_cmd,
        "write_command": write_cmd,
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": max(copy_f[2]) if copy_f else None,
        "copy_write_kib": max(copy_w[2]) if copy_w else None,
        "fetch_scale": scale_f,
        "write_scale": scale_w,
        "per_grid_kib_per_dispatch": rows,
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)


def _copy_scale(table, counter: str, copy_bytes: int):
    """Bytes per counter unit from the run's calibration copy (the largest
    copy dispatch), or None."""
    best = None
    for (name, _grid, cname), v in table.items():
        if "copy" in name and cname == counter and (best is None or max(v) > best):
            best = max(v)
    return copy_bytes / (best * 1024.0) if best else None


def write_pmc_serve(fetch_dir: str, write_dir: str, out: str, fetch_cmd: str, write_cmd: str,
                    copy_bytes: int, run_shape: dict) -> None:
    fetch = counter_table(fetch_dir)
    write = counter_table(write_dir)
    kernel = SEARCH_UNITS["bf16"][1]
    scale_f = _copy_scale(fetch, "FETCH_SIZE", copy_bytes)
    scale_w = _copy_scale(write, "WRITE_SIZE", copy_bytes)

    def per_dispatch(table, counter):
        vals = [x for (name, _g, cname), v in table.items()
                if kernel in name and cname == counter for x in v]
        return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)

    f_kib, nf = per_dispatch(fetch, "FETCH_SIZE")
    w_kib, nw = per_dispatch(write, "WRITE_SIZE")
    total = None
    if f_kib is not None and w_kib is not None and scale_f and scale_w:
        total = 1024.0 * (f_kib * scale_f + w_kib * scale_w)
    rec = {
        "kernel": "k_search (bf16 rows), serving run",
        "source_hash": search_kernel_hash("bf16"),
        "run": run_shape,
        "fetch_command": fetch_cmd,
        "write_command": write_cmd,
        "copy_bytes": copy_bytes,
        "fetch_scale": scale_f,
        "write_scale": scale_w,
        "dispatches": [nf, nw],
        "fetch_kib_per_dispatch": f_kib,
        "write_kib_per_dispatch": w_kib,
        "bytes_per_dispatch": total,
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        write_trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == "pmc":
        write_pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6],
                  int(sys.argv[7]))
    elif mode == "pmc-serve":
        write_pmc_serve(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6],
                        int(sys.argv[7]), json.loads(sys.argv[8]))
    else:
        raise SystemExit(__doc__)
