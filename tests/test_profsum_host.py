"""Host logic of the profile summaries: kernel-trace statistics, the HBM
counter record scaled by the calibration copy, and the per-launch traffic
the benchmark derives from a record (only for the kernel it was taken on).
Synthetic rocprofv3 CSV files; no GPU."""

import csv
import json
import os

import pytest

import bench
from paper_1602_06819_amd import profsum

SEARCH = "void knng::k_search<knng::ScoreI8<2, 2>, 2, 2, 16, false>(knng::SearchArgs)"
COPY = "__amd_rocclr_copyBuffer"


def write_csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_trace_statistics(tmp_path):
    fields = ["Kernel_Name", "Grid_Size_X", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"]
    rows = [
        {"Kernel_Name": SEARCH, "Grid_Size_X": 16384, "Workgroup_Size_X": 64,
         "Start_Timestamp": 1_000_000, "End_Timestamp": 1_000_000 + d}
        for d in (2_000_000, 2_200_000, 2_400_000)
    ] + [{"Kernel_Name": "k_merge", "Grid_Size_X": 512, "Workgroup_Size_X": 64,
          "Start_Timestamp": 0, "End_Timestamp": 400_000}]
    write_csv(str(tmp_path / "t" / "run_kernel_trace.csv"), fields, rows)
    stats = profsum.kernel_table(str(tmp_path / "t"))
    v = stats[(SEARCH, "16384", "64")]
    assert sorted(v) == [2000.0, 2200.0, 2400.0]          # microseconds
    out = str(tmp_path / "t.md")
    profsum.write_trace(str(tmp_path / "t"), out, "the command")
    text = open(out).read()
    assert "the command" in text
    row = [line for line in text.splitlines() if "16384" in line][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    # calls, avg, min, max, total, share of all kernel time
    assert cells[3:] == ["3", "2200.0", "2000.0", "2400.0", "6600.0", f"{100 * 6600 / 7000:.1f}"]


def counters(path, rows):
    write_csv(path, ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], rows)


def test_counter_record_and_traffic(tmp_path, monkeypatch):
    copy_bytes = 256 << 20
    # the copy reads 128 MiB and writes 256 MiB as the counters see them
    counters(str(tmp_path / "f" / "pmc_counter_collection.csv"), [
        {"Kernel_Name": COPY, "Grid_Size": 65536, "Counter_Name": "FETCH_SIZE", "Counter_Value": 131072},
        {"Kernel_Name": COPY, "Grid_Size": 512, "Counter_Name": "FETCH_SIZE", "Counter_Value": 12},
        {"Kernel_Name": SEARCH, "Grid_Size": 16384, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000},
        {"Kernel_Name": SEARCH, "Grid_Size": 16384, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000},
        {"Kernel_Name": SEARCH, "Grid_Size": 640000, "Counter_Name": "FETCH_SIZE", "Counter_Value": 9000},
    ])
    counters(str(tmp_path / "w" / "pmc_counter_collection.csv"), [
        {"Kernel_Name": COPY, "Grid_Size": 65536, "Counter_Name": "WRITE_SIZE", "Counter_Value": 262144},
        {"Kernel_Name": SEARCH, "Grid_Size": 16384, "Counter_Name": "WRITE_SIZE", "Counter_Value": 50},
    ])
    out = str(tmp_path / "rec.json")
    profsum.write_pmc(str(tmp_path / "f"), str(tmp_path / "w"), out, "fetch cmd", "write cmd",
                      copy_bytes)
    rec = json.load(open(out))
    assert rec["fetch_scale"] == pytest.approx(2.0)        # the largest copy dispatch
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["per_grid_kib_per_dispatch"]["FETCH_SIZE"] == {"16384": 2000.0, "640000": 9000.0}
    assert rec["source_hash"] == profsum.search_kernel_hash()

    # the benchmark reads its record from profiles/ under its root
    os.makedirs(tmp_path / "profiles")
    os.replace(out, tmp_path / "profiles" / "traffic_k_search_i8.json")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic(16384) == pytest.approx(1024.0 * (2000.0 * 2.0 + 50.0 * 1.0))
    assert bench.recorded_traffic(64) is None              # no dispatch of that grid
    # a record taken on other kernel sources or flags is never used
    path = tmp_path / "profiles" / "traffic_k_search_i8.json"
    rec = json.load(open(path))
    rec["source_hash"] = "0" * 16
    json.dump(rec, open(path, "w"))
    assert bench.recorded_traffic(16384) is None


def test_hash_covers_compile_flags(monkeypatch):
    from paper_1602_06819_amd import build
    h0 = profsum.search_kernel_hash()
    monkeypatch.setitem(build.SOURCE_FLAGS, "search_u8.hip", ["-O2"])
    assert profsum.search_kernel_hash() != h0


def test_search_algorithmic_bytes():
    # int8 rows of 64 bytes, k = 10: 64 B per evaluation, 40 B per list read,
    # 64 B of query and 80 B of output per point
    got = bench.search_algorithmic_bytes("u8", 64, 10, 256, 2_000_000.0, 150_000.0)
    assert got == pytest.approx(2_000_000 * 64 + 150_000 * 40 + 256 * (64 + 80))
    # float graphs add the re-rank's float32 rows of the kept candidates
    b = bench.search_algorithmic_bytes("bf16", 128, 20, 1, 100.0, 10.0)
    assert b == pytest.approx(100 * 256 + 10 * 80 + 512 + 160 + 40 * 512)
    b = bench.search_algorithmic_bytes("fp8", 960, 50, 1, 1.0, 0.0)
    # FP8 keeps 4k candidates, at most 128, for the re-rank
    assert b == pytest.approx(964 + 3840 + 400 + 128 * 3840)


def test_serving_counter_record_and_traffic(tmp_path, monkeypatch):
    """The serving record averages the bfloat16 search over all its
    dispatches (epochs differ in size) and is reported only for its kernel
    source and run shape."""
    search = "void knng::k_search<knng::ScoreBF16<4, 4>, 4, 4, 16, true>(knng::SearchArgs)"
    other = "void knng::k_search<knng::ScoreI8<2, 2>, 2, 2, 16, false>(knng::SearchArgs)"
    copy_bytes = 256 << 20
    counters(str(tmp_path / "f" / "pmc_counter_collection.csv"), [
        {"Kernel_Name": COPY, "Grid_Size": 65536, "Counter_Name": "FETCH_SIZE", "Counter_Value": 131072},
        {"Kernel_Name": search, "Grid_Size": 1048576, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000},
        {"Kernel_Name": search, "Grid_Size": 262144, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000},
        {"Kernel_Name": other, "Grid_Size": 16384, "Counter_Name": "FETCH_SIZE", "Counter_Value": 99999},
    ])
    counters(str(tmp_path / "w" / "pmc_counter_collection.csv"), [
        {"Kernel_Name": COPY, "Grid_Size": 65536, "Counter_Name": "WRITE_SIZE", "Counter_Value": 262144},
        {"Kernel_Name": search, "Grid_Size": 1048576, "Counter_Name": "WRITE_SIZE", "Counter_Value": 30},
        {"Kernel_Name": search, "Grid_Size": 262144, "Counter_Name": "WRITE_SIZE", "Counter_Value": 10},
    ])
    from datagen import get_workload
    w = get_workload("serve-f32-d96-1m-2m")
    shape = bench.serving_run_shape(w, 20, 50_000, 16384, 4096)
    out = str(tmp_path / "rec.json")
    profsum.write_pmc_serve(str(tmp_path / "f"), str(tmp_path / "w"), out, "fc", "wc", copy_bytes,
                            shape)
    rec = json.load(open(out))
    assert rec["dispatches"] == [2, 2]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # mean fetch 2000 KiB x 2 + mean write 20 KiB x 1, per dispatch
    assert rec["bytes_per_dispatch"] == pytest.approx(1024.0 * (2000 * 2.0 + 20 * 1.0))
    profiles = tmp_path / "profiles"
    profiles.mkdir()
    (profiles / f"traffic_k_search_{w.name}.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_serving_traffic(w.name, shape) == pytest.approx(rec["bytes_per_dispatch"])
    other_shape = dict(shape, speedup=10)
    assert bench.recorded_serving_traffic(w.name, other_shape) is None
    rec["source_hash"] = "0" * 16
    (profiles / f"traffic_k_search_{w.name}.json").write_text(json.dumps(rec))
    assert bench.recorded_serving_traffic(w.name, shape) is None
