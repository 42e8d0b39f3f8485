"""Host logic of bench.py (no GPU): the per-kernel byte accounting, the
summary of rocprofv3 CSV output with its copy calibration, and the rule that
committed traffic counters are used only for the kernel sources and visit
buffer they were taken with."""
import csv
import json
import os

import pytest

import bench


def test_algorithmic_bytes_follow_the_per_unit_figures():
    st = {"walk_steps": 1000, "walks": 100, "gather_probes": 5000}
    transitions = 900
    assert bench.algorithmic_bytes("action_walk", st) == 12 * transitions + 8 * 1000
    assert bench.algorithmic_bytes("diag_walk", st) == 12 * transitions
    assert bench.algorithmic_bytes("diag_gather", st, atomics=70) == 4 * 5000 + 8 * 70
    assert bench.layout_bytes("diag_walk", st) == 12 * 1000 + 4 * transitions
    assert bench.layout_bytes("diag_gather", st) == 12 * 1000
    assert bench.layout_bytes("action_walk", st) == 0
    with pytest.raises(ValueError):
        bench.algorithmic_bytes("spmv", st)


def _write_csv(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _counter_run(tmp_path, name, counter, walk_kib, copy_kib, chunk):
    d = tmp_path / name
    d.mkdir()
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = [
        {"Dispatch_Id": 1, "Kernel_Name": "void mcmf::k_diag_walk_wide<double, false, false>(int)",
         "Counter_Name": counter, "Counter_Value": walk_kib / 2},
        {"Dispatch_Id": 1, "Kernel_Name": "void mcmf::k_diag_walk_wide<double, false, false>(int)",
         "Counter_Name": counter, "Counter_Value": walk_kib / 2},
        {"Dispatch_Id": 2, "Kernel_Name": "void mcmf::k_diag_walk_wide<double, false, false>(int)",
         "Counter_Name": counter, "Counter_Value": walk_kib},
        {"Dispatch_Id": 3, "Kernel_Name": "void at::native::neg_kernel(...)",
         "Counter_Name": counter, "Counter_Value": copy_kib},
    ]
    _write_csv(d / "run_counter_collection.csv", fields, rows)
    rec = {src: bench.source_sha(src) for _, src in bench.KERNELS.values()}
    rec[bench.CHUNK_KEY] = chunk
    (d / "sources.json").write_text(json.dumps(rec))
    return str(d)


def test_summary_scales_counters_by_the_copy_and_records_the_buffer(tmp_path):
    probe = 1 << 30
    chunk = 16 << 30
    # The copy reads 1 GiB and shows 512 MiB of FETCH_SIZE (factor 2) and
    # 1 GiB of WRITE_SIZE (factor 1); the walk shows 100 KiB per dispatch.
    fetch = _counter_run(tmp_path, "fetch", "FETCH_SIZE", 100.0, probe / 2048.0, chunk)
    write = _counter_run(tmp_path, "write", "WRITE_SIZE", 30.0, probe / 1024.0, chunk)
    out = bench.summarize(f"{fetch},{write}", probe)
    line = [l for l in out.splitlines() if l.startswith("traffic: ")]
    assert len(line) == 1
    t = json.loads(line[0][len("traffic: "):])["diag_walk"]
    assert t["sha"] == bench.source_sha("walk.hip+walk_core.hpp")
    assert t[bench.CHUNK_KEY] == chunk
    assert t["fetch_size_bytes_per_launch"] == pytest.approx(100.0 * 1024 * 2.0)
    assert t["write_size_bytes_per_launch"] == pytest.approx(30.0 * 1024 * 1.0)


def test_kernel_trace_summary(tmp_path):
    d = tmp_path / "trace"
    d.mkdir()
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [{"Kernel_Name": "void mcmf::k_diag_gather<false, double>(GatherArgs)",
             "Start_Timestamp": 1000, "End_Timestamp": 1000 + ns} for ns in (2_000_000, 4_000_000)]
    _write_csv(d / "bench_kernel_trace.csv", fields, rows)
    out = bench.summarize(str(d), 0)
    assert "| `k_diag_gather<false, double>` | 2 | 6.00 | 3.000 |" in out


def test_committed_traffic_is_gated_on_sources_and_buffer(tmp_path, monkeypatch):
    chunk = 16 << 30
    entry = {"source": "walk.hip+walk_core.hpp", "sha": bench.source_sha("walk.hip+walk_core.hpp"),
             bench.CHUNK_KEY: chunk, "fetch_size_bytes_per_launch": 7.0, "write_size_bytes_per_launch": 3.0}
    stale = dict(entry, sha="0" * 16)
    action = {k: v for k, v in entry.items() if k != bench.CHUNK_KEY}
    f = tmp_path / "traffic.md"
    f.write_text("text\n\ntraffic: " + json.dumps({"diag_walk": entry, "diag_gather": stale,
                                                    "action_walk": action}) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("diag_walk", chunk) == 10.0
    assert bench.load_traffic("diag_walk", chunk // 2) is None  # other work per launch
    assert bench.load_traffic("diag_gather", chunk) is None     # sources changed
    assert bench.load_traffic("action_walk", None) == 10.0      # no visit buffer involved
    monkeypatch.setattr(bench, "TRAFFIC_FILE", os.path.join(str(tmp_path), "missing.md"))
    assert bench.load_traffic("diag_walk", chunk) is None
