"""Host logic of the measurement tooling (no GPU): the kernel-trace summary,
the HBM-traffic record that bench.py reads, and bench.py's refusal of more
than one GPU.  The rocprofv3 output files are written here by hand in the
columns rocprofv3 uses."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_1401_4350_amd import prof

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_trace(path, rows):
    cols = ["Kernel_Name", "Grid_Size_X", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        t = 1_000_000
        for name, grid, wg, us in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size_X": grid, "Workgroup_Size_X": wg,
                        "Start_Timestamp": t, "End_Timestamp": t + int(us * 1000)})
            t += int(us * 1000) + 500


def write_counters(dir_, name, rows):
    os.makedirs(dir_, exist_ok=True)
    with open(os.path.join(dir_, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, value in rows:
            w.writerow({"Kernel_Name": kernel, "Counter_Name": name, "Counter_Value": value})


def table_row(md, key):
    for line in md.splitlines():
        if key in line:
            return [c.strip() for c in line.strip().strip("|").split("|")]
    raise AssertionError(key)


def test_stats_separates_full_launches(tmp_path):
    """Calls shorter than half the longest (a rebuild step with no rebuild
    due, a fused launch that finds its lists stale) are counted apart."""
    f = tmp_path / "trace.csv"
    k = "void md::k_vertex_lj<0, 4, true, false, true>(md::Sys)"
    write_trace(f, [(k, 4096 * 256, 256, 40.0), (k, 4096 * 256, 256, 44.0),
                    (k, 4096 * 256, 256, 2.0), ("md::k_build(md::Sys)", 1024 * 256, 256, 1.0),
                    ("md::k_build(md::Sys)", 1024 * 256, 256, 200.0)])
    md = prof.stats_markdown(str(f), "cmd")
    assert md.startswith("Command: `cmd`")
    r = table_row(md, "k_vertex_lj")
    # workgroups, calls, total ms, average, min, max, full calls, full average
    assert r[1] == "4096" and r[2] == "3"
    assert float(r[3]) == pytest.approx(0.086)
    assert float(r[4]) == pytest.approx(86.0 / 3, abs=0.01)
    assert r[7] == "2" and float(r[8]) == pytest.approx(42.0)
    b = table_row(md, "k_build")
    assert b[1] == "1024" and b[7] == "1" and float(b[8]) == pytest.approx(200.0)


def test_traffic_scales_by_the_copy_and_drops_skipped_launches(tmp_path):
    """FETCH_SIZE reads half a device copy's bytes and WRITE_SIZE all of
    them; the record scales each kernel reading by the copy's, over the full
    launches only."""
    k = "void md::k_vertex_lj<0, 4, true, false, true>(md::Sys)"
    copy = 1 << 20
    write_counters(tmp_path / "f", "FETCH_SIZE",
                   [("__amd_rocclr_copyBuffer", copy / 2048), (k, 1000.0), (k, 1200.0), (k, 3.0)])
    write_counters(tmp_path / "w", "WRITE_SIZE",
                   [("__amd_rocclr_copyBuffer", copy / 1024), (k, 500.0), (k, 2.0)])
    rec = prof.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_vertex_lj<0, 4, true, false, true>",
                       copy)
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_dispatches"] == 2 and rec["write_dispatches"] == 1
    assert rec["fetch_bytes"] == pytest.approx(1100.0 * 1024 * 2)
    assert rec["write_bytes"] == pytest.approx(500.0 * 1024)
    assert rec["traffic_bytes"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["source_sha"] == prof.source_hash()
    out = tmp_path / "rec.txt"
    prof.write_record(str(out), rec, "cmd")
    back = prof.read_record(str(out))
    assert back["command"] == "cmd"
    assert float(back["traffic_bytes"]) == pytest.approx(rec["traffic_bytes"])


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in line["error"]
