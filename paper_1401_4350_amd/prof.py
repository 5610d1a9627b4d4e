"""Summaries of rocprofv3 output for the profiles/ folder, and the HBM-traffic
record that bench.py reads.

  python -m paper_1401_4350_amd.prof stats <kernel_trace.csv> <out.md> "<command>"
      kernel-trace statistics per (kernel, grid size) as a markdown table;
  python -m paper_1401_4350_amd.prof traffic <fetch_dir> <write_dir> <kernel> <copy_bytes> \
      <out.txt> "<command>"
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of `kernel`, each scaled by
      what the same counter reads for the plain device copy of copy_bytes in
      the same run (the largest copy dispatch), as bytes per launch.

The traffic record carries a hash of the kernel sources; bench.py uses it
only while the sources are unchanged.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("md_kernels.hip", "md_internal.h")]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats_markdown(trace_csv: str, command: str, top: int = 40,
                   keep: tuple[str, ...] = ("k_vertex_lj",)) -> str:
    """Per (kernel, grid) statistics of a kernel trace: the same kernel
    launched on systems of different size is listed once per grid size, so
    the headline launches can be told apart from the others.  The `top` rows
    by total time, then every other row whose name contains one of `keep`."""
    agg: dict[tuple[str, int], list[float]] = {}
    for r in csv.DictReader(open(trace_csv)):
        key = (r["Kernel_Name"], int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"])))
        agg.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = sorted(agg.items(), key=lambda kv: -sum(kv[1]))
    out = [f"Command: `{command}`", "",
           "| kernel | workgroups | calls | total ms | average us | min us | max us |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    rows = rows[:top] + [r for r in rows[top:] if any(s in r[0][0] for s in keep)]
    for (name, wg), d in rows:
        out.append(f"| `{name[:70]}` | {wg} | {len(d)} | {sum(d) / 1e3:.3f} | {sum(d) / len(d):.2f} "
                   f"| {min(d):.2f} | {max(d):.2f} |")
    return "\n".join(out) + "\n"


def _counter(dir_: str, name: str) -> dict[str, list[float]]:
    f = glob.glob(os.path.join(dir_, "*counter_collection.csv"))[0]
    agg: dict[str, list[float]] = {}
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] == name:
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int) -> dict:
    out = {"kernel": kernel, "copy_bytes": copy_bytes, "source_sha": source_hash()}
    for key, d, name in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        agg = _counter(d, name)
        copy_kib = max(v for k, vs in agg.items() if "copyBuffer" in k for v in vs)
        scale = copy_bytes / (copy_kib * 1024.0)
        vals = [v for k, vs in agg.items() if kernel in k for v in vs]
        if not vals:
            raise SystemExit(f"no dispatch of {kernel} in {d}")
        mean_kib = sum(vals) / len(vals)
        out[f"{key}_kib_per_dispatch"] = mean_kib
        out[f"{key}_copy_kib"] = copy_kib
        out[f"{key}_scale"] = scale
        out[f"{key}_bytes"] = mean_kib * 1024.0 * scale
        out[f"{key}_dispatches"] = len(vals)
    out["traffic_bytes"] = out["fetch_bytes"] + out["write_bytes"]
    return out


def write_record(path: str, rec: dict, command: str):
    with open(path, "w") as f:
        f.write(f"command: {command}\n")
        for k, v in rec.items():
            f.write(f"{k}: {v}\n")


def read_record(path: str) -> dict | None:
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        k, _, v = line.partition(":")
        rec[k.strip()] = v.strip()
    return rec


def main(argv):
    if argv[0] == "stats":
        with open(argv[2], "w") as f:
            f.write(stats_markdown(argv[1], argv[3]))
    elif argv[0] == "traffic":
        rec = traffic(argv[1], argv[2], argv[3], int(argv[4]))
        write_record(argv[5], rec, argv[6])
        print(rec)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
