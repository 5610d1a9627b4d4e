"""Summaries of rocprofv3 output for the profiles/ folder, and the HBM-traffic
record that bench.py reads.

  python -m paper_1401_4350_amd.prof stats <kernel_trace.csv> <out.md> "<command>"
      kernel-trace statistics per (kernel, grid size) as a markdown table;
  python -m paper_1401_4350_amd.prof traffic <fetch_dir> <write_dir> <kernel> <copy_bytes> \
      <out.txt> "<command>"
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of `kernel`, each scaled by
      what the same counter reads for the plain device copy of copy_bytes in
      the same run (the largest copy dispatch), as bytes per launch.

  python -m paper_1401_4350_amd.prof counters <out.md> "<command>" "<kernel>|<kernel>..." <dir>...
      per-dispatch means of every counter found in the pmc output folders,
      for the dispatches of each named kernel at its largest grid (the
      full-size launches), with the resources of the dispatch (VGPRs, LDS)
      and a few ratios derived from them.

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
           "Full launches: the calls that took at least half the longest one (launches that "
           "return at once -- a rebuild step with no rebuild due, a fused step launch whose "
           "lists are stale -- are the others).", "",
           "| kernel | workgroups | calls | total ms | average us | min us | max us "
           "| full calls | full average us |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    rows = rows[:top] + [r for r in rows[top:] if any(s in r[0][0] for s in keep)]
    for (name, wg), d in rows:
        full = [x for x in d if x >= 0.5 * max(d)]
        out.append(f"| `{name[:70]}` | {wg} | {len(d)} | {sum(d) / 1e3:.3f} | {sum(d) / len(d):.2f} "
                   f"| {min(d):.2f} | {max(d):.2f} | {len(full)} | {sum(full) / len(full):.2f} |")
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
        # full launches only (a fused step launch that finds its lists stale
        # returns at once and moves almost nothing)
        vals = [v for v in vals if v >= 0.5 * max(vals)]
        mean_kib = sum(vals) / len(vals)
        out[f"{key}_kib_per_dispatch"] = mean_kib
        out[f"{key}_copy_kib"] = copy_kib
        out[f"{key}_scale"] = scale
        out[f"{key}_bytes"] = mean_kib * 1024.0 * scale
        out[f"{key}_dispatches"] = len(vals)
    out["traffic_bytes"] = out["fetch_bytes"] + out["write_bytes"]
    return out


def counters_markdown(dirs: list[str], kernels: list[str], command: str) -> str:
    """Mean value per dispatch of each counter, per kernel, from one or more
    rocprofv3 --pmc folders.  A kernel is every full name that contains the
    given text, at its largest grid (the full-size launches); dispatches that
    took less than half the longest one of that kernel and grid are left out
    (launches that return at once when no list rebuild is due)."""
    rows = []
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows.extend(csv.DictReader(open(f)))

    def dur(r):
        return int(r["End_Timestamp"]) - int(r["Start_Timestamp"])

    out = [f"Command: `{command}`", "",
           "Mean per dispatch over the full-length dispatches of the kernel at its largest "
           "grid (each pass is its own run; the counters of one dispatch come from one pass).",
           ""]
    for k in kernels:
        groups: dict[tuple[str, int], list[dict]] = {}
        for r in rows:
            if k in r["Kernel_Name"]:
                groups.setdefault((r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0)), []).append(r)
        if not groups:
            out.append(f"## `{k}`: no dispatch found\n")
            continue
        names = sorted({name for name, _ in groups})
        for name in names:
            grid = max(g for nm, g in groups if nm == name)
            sel = groups[(name, grid)]
            longest = {}
            for r in sel:  # per pass (a counter set), the longest dispatch
                longest[r["Counter_Name"]] = max(longest.get(r["Counter_Name"], 0), dur(r))
            vals: dict[str, list[float]] = {}
            for r in sel:
                if dur(r) >= 0.5 * longest[r["Counter_Name"]]:
                    vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            r = sel[0]
            out.append(f"## `{name[:100]}`")
            out.append("")
            out.append(f"grid {grid} threads, workgroup {r['Workgroup_Size']}, LDS "
                       f"{r['LDS_Block_Size']} B, VGPR {r['VGPR_Count']} (+{r['Accum_VGPR_Count']} "
                       f"AGPR), SGPR {r['SGPR_Count']}")
            out.append("")
            out.append("| counter | mean per dispatch | dispatches |")
            out.append("|---|---:|---:|")
            m = {c: sum(v) / len(v) for c, v in vals.items()}
            for c in sorted(m):
                out.append(f"| {c} | {m[c]:.6g} | {len(vals[c])} |")
            derived = []
            if m.get("SQ_ACTIVE_INST_LDS") and "SQ_LDS_BANK_CONFLICT" in m:
                derived.append(("LDS bank-conflict cycles / LDS active cycles",
                                m["SQ_LDS_BANK_CONFLICT"] / m["SQ_ACTIVE_INST_LDS"]))
            if m.get("SQ_WAVE_CYCLES"):
                for c, what in (("SQ_WAIT_INST_ANY", "waiting on a dependency"),
                                ("SQ_ACTIVE_INST_VALU", "issuing VALU"),
                                ("SQ_ACTIVE_INST_LDS", "issuing LDS"),
                                ("SQ_WAIT_INST_LDS", "waiting on LDS")):
                    if c in m:
                        derived.append((f"{c} / SQ_WAVE_CYCLES ({what})", m[c] / m["SQ_WAVE_CYCLES"]))
            if m.get("SQ_WAVES"):
                for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_SALU",
                          "SQ_INSTS_LDS_ATOMIC"):
                    if c in m:
                        derived.append((f"{c} per wave", m[c] / m["SQ_WAVES"]))
            if derived:
                out.append("")
                out.append("| derived | value |")
                out.append("|---|---:|")
                for nm, v in derived:
                    out.append(f"| {nm} | {v:.4g} |")
            out.append("")
    return "\n".join(out) + "\n"


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
    elif argv[0] == "counters":
        with open(argv[1], "w") as f:
            f.write(counters_markdown(argv[4:], argv[3].split("|"), argv[2]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
