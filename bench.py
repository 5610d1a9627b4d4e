#!/usr/bin/env python3
"""Benchmark of the pair-force MD step on one MI355X.

Workload (default): Lennard-Jones fluid, N = 262144, rho = 0.8, r_c = 2.5,
skin 0.3, dt = 0.001, T = 1.5, FP64.  One timed step is one velocity-Verlet MD
step: half kick + drift + rebuild test, the cell sort and list build when due
(on the device), the force pass and the closing half kick.  The headline value
is pair-force evaluations per second of the vertex decomposition, counting
|E| (half-list entries, the edge method's thread count) per force pass; the
edge decomposition and the FP32-force variants are timed the same way and
reported beside it.

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic FP64 operations of one LJ list entry in the vertex pass (FMA = 2):
# separation 3, r^2 5, 1/r^2 1, (sigma/r)^2 1, ^6 2, force factor 5, the three
# force components accumulated 6.
LJ_ENTRY_FLOPS = 23


def vertex_step_bytes(n: int, pairs: int) -> int:
    """Algorithmic bytes of one vertex force launch with the fused closing
    half kick and the next step's half kick and drift (LJ, FP64): every
    full-list entry read once as a 4-byte index (2|E| entries; the kernel
    itself reads 2-byte region indices in tiles staged in LDS, so its list
    traffic is half of this), per particle the list length (4 B), its own
    position (24 B), the force written (24 B), the velocity read and written
    (48 B), the build position read (24 B) and the drifted position written
    (24 B).  Neighbour positions are gathers that the method assumes are
    cache hits."""
    return 8 * pairs + 148 * n


def patchy_vertex_bytes(n: int, pairs: int) -> int:
    """Algorithmic bytes of one patchy vertex force launch with the closing
    half kick (FP64): every full-list entry read once (4 B, 2|E| entries), per
    particle the list length (4 B), its position (24 B) and orientation
    (32 B), the force and torque written (48 B), the velocity and angular
    momentum read and written (96 B).  Neighbour records are gathers that the
    method assumes are cache hits."""
    return 8 * pairs + 204 * n


def step_bytes(w, pairs: int) -> int:
    """Algorithmic bytes of the vertex force launch of workload w."""
    return vertex_step_bytes(w.n, pairs) if w.pot == "lj" else patchy_vertex_bytes(w.n, pairs)


def edge_pass_bytes(n: int, pairs: int) -> int:
    """Algorithmic bytes of one LJ edge force pass + kick: every half-list
    entry (partner slot 4 B, region index 2 B), per particle the row start
    (4 B), its own position (24 B), forces written (24 B) and read back by the
    kick (24 B), velocity read and written (48 B).  Atomic read-modify-write
    traffic is not counted here."""
    return 6 * pairs + 124 * n


def edge_det_bytes(n: int, pairs: int) -> int:
    """Algorithmic bytes of one deterministic edge pass + kick (LJ): the store
    pass reads every half-list entry (4 B) and writes its force record (32 B);
    the gather reads every full-list entry's edge index (4 B, 2|E|) and that
    edge's record (32 B); per particle the row start (4 B), its own position
    (24 B), the list length (4 B), forces written (24 B) and read back by the
    kick (24 B), velocity read and written (48 B)."""
    return 36 * pairs + 72 * pairs + 128 * n


def newton_pass_bytes(n: int, pairs: int, m: int) -> int:
    """Algorithmic bytes of one Newton-mode pass + kick (LJ): every half-list
    entry (4 B; with LDS accumulation also its 2 B region index), per
    particle the row start (4 B), its own position (24 B), velocity read and
    written (48 B); with m replicas the own force stored (24 B), and the
    combining pass reading F (24 B), reading and clearing every replica
    (2 x 32 B each) and writing F (24 B); with LDS accumulation forces
    written (24 B) and read back by the kick (24 B)."""
    if m == 0:
        return 6 * pairs + 124 * n
    return 4 * pairs + n * (4 + 24 + 48 + 24 + 24 + 64 * m + 24)


def time_mode(md, torch, w, state, mode, prec, steps, warmup, newton_m=0, cell_order="row_major"):
    g = md.System(md.make_params(w, prec, newton_m=newton_m, edge_store=mode == "edge_det",
                                 cell_order=cell_order))
    g.set_state(state.x, state.v, state.q, state.angmom)
    g.build()
    g.forces(mode)
    if warmup:
        g.step(warmup, mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps, mode)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # phase breakdown from a second run with HIP events around every phase
    # (recorded on the system's stream; kept out of the timed run above)
    g.profile(True)
    g.step(steps, mode)
    prof = g.profile_read()
    st = g.stats()
    ke, pe, _ = g.energy()
    g.close()
    wall = t1 - t0
    return dict(mode=mode, prec=prec, wall_s=wall, ms_per_step=1e3 * wall / steps,
                pairs=int(st["pairs"]), rebuilds_total=int(st["rebuilds"]),
                tiles_staged=int(st["tiles_staged"]), tiles_total=int(st["tiles_total"]),
                force_ms_per_step=prof["force_ms"] / steps,
                integrate_ms_per_step=prof["integrate_ms"] / steps,
                rebuild_ms_per_step=prof["rebuild_ms"] / steps,
                energy_per_particle=(ke + pe) / w.n)


def thermostat_us(md, torch, w, state, calls=200, prob=0.01):
    """Average duration of one md_thermostat call (the NVT momentum refresh)
    on the workload, timed over `calls` back-to-back calls."""
    g = md.System(md.make_params(w, "fp64"))
    g.set_state(state.x, state.v, state.q, state.angmom)
    g.build()
    g.thermostat(w.temp, prob, 1, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(calls):
        g.thermostat(w.temp, prob, 1, c + 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    return 1e6 * dt / calls


def cpu_baseline(w, state, pairs, budget_s=20.0):
    """The FP64 oracle (single-threaded C) on the same state: a few velocity-
    Verlet steps, scaled to pair evaluations per second."""
    import oracle
    lj = oracle.LJ(w.eps, w.sigma, w.rcut)
    t0 = time.perf_counter()
    oracle.run(state.x, state.v, state.box, pot="lj", nsteps=1, dt=w.dt, skin=w.skin, lj=lj)
    t1 = time.perf_counter() - t0          # two force evaluations
    k = max(1, min(60, int(budget_s / max(t1 / 2, 1e-6)) - 1))
    t0 = time.perf_counter()
    oracle.run(state.x, state.v, state.box, pot="lj", nsteps=k, dt=w.dt, skin=w.skin, lj=lj)
    dt = time.perf_counter() - t0
    calls = k + 1                           # initial force + one per step
    return {"value": pairs * calls / dt, "unit": "pair evals/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle velocity Verlet, {k} steps ({calls} force passes) of the same "
                      f"N={w.n} state, {dt:.1f} s single-threaded",
            "steps_per_s": k / dt}


def serving_bench(count, rate, steps, max_systems=64):
    """Continuous batching of a Poisson stream of independent requests (N
    log-uniform in [500, 50000], 70 % LJ / 30 % patchy; inputs.serving_requests)
    through md_batch_*, against the single-system path serving the same stream
    one request at a time.  Reports p50/p99 time-to-completion and aggregate
    pair evaluations per second."""
    from paper_1401_4350_amd.inputs import serving_requests
    from paper_1401_4350_amd.serve import (GpuExecutor, Scheduler, SequentialExecutor,
                                           footprint_bytes, summarize)
    reqs = serving_requests(count, rate, seed=0, steps=steps)
    pool = 64 << 30
    out = {"requests": count, "rate_per_s": rate, "steps_per_request": steps,
           "footprint_max_MB": max(footprint_bytes(r) for r in reqs) / 2 ** 20,
           "footprint_mean_MB": sum(footprint_bytes(r) for r in reqs) / count / 2 ** 20}
    for prec, graph in (("fp32", True), ("fp64", True), ("fp32", False)):
        ex = GpuExecutor(max_systems, sum(r.workload.n for r in reqs), pool, "vertex", prec, 64,
                         use_graph=graph)
        rep = Scheduler(ex, pool, max_systems).run(reqs)
        s = summarize(rep)
        s["captures"] = ex.batch.info()["captures"]
        ex.close()
        out[f"batched_{prec}" + ("" if graph else "_direct_launches")] = s
    for prec in ("fp64", "fp32"):
        ex = SequentialExecutor("vertex", prec)
        out[f"single_{prec}"] = summarize(Scheduler(ex, pool, 1).run(reqs))
    b, a = out["batched_fp32"], out["single_fp64"]
    out["throughput_gain_vs_single_fp64"] = b["pair_evals_per_s"] / a["pair_evals_per_s"]
    return out


def crossover_bench(torch, steps=100, warmup=20, which=("lj", "patchy", "patchy_paper")):
    """Vertex against edge over system size and density, for each potential:
    per point the MD step and the force pass of each decomposition (FP64).
    Sizes N = 2^10 .. 2^20 at each potential's own density (LJ 0.8, patchy
    0.5), and densities 0.1, 0.3, 0.5, 0.8 at N = 2^17 (0.1, 0.3, 0.5, the
    paper's, for its two-patch model)."""
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS, make_state
    points = []
    for pot, base in (("lj", "lj_many"), ("patchy", "patchy"), ("patchy_paper", "patchy_paper")):
        if pot not in which:
            continue
        b = WORKLOADS[base]
        grid = [(2 ** e, b.rho) for e in range(10, 21, 2)]
        dens = (0.1, 0.3, 0.5) if pot == "patchy_paper" else (0.1, 0.3, 0.5, 0.8)
        grid += [(2 ** 17, r) for r in dens]
        for n, rho in grid:
            w = b.with_(n=n, rho=rho)
            if w.box <= 2 * w.rv:
                continue
            st = make_state(w, 1)
            row = {"pot": pot, "n": n, "rho": rho}
            for mode in ("vertex", "edge"):
                r = time_mode(md, torch, w, st, mode, "fp64", steps, warmup)
                row[f"{mode}_step_us"] = 1e3 * r["ms_per_step"]
                row[f"{mode}_force_us"] = 1e3 * r["force_ms_per_step"]
                row["pairs"] = r["pairs"]
            row["edge_over_vertex_force"] = row["vertex_force_us"] / row["edge_force_us"]
            row["faster"] = "edge" if row["edge_step_us"] < row["vertex_step_us"] else "vertex"
            points.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return points


def locality_bench(torch, steps=100, warmup=20):
    """Slot order of the cells against the force pass (FP64): row-major cells
    with LDS-staged tiles (the default), and row-major, Morton and Hilbert
    cell orders with every neighbour gathered from global memory, for the LJ
    and the patchy workload, vertex and edge."""
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS, make_state
    rows = []
    for base in ("lj_many", "patchy"):
        w = WORKLOADS[base]
        st = make_state(w, 1)
        for order in ("row_major", "row_major_gather", "morton", "hilbert"):
            row = {"workload": base, "cell_order": order}
            for mode in ("vertex", "edge"):
                r = time_mode(md, torch, w, st, mode, "fp64", steps, warmup, cell_order=order)
                row[f"{mode}_step_us"] = 1e3 * r["ms_per_step"]
                row[f"{mode}_force_us"] = 1e3 * r["force_ms_per_step"]
                row["tiles_staged"] = r["tiles_staged"]
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return rows


def nvt_bench(torch, target=0.3, steps=6000, every=100, prob=0.1, report=500):
    """The two-patch workload (131 072 particles, rho = 0.5, prepared at
    k_B T = 0.15) run in NVT at k_B T = `target`: blocks of `every` vertex
    steps, each followed by md_thermostat with probability `prob`.  Reports
    the kinetic temperature 2 E_kin / (6 N) (three translational and three
    rotational degrees of freedom per particle) every `report` steps, the
    potential energy per particle, and the MD steps per second with the
    thermostat calls included."""
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS, make_state
    w = WORKLOADS["patchy_paper"]
    st = make_state(w, 1)
    g = md.System(md.make_params(w, "fp64"))
    g.set_state(st.x, st.v, st.q, st.angmom)
    g.build()
    g.forces("vertex")
    rows = []
    ke, pe, _ = g.energy()
    rows.append({"step": 0, "kT": 2 * ke / (6 * w.n), "e_pot": pe / w.n})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, timed = 0, 0.0
    while done < steps:
        t1 = time.perf_counter()
        g.step(every, "vertex")
        g.thermostat(target, prob, 7, done // every)
        torch.cuda.synchronize()
        timed += time.perf_counter() - t1
        done += every
        if done % report == 0:
            ke, pe, _ = g.energy()
            rows.append({"step": done, "kT": 2 * ke / (6 * w.n), "e_pot": pe / w.n})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    g.close()
    return {"workload": w.name, "n": w.n, "target_kT": target, "thermostat_every": every,
            "prob": prob, "md_steps_per_s": steps / timed, "samples": rows,
            "wall_s": time.perf_counter() - t0}


def drift_bench(torch, steps=10000, every=500):
    """Total-energy drift of the 1M-particle LJ workload (dt = 0.005) over
    `steps` velocity-Verlet steps for each precision variant: slope of a
    least-squares line through E(t) sampled every `every` steps, per particle
    and per 10 000 steps, plus the rms fluctuation about that line."""
    import numpy as np
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS, make_state
    w = WORKLOADS["lj_precision"]
    st = make_state(w, 1)
    out = {}
    for prec in ("fp64", "fp32", "fp32_kahan"):
        g = md.System(md.make_params(w, prec))
        g.set_state(st.x, st.v)
        g.build()
        g.forces("vertex")
        ts, es = [], []
        t_gpu = 0.0
        for k in range(0, steps + 1, every):
            if k:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.step(every, "vertex")
                t_gpu += time.perf_counter() - t0
            ke, pe, _ = g.energy()
            ts.append(k)
            es.append((ke + pe) / w.n)
        g.close()
        ts, es = np.array(ts, float), np.array(es)
        slope, icpt = np.polyfit(ts, es, 1)
        resid = es - (slope * ts + icpt)
        out[prec] = {"drift_per_particle_per_10k_steps": slope * 1e4,
                     "rms_fluctuation_per_particle": float(np.sqrt((resid ** 2).mean())),
                     "e0_per_particle": float(es[0]), "ms_per_step": 1e3 * t_gpu / steps}
        print(json.dumps({prec: out[prec]}), file=sys.stderr, flush=True)
    return {"workload": w.name, "n": w.n, "dt": w.dt, "steps": steps, "variants": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="lj_many")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "fp32_kahan"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the headline (vertex) and edge modes")
    ap.add_argument("--serving-requests", type=int, default=48,
                    help="requests of the serving comparison (0: skip it)")
    ap.add_argument("--serving-rate", type=float, default=400.0)
    ap.add_argument("--serving-steps", type=int, default=1000)
    ap.add_argument("--crossover", action="store_true",
                    help="print the vertex/edge crossover sweep instead of the headline line")
    ap.add_argument("--crossover-pots", default="lj,patchy,patchy_paper",
                    help="potentials of the crossover sweep (comma-separated)")
    ap.add_argument("--locality", action="store_true",
                    help="cell orders (row-major staged / gathered, Morton, Hilbert) instead of the bench line")
    ap.add_argument("--nvt", action="store_true",
                    help="print the NVT run of the two-patch model with the thermostat instead")
    ap.add_argument("--drift", action="store_true",
                    help="print the energy-drift study of the precision variants instead")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (for counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs one system per GPU on a single GPU; "
                                   "--gpus must be 1 (multi-GPU sharding is a design note "
                                   "only)"}))
        sys.exit(2)

    import torch
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS, make_state

    torch.cuda.set_device(0)
    if args.crossover:
        pots = tuple(args.crossover_pots.split(","))
        print(json.dumps({"crossover": crossover_bench(torch, which=pots)}), flush=True)
        return
    if args.drift:
        print(json.dumps({"drift": drift_bench(torch)}), flush=True)
        return
    if args.nvt:
        print(json.dumps({"nvt": nvt_bench(torch)}), flush=True)
        return
    if args.locality:
        print(json.dumps({"locality": locality_bench(torch)}), flush=True)
        return
    w = WORKLOADS[args.workload]
    state = make_state(w, args.seed)

    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    runs = {}
    for mode in ("vertex", "edge"):
        runs[mode] = time_mode(md, torch, w, state, mode, args.prec, args.steps, args.warmup)
    variants = {}
    if not args.no_variants and args.prec == "fp64":
        for mode in ("vertex", "edge"):
            variants[f"{mode}_fp32"] = time_mode(md, torch, w, state, mode, "fp32",
                                                 args.steps, args.warmup)
    if not args.no_variants:
        variants["edge_det"] = time_mode(md, torch, w, state, "edge_det", args.prec,
                                         args.steps, args.warmup)
    newton = {}
    if not args.no_variants and w.pot == "lj":
        for m in (0, 1, 4, 16):
            newton[m] = time_mode(md, torch, w, state, "newton", args.prec, args.steps,
                                  args.warmup, newton_m=m)

    head = runs["vertex"]
    pairs = head["pairs"]
    value = pairs / (head["ms_per_step"] * 1e-3)
    nb = step_bytes(w, pairs)
    t_kernel = head["force_ms_per_step"] * 1e-3
    achieved = nb / t_kernel / 1e9

    def summary(r, nbytes):
        return {"ms_per_step": r["ms_per_step"], "md_steps_per_s": 1e3 / r["ms_per_step"],
                "pair_evals_per_s": r["pairs"] / (r["ms_per_step"] * 1e-3),
                "force_pass_us": 1e3 * r["force_ms_per_step"],
                "integrate_us": 1e3 * r["integrate_ms_per_step"],
                "rebuild_us_amortised": 1e3 * r["rebuild_ms_per_step"],
                "force_pass_GBps": nbytes / (r["force_ms_per_step"] * 1e-3) / 1e9,
                "pairs": r["pairs"], "list_builds": r["rebuilds_total"],
                "tiles_staged": r["tiles_staged"], "tiles_total": r["tiles_total"],
                "energy_per_particle": r["energy_per_particle"]}

    modes = {"vertex": summary(runs["vertex"], nb),
             "edge": summary(runs["edge"], edge_pass_bytes(w.n, runs["edge"]["pairs"]))}
    for k, r in variants.items():
        if k.startswith("vertex"):
            nbv = step_bytes(w, r["pairs"])
        elif k == "edge_det":
            nbv = edge_det_bytes(w.n, r["pairs"])
        else:
            nbv = edge_pass_bytes(w.n, r["pairs"])
        modes[k] = summary(r, nbv)
    for m, r in newton.items():
        modes[f"newton_m{m}"] = summary(r, newton_pass_bytes(w.n, r["pairs"], m))
    if not args.no_variants:
        modes["thermostat_call_us"] = thermostat_us(md, torch, w, state)
    modes["edge_over_vertex_speedup"] = runs["vertex"]["ms_per_step"] / runs["edge"]["ms_per_step"]

    out = {
        "metric": "pair-force evals/s (%s MD step, vertex decomposition)" % (
            "LJ" if w.pot == "lj" else "patchy"),
        "value": value,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "md_steps_per_s": 1e3 / head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32 pair maths, f64 sums and integration",
        "data": "synthetic",
        "config": {"workload": w.name, "pot": w.pot, "n": w.n, "rho": w.rho, "temp": w.temp,
                   "rcut": w.rcut, "skin": w.skin, "dt": w.dt, "prec": args.prec,
                   "max_neighbors": w.list_capacity(), "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("k_vertex_lj<FP64, closing kick + next kick and drift>"
                                if w.pot == "lj" else "k_vertex_patchy<FP64, closing kick>"),
                     "bytes_per_launch": nb, "avg_launch_us": t_kernel * 1e6,
                     # the same kernel against the FP64 vector rate: 2|E| list
                     # entries of LJ_ENTRY_FLOPS each per launch (LJ only: a
                     # patchy pair's operation count depends on its geometry)
                     "valu": ({"achieved": 2 * pairs * LJ_ENTRY_FLOPS / t_kernel / 1e12,
                               "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": 2 * pairs * LJ_ENTRY_FLOPS / t_kernel / 1e12
                               / FP64_VECTOR_PEAK_TFLOPS} if w.pot == "lj" else None)},
        "modes": modes,
    }
    # HBM traffic of the same kernel from the committed FETCH_SIZE / WRITE_SIZE
    # record, used only while the kernel sources are the ones it was taken on
    from paper_1401_4350_amd import prof
    rec = prof.read_record(os.path.join(ROOT, "profiles", f"traffic_{w.name}_{args.prec}.txt"))
    if rec and rec.get("source_sha") == prof.source_hash():
        out["roofline"]["traffic"] = float(rec["traffic_bytes"])
        out["roofline"]["traffic_over_algorithmic"] = float(rec["traffic_bytes"]) / nb
    if args.serving_requests > 0:
        out["serving"] = serving_bench(args.serving_requests, args.serving_rate,
                                       args.serving_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, state, pairs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
