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

Protocol (the paper's Methods: each algorithm timed over the same number of
steps, after the system has decorrelated, five repetitions): for each seed
(1 .. 5 by default) the lattice state is equilibrated on the GPU for a fixed
number of vertex steps, untimed and independent of --warmup; both
decompositions then start from that snapshot, run W untimed steps and K timed
ones.  The headline is the mean over the seeds, with its standard deviation.

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


def vertex_force_bytes(n: int, pairs: int) -> int:
    """Algorithmic bytes of one LJ vertex force pass: every full-list entry
    read once as a 4-byte index (2|E| entries), per particle the list length
    (4 B), its own position (24 B) and its force written (24 B); neighbour
    positions are gathers the method assumes are cache hits.  The headline
    kernel also does the closing half kick and the next step's half kick and
    drift (vertex_step_bytes), whose traffic this count leaves out."""
    return 8 * pairs + 52 * n


def edge_force_bytes(n: int, pairs: int) -> int:
    """Algorithmic bytes of one LJ edge force pass: every half-list entry read
    once as a 4-byte index, per particle the row start (4 B), its position
    (24 B), its force zeroed (24 B) and written (24 B).  Atomic
    read-modify-write traffic is counted in the atomic roofline instead."""
    return 4 * pairs + 76 * n


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


def equilibrate(md, torch, w, seed, steps):
    """make_state(w, seed) advanced by `steps` FP64 vertex steps on the GPU
    (untimed): the snapshot both decompositions start from."""
    from types import SimpleNamespace
    from paper_1401_4350_amd.inputs import make_state
    s = make_state(w, seed)
    if steps <= 0:
        return s
    g = md.System(md.make_params(w, "fp64"))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    g.step(steps, "vertex")
    out = g.get_state()
    g.close()
    return SimpleNamespace(x=out["x"], v=out["v"], q=out.get("q"), angmom=out.get("angmom"),
                           box=s.box, seed=seed, equilibration_steps=steps)


def default_equilibration(w) -> int:
    """Untimed steps before every timed window: 2 000 for the LJ fluids,
    10 000 for patchy particles (bonds form over ~10^4 steps)."""
    return 2000 if w.pot == "lj" else 10000


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
                pairs=int(st["pairs"]), nonzero_pairs=int(st["nonzero_pairs"]),
                rebuilds_total=int(st["rebuilds"]),
                tiles_staged=int(st["tiles_staged"]), tiles_total=int(st["tiles_total"]),
                force_ms_per_step=prof["force_ms"] / steps,
                kick_ms_per_step=prof["kick_ms"] / steps,
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, state, pairs, budget_s=20.0):
    """The FP64 oracle (plain C, per-particle OpenMP loop) on the same
    snapshot: velocity-Verlet steps at one thread and at every host core,
    scaled to pair evaluations per second (|E| per force call, as the GPU
    headline)."""
    import oracle
    kw = dict(dt=w.dt, skin=w.skin, mass=w.mass)
    if w.pot == "lj":
        kw.update(pot="lj", lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    else:
        kw.update(pot="patchy", inertia=w.inertia, q=state.q, angmom=state.angmom,
                  patchy=oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p,
                                       w=w.patch_w, delta=w.patch_delta, rpc=w.patch_rcut,
                                       model=1 if w.patch_model == "polar2" else 0))
    cores = os.cpu_count() or 1
    out = {}
    for threads in (1, cores):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.run(state.x, state.v, state.box, nsteps=1, **kw)
        t1 = time.perf_counter() - t0          # two force evaluations and a list build
        share = budget_s * (0.7 if threads == 1 else 0.3)
        k = max(1, min(30, int(share / max(t1 / 2, 1e-6)) - 1))
        t0 = time.perf_counter()
        oracle.run(state.x, state.v, state.box, nsteps=k, **kw)
        dt = time.perf_counter() - t0
        calls = k + 1                           # initial force + one per step
        out[threads] = {"value": pairs * calls / dt, "steps": k, "force_calls": calls,
                        "seconds": dt, "steps_per_s": k / dt}
    oracle.set_threads(cores)
    a, one = out[cores], out[1]
    return {"value": a["value"], "unit": "pair evals/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle velocity Verlet on the same equilibrated N={w.n} snapshot: "
                      f"{a['steps']} steps ({a['force_calls']} force passes) in {a['seconds']:.1f} s "
                      f"at {cores} threads, {one['steps']} steps in {one['seconds']:.1f} s at 1 thread",
            "cpu_model": cpu_model(), "nproc": cores, "steps_per_s": a["steps_per_s"],
            "single_thread": {"value": one["value"], "steps_per_s": one["steps_per_s"],
                              "cores": 1},
            "speedup_all_cores_over_one": a["value"] / one["value"]}


def probe_rates(torch):
    """Measured ceilings beside the published peaks (libmdprobe.so): HBM
    streaming read and device copy (GB/s), device-scope FP64 atomic adds at
    scattered and at coalesced addresses, and LDS FP64 atomic adds at
    scattered addresses (adds/s).  Each is the best of three launches timed
    with events on the current stream."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1401_4350_amd", "libmdprobe.so"))
    lib.probe_global_atomics.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.probe_lds_atomics.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.probe_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p]
    stream = torch.cuda.current_stream()

    def best(launch, reps=3):
        times = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rc = launch()
            b.record(stream)
            if rc != 0:
                raise RuntimeError(f"probe launch failed ({rc})")
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) * 1e-3)
        return min(times[1:])

    out = {}
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(8192 * 256, dtype=torch.int32, device="cuda")
    t = best(lambda: lib.probe_read(src.data_ptr(), nbytes, sink.data_ptr(), 8192,
                                    stream.cuda_stream))
    out["hbm_read_GBps"] = nbytes / t / 1e9

    def copy():
        dst.copy_(src)
        return 0
    out["hbm_copy_GBps"] = 2 * nbytes / best(copy) / 1e9
    del src, dst, sink
    # forces of 262 144 particles: 32-byte records, three of the four words used
    slots = 4 * 262144
    buf = torch.zeros(slots, dtype=torch.float64, device="cuda")
    threads, ops = 262144, 64
    for kind, name in ((0, "global_fp64_atomics_scattered_per_s"),
                       (1, "global_fp64_atomics_coalesced_per_s")):
        t = best(lambda: lib.probe_global_atomics(buf.data_ptr(), slots, threads, ops, kind,
                                                  stream.cuda_stream))
        out[name] = threads * ops / t
    lslots, blocks, ops = 5000, 4096, 64  # a 40 KB accumulator, as a staged tile region
    lout = torch.empty(blocks * lslots, dtype=torch.float64, device="cuda")
    for kind, name in ((0, "lds_fp64_atomics_scattered_per_s"),
                       (1, "lds_fp64_atomics_distinct_per_s"),
                       (2, "lds_fp64_plain_rmw_distinct_per_s")):
        t = best(lambda: lib.probe_lds_atomics(lout.data_ptr(), lslots, blocks, ops, kind,
                                               stream.cuda_stream))
        out[name] = blocks * 256 * ops / t
    return out


def atomic_roofline(w, r, probes, lj):
    """The edge pass against its atomic ceiling: the atomic adds its non-zero
    pairs need at the least (three per pair for the partner's force: into the
    tile's LDS accumulator for LJ, device-scope at scattered addresses for
    patchy particles), at the probe-measured rate, over the pass's duration.
    frac near 1 means the pass runs at the atomic rate."""
    nz = r["nonzero_pairs"]
    t = r["force_ms_per_step"] * 1e-3
    if lj:
        kind, rate = "LDS FP64 atomic add, scattered", probes["lds_fp64_atomics_scattered_per_s"]
    else:
        kind, rate = ("device-scope FP64 atomic add, scattered",
                      probes["global_fp64_atomics_scattered_per_s"])
    adds = 3 * nz
    bound = adds / rate
    return {"kind": kind, "adds_per_pass": adds, "measured_rate_per_s": rate,
            "achieved_per_s": adds / t, "bound_us": bound * 1e6, "frac": bound / t}


def dense_bench(md, torch, args):
    """The dense LJ fluid (N = 262 144, rho = 1.0, r_c = 3.0, about 150
    neighbours within r_v): vertex and edge force passes of the FP64 MD step
    from one equilibrated snapshot, with their algorithmic bytes."""
    from paper_1401_4350_amd.inputs import WORKLOADS
    w = WORKLOADS["lj_many_dense"]
    snap = equilibrate(md, torch, w, args.seed, default_equilibration(w))
    out = {"workload": w.name, "n": w.n, "rho": w.rho, "rcut": w.rcut}
    for mode, fn in (("vertex", vertex_force_bytes), ("edge", edge_force_bytes)):
        r = time_mode(md, torch, w, snap, mode, "fp64", args.steps, args.warmup)
        nb = fn(w.n, r["pairs"])
        t = r["force_ms_per_step"] * 1e-3
        out[mode] = {"ms_per_step": r["ms_per_step"], "force_pass_us": t * 1e6,
                     "bytes_per_launch": nb, "GBps": nb / t / 1e9,
                     "frac": nb / t / 1e9 / HBM_PEAK_GBS, "pairs": r["pairs"],
                     "nonzero_pairs": r["nonzero_pairs"],
                     "pair_evals_per_s": r["pairs"] / (r["ms_per_step"] * 1e-3)}
    out["edge_over_vertex_speedup"] = out["vertex"]["ms_per_step"] / out["edge"]["ms_per_step"]
    return out


def serving_bench(count, steps, occupancy=0.8, max_systems=64, accuracy_sample=4):
    """Continuous batching of a Poisson stream of independent requests (N
    log-uniform in [500, 50000], 70 % LJ / 30 % patchy; inputs.serving_requests)
    through md_batch_*, against the single-system path serving the same stream
    one request at a time.

    Load: the stream is first served saturated (every request present at
    t = 0) by the batched FP32 path, which gives the saturated aggregate rate
    T_sat (pair evals/s) and the mean work per request E[|E| x steps]; the
    arrival rate is then lambda = occupancy * T_sat / E[work] and every path
    serves the same stream at that rate (the draws do not depend on the rate,
    only the gaps scale).  Reports p50/p99 time-to-completion and aggregate
    pair evaluations per second, and the FP32 force error against the oracle
    on a few requests' initial states (the batched vertex step is bitwise the
    single-system one, so this is also the batched accuracy)."""
    import numpy as np
    import oracle
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import make_state, serving_requests
    from paper_1401_4350_amd.serve import (GpuExecutor, Scheduler, SequentialExecutor,
                                           footprint_bytes, summarize)
    pool = 64 << 30
    probe = serving_requests(count, 1.0, seed=0, steps=steps)
    max_particles = sum(r.workload.n for r in probe)

    def batched(reqs, prec, graph=True):
        ex = GpuExecutor(max_systems, max_particles, pool, "vertex", prec, 64, use_graph=graph)
        rep = Scheduler(ex, pool, max_systems).run(reqs)
        s = summarize(rep)
        info = ex.batch.info()
        s["captures"], s["regrids"] = info["captures"], info["regrids"]
        ex.close()
        return s, rep

    # saturated run: every request at t = 0
    sat_reqs = [type(r)(rid=r.rid, arrival=0.0, workload=r.workload, seed=r.seed) for r in probe]
    sat, sat_rep = batched(sat_reqs, "fp32")
    t_sat = sat["pair_evals_per_s"]
    work = [rec.pairs * rec.steps for rec in sat_rep.records if rec.status == "done"]
    e_work = sum(work) / len(work)
    lam = occupancy * t_sat / e_work
    reqs = serving_requests(count, lam, seed=0, steps=steps)
    out = {"requests": count, "steps_per_request": steps,
           "load": {"occupancy": occupancy, "saturated_pair_evals_per_s": t_sat,
                    "mean_work_pair_evals": e_work, "rate_per_s": lam,
                    "rule": "rate = occupancy * T_sat / E[|E| x steps], T_sat from the "
                            "saturated batched FP32 run of the same requests"},
           "saturated_batched_fp32": sat,
           "footprint_max_MB": max(footprint_bytes(r) for r in reqs) / 2 ** 20,
           "footprint_mean_MB": sum(footprint_bytes(r) for r in reqs) / count / 2 ** 20,
           "span_of_arrivals_s": reqs[-1].arrival}
    for prec, graph in (("fp32", True), ("fp64", True), ("fp32", False)):
        s, _ = batched(reqs, prec, graph)
        out[f"batched_{prec}" + ("" if graph else "_direct_launches")] = s
    for prec in ("fp64", "fp32"):
        ex = SequentialExecutor("vertex", prec)
        out[f"single_{prec}"] = summarize(Scheduler(ex, pool, 1).run(reqs))
    b, a = out["batched_fp32"], out["single_fp64"]
    out["throughput_gain_vs_single_fp64"] = b["pair_evals_per_s"] / a["pair_evals_per_s"]
    # accuracy of the two sides of the comparison, per request, against the oracle
    acc = {"fp32": [], "fp64": []}
    for r in reqs[:accuracy_sample]:
        w = r.workload
        st = make_state(w, r.seed)
        if w.pot == "lj":
            F, _, _, A = oracle.lj_forces(st.x, st.box, oracle.LJ(w.eps, w.sigma, w.rcut),
                                          with_abs=True)
            scale = {"fp32": A, "fp64": A}
        else:  # FP32: per-term scale (its rounding), FP64: per-pair scale (the tighter)
            pp = oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                               delta=w.patch_delta, rpc=w.patch_rcut)
            F, _, _, _, FA, _ = oracle.patchy_forces(st.x, st.q, st.box, pp, with_abs=True)
            scale = {"fp32": FA, "fp64": oracle.patchy_pair_scales(st.x, st.q, st.box, pp)[0]}
        for prec in acc:
            g = md.System(md.make_params(w, prec))
            g.set_state(st.x, st.v, st.q, st.angmom)
            g.build()
            g.forces("vertex")
            f = g.get_state()["f"]
            g.close()
            acc[prec].append(float(np.max(np.abs(f - F) / np.maximum(scale[prec], 1e-300))))
    out["force_rel_err_vs_oracle"] = {
        "requests": [r.rid for r in reqs[:accuracy_sample]],
        "fp32_max": max(acc["fp32"]), "fp64_max": max(acc["fp64"]),
        "bars": {"fp32": 1e-5, "fp64": 1e-10},
        "measure": "max over particles and components of |F - F*| / the oracle's tolerance "
                   "scale (LJ: sum_j |F_ij|; patchy: per-term sums for FP32, per-pair for "
                   "FP64), at each request's initial state"}
    return out


def crossover_bench(torch, steps=100, warmup=20, which=("lj", "patchy", "patchy_paper"),
                    equil=1000):
    """Vertex against edge over system size and density, for each potential:
    per point the MD step and the force pass of each decomposition (FP64),
    both from one snapshot equilibrated for `equil` vertex steps.  Sizes
    N = 2^10 .. 2^20 at each potential's own density (LJ 0.8, patchy 0.5), and
    densities 0.1, 0.3, 0.5, 0.8 at N = 2^17 (0.1, 0.3, 0.5, the paper's, for
    its two-patch model)."""
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS
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
            st = equilibrate(md, torch, w, 1, equil)
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


def locality_bench(torch, steps=100, warmup=20, equil=1000):
    """Slot order of the cells against the force pass (FP64): row-major cells
    with LDS-staged tiles (the default), and row-major, Morton and Hilbert
    cell orders with every neighbour gathered from global memory, for the LJ
    and the patchy workload, vertex and edge, from one snapshot equilibrated
    for `equil` vertex steps."""
    from paper_1401_4350_amd import md
    from paper_1401_4350_amd.inputs import WORKLOADS
    rows = []
    for base in ("lj_many", "patchy"):
        w = WORKLOADS[base]
        st = equilibrate(md, torch, w, 1, equil)
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
    ap.add_argument("--seed", type=int, default=1, help="first seed")
    ap.add_argument("--seeds", type=int, default=5,
                    help="repetitions with seeds seed .. seed + seeds - 1 (mean and sd)")
    ap.add_argument("--equilibrate", type=int, default=-1,
                    help="untimed vertex steps from the lattice before every timed window "
                         "(-1: 2000 for LJ, 10000 for patchy)")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the atomic and HBM rate probes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the headline (vertex) and edge modes")
    ap.add_argument("--serving-requests", type=int, default=160,
                    help="requests of the serving comparison (0: skip it)")
    ap.add_argument("--serving-occupancy", type=float, default=0.8,
                    help="arrival rate as this fraction of the saturated batched throughput")
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
    from paper_1401_4350_amd.inputs import WORKLOADS

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
    equil = default_equilibration(w) if args.equilibrate < 0 else args.equilibrate
    seeds = list(range(args.seed, args.seed + args.seeds))

    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    # both decompositions from the same equilibrated snapshot, per seed
    per_seed = []
    snapshots = {}
    for sd in seeds:
        snap = equilibrate(md, torch, w, sd, equil)
        snapshots[sd] = snap
        runs_sd = {mode: time_mode(md, torch, w, snap, mode, args.prec, args.steps, args.warmup)
                   for mode in ("vertex", "edge")}
        per_seed.append(runs_sd)
        print(json.dumps({"seed": sd, **{m: round(1e3 * r["ms_per_step"], 2)
                                         for m, r in runs_sd.items()}}), file=sys.stderr,
              flush=True)
    state = snapshots[seeds[0]]
    runs = per_seed[0]
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

    def mean_sd(vals):
        m = sum(vals) / len(vals)
        sd = math.sqrt(sum((v - m) ** 2 for v in vals) / (len(vals) - 1)) if len(vals) > 1 else 0.0
        return m, sd

    def over_seeds(mode, fn):
        return mean_sd([fn(r[mode]) for r in per_seed])

    def evals(r):
        return r["pairs"] / (r["ms_per_step"] * 1e-3)

    value, value_sd = over_seeds("vertex", evals)
    ms_step, ms_step_sd = over_seeds("vertex", lambda r: r["ms_per_step"])
    head = runs["vertex"]
    lj = w.pot == "lj"
    # roofline of the dominant kernel (the vertex force launch): algorithmic
    # bytes per launch / its event-timed duration, averaged over the seeds
    if lj:
        nb_of = lambda r: vertex_force_bytes(w.n, r["pairs"])  # noqa: E731
    else:
        nb_of = lambda r: patchy_vertex_bytes(w.n, r["pairs"])  # noqa: E731
    t_kernel, t_kernel_sd = over_seeds("vertex", lambda r: r["force_ms_per_step"] * 1e-3)
    achieved, achieved_sd = over_seeds("vertex", lambda r: nb_of(r) / (r["force_ms_per_step"] * 1e-3) / 1e9)
    pairs = head["pairs"]
    nb = nb_of(head)

    def summary(r, nbytes):
        return {"ms_per_step": r["ms_per_step"], "md_steps_per_s": 1e3 / r["ms_per_step"],
                "pair_evals_per_s": r["pairs"] / (r["ms_per_step"] * 1e-3),
                "force_pass_us": 1e3 * r["force_ms_per_step"],
                "closing_kick_us": 1e3 * r["kick_ms_per_step"],
                "integrate_us": 1e3 * r["integrate_ms_per_step"],
                "rebuild_us_amortised": 1e3 * r["rebuild_ms_per_step"],
                "force_pass_GBps": nbytes / (r["force_ms_per_step"] * 1e-3) / 1e9,
                "force_pass_bytes": nbytes,
                "pairs": r["pairs"], "nonzero_pairs": r["nonzero_pairs"],
                "list_builds": r["rebuilds_total"],
                "tiles_staged": r["tiles_staged"], "tiles_total": r["tiles_total"],
                "energy_per_particle": r["energy_per_particle"]}

    def edge_bytes(r):
        return edge_force_bytes(w.n, r["pairs"]) if lj else \
            edge_force_bytes(w.n, r["pairs"]) + 80 * w.n  # + q 32, tau zero 24 + write 24

    modes = {"vertex": summary(runs["vertex"], nb),
             "edge": summary(runs["edge"], edge_bytes(runs["edge"]))}
    for k, r in variants.items():
        if k.startswith("vertex"):
            nbv = nb_of(r)
        elif k == "edge_det":
            nbv = edge_det_bytes(w.n, r["pairs"])
        else:
            nbv = edge_bytes(r)
        modes[k] = summary(r, nbv)
    for m, r in newton.items():
        modes[f"newton_m{m}"] = summary(r, newton_pass_bytes(w.n, r["pairs"], m))
    if not args.no_variants:
        modes["thermostat_call_us"] = thermostat_us(md, torch, w, state)
    e_step, e_step_sd = over_seeds("edge", lambda r: r["ms_per_step"])
    modes["edge_over_vertex_speedup"] = ms_step / e_step
    modes["seeds"] = [{"seed": sd, "vertex_ms_per_step": r["vertex"]["ms_per_step"],
                       "edge_ms_per_step": r["edge"]["ms_per_step"],
                       "vertex_force_us": 1e3 * r["vertex"]["force_ms_per_step"],
                       "edge_force_us": 1e3 * r["edge"]["force_ms_per_step"],
                       "pairs": r["vertex"]["pairs"]} for sd, r in zip(seeds, per_seed)]
    modes["edge_ms_per_step_mean_sd"] = [e_step, e_step_sd]

    probes = probe_rates(torch) if not args.no_probes else None
    e_t, e_t_sd = over_seeds("edge", lambda r: r["force_ms_per_step"] * 1e-3)
    e_ach, e_ach_sd = over_seeds("edge", lambda r: edge_bytes(r) / (r["force_ms_per_step"] * 1e-3) / 1e9)
    edge_roof = {"bound": "hbm", "kernel": ("k_edge_lj_tile<FP64>" if lj else "k_edge<patchy, FP64>"),
                 "bytes_per_launch": edge_bytes(runs["edge"]), "avg_launch_us": e_t * 1e6,
                 "avg_launch_us_sd": e_t_sd * 1e6, "achieved": e_ach, "achieved_sd": e_ach_sd,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": e_ach / HBM_PEAK_GBS}
    if probes:
        edge_roof["frac_of_measured_read"] = e_ach / probes["hbm_read_GBps"]
        edge_roof["atomic"] = atomic_roofline(w, runs["edge"], probes, lj)
    out = {
        "metric": "pair-force evals/s (%s MD step, vertex decomposition)" % (
            "LJ" if lj else "patchy"),
        "value": value,
        "value_sd": value_sd,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_sd": ms_step_sd,
        "md_steps_per_s": 1e3 / ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32 pair maths, f64 sums and integration",
        "data": "synthetic",
        "config": {"workload": w.name, "pot": w.pot, "n": w.n, "rho": w.rho, "temp": w.temp,
                   "rcut": w.rcut, "skin": w.skin, "dt": w.dt, "prec": args.prec,
                   "max_neighbors": w.list_capacity(), "seeds": seeds,
                   "equilibration_steps": equil},
        "roofline": {"bound": "hbm", "achieved": achieved, "achieved_sd": achieved_sd,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("k_vertex_lj<FP64, closing kick + next kick and drift>"
                                if lj else "k_vertex_patchy<FP64, closing kick>"),
                     "bytes_per_launch": nb,
                     "bytes_model": ("8|E| + 52N: 4-byte index per full-list entry, list "
                                     "length, own position, force written" if lj else
                                     "8|E| + 204N (with orientation, torque and the kick)"),
                     "avg_launch_us": t_kernel * 1e6, "avg_launch_us_sd": t_kernel_sd * 1e6,
                     # the same kernel against the FP64 vector rate: 2|E| list
                     # entries of LJ_ENTRY_FLOPS each per launch (LJ only: a
                     # patchy pair's operation count depends on its geometry)
                     "valu": ({"achieved": 2 * pairs * LJ_ENTRY_FLOPS / t_kernel / 1e12,
                               "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": 2 * pairs * LJ_ENTRY_FLOPS / t_kernel / 1e12
                               / FP64_VECTOR_PEAK_TFLOPS} if lj else None),
                     "edge": edge_roof},
        "modes": modes,
    }
    if probes:
        out["roofline"]["frac_of_measured_read"] = achieved / probes["hbm_read_GBps"]
        out["probes"] = probes
    # HBM traffic of the same kernel from the committed FETCH_SIZE / WRITE_SIZE
    # record, used only while the kernel sources are the ones it was taken on
    from paper_1401_4350_amd import prof
    rec = prof.read_record(os.path.join(ROOT, "profiles", f"traffic_{w.name}_{args.prec}.txt"))
    if rec and rec.get("source_sha") == prof.source_hash():
        out["roofline"]["traffic"] = float(rec["traffic_bytes"])
        out["roofline"]["traffic_over_algorithmic"] = float(rec["traffic_bytes"]) / nb
    if lj and not args.no_variants and w.name == "lj_many":
        out["dense"] = dense_bench(md, torch, args)
    if args.serving_requests > 0:
        out["serving"] = serving_bench(args.serving_requests, args.serving_steps,
                                       args.serving_occupancy)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, state, pairs)
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
