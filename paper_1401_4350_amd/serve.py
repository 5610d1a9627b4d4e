"""Continuous-batching request loop for independent MD simulations.

Requests (inputs.serving_requests) arrive over time.  The scheduler keeps a
FIFO queue and admits the request at its head as soon as a batch slot and
enough of the HBM footprint budget are free; admitted systems advance
together, one batched launch at a time (md_batch_step), and each is retired
the moment its steps are done, which frees its slot and footprint for the
next request.  Arrivals never wait for a batch to drain.

The loop talks to an executor:

  GpuExecutor   the md_batch_* C ABI on the current HIP device, with every
                system's buffers allocated by torch at admission and freed at
                retirement;
  FakeExecutor  a virtual clock and a cost model, no GPU, for testing the
                scheduling logic.

Both report the same record per request (arrival, admission and completion
time, steps, pair count), from which summarize() derives p50/p99
time-to-completion and aggregate pair evaluations per second.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .inputs import Request, make_state


@dataclass
class Record:
    rid: int
    n: int
    pot: str
    steps: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    pairs: int = 0          # half-list entries at the last list build
    status: str = "queued"  # queued | running | done | rejected | failed
    error: str = ""


@dataclass
class Report:
    records: list[Record]
    wall: float
    launches: int
    peak_bytes: int
    peak_active: int
    budget_bytes: int
    extra: dict = field(default_factory=dict)


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (the smallest value with at least q % of the
    values at or below it); nan for an empty list."""
    v = sorted(values)
    if not v:
        return math.nan
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return float(v[k - 1])


def summarize(rep: Report) -> dict:
    done = [r for r in rep.records if r.status == "done"]
    lat = [r.done - r.arrival for r in done]
    wait = [r.admitted - r.arrival for r in done]
    evals = sum(r.pairs * r.steps for r in done)
    span = (max(r.done for r in done) - min(r.arrival for r in done)) if done else math.nan
    return {
        "requests": len(rep.records),
        "completed": len(done),
        "rejected": sum(r.status == "rejected" for r in rep.records),
        "failed": sum(r.status == "failed" for r in rep.records),
        "p50_s": percentile(lat, 50),
        "p99_s": percentile(lat, 99),
        "queue_p50_s": percentile(wait, 50),
        "queue_p99_s": percentile(wait, 99),
        "pair_evals_per_s": evals / span if done and span > 0 else math.nan,
        "steps_per_s": sum(r.steps for r in done) / span if done and span > 0 else math.nan,
        "wall_s": rep.wall,
        "launches": rep.launches,
        "peak_bytes": rep.peak_bytes,
        "peak_active": rep.peak_active,
        "budget_bytes": rep.budget_bytes,
    }


class Scheduler:
    """FIFO admission by footprint.  A request whose footprint alone exceeds
    the budget is rejected at once (it could never run); others wait at the
    head of the queue until it fits."""

    def __init__(self, executor, budget_bytes: int, max_slots: int):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)

    def run(self, requests: list[Request], cancel: dict[int, float] | None = None) -> Report:
        """Serves `requests`; cancel[rid] = t cancels that request at time t
        (or when it is admitted, if later): its slot and footprint are freed
        and it is recorded as failed with error "cancelled"."""
        ex = self.ex
        cancel = dict(cancel or {})
        arrivals = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        recs = {r.rid: Record(r.rid, r.workload.n, r.workload.pot, r.workload.steps, r.arrival)
                for r in requests}
        queue: deque[Request] = deque()
        active: dict[int, tuple[Request, int]] = {}  # handle -> (request, footprint)
        used = peak = peak_active = launches = 0
        t0 = ex.now()
        while arrivals or queue or active:
            now = ex.now()
            while arrivals and arrivals[0].arrival <= now:
                queue.append(arrivals.popleft())
            while queue:
                req = queue[0]
                foot = ex.footprint(req)
                rec = recs[req.rid]
                if foot > self.budget:
                    queue.popleft()
                    rec.status, rec.error = "rejected", f"footprint {foot} B exceeds the budget"
                    continue
                if used + foot > self.budget or len(active) >= self.max_slots:
                    break
                h = ex.admit(req)
                if h is None:  # the batch's own capacity (slots, grids) is full
                    break
                queue.popleft()
                used += foot
                active[h] = (req, foot)
                rec.admitted, rec.status = ex.now(), "running"
                peak, peak_active = max(peak, used), max(peak_active, len(active))
            cancelled = False
            for h, (req, foot) in list(active.items()):
                if req.rid in cancel and cancel[req.rid] <= ex.now():
                    ex.retire(h, cancelled=True)
                    del active[h]
                    used -= foot
                    rec = recs[req.rid]
                    rec.status, rec.error, rec.done = "failed", "cancelled", ex.now()
                    cancelled = True
            if cancelled:
                continue  # the freed room may admit the next request
            if not active:
                if queue:
                    raise RuntimeError("the request at the head of the queue fits the budget "
                                       "but the executor cannot admit it into an empty batch")
                if arrivals:
                    ex.wait_until(arrivals[0].arrival)
                continue
            ex.step()
            launches += 1
            for h in ex.finished():
                req, foot = active.pop(h)
                rec = recs[req.rid]
                out = ex.retire(h)
                used -= foot
                rec.done = ex.now()
                rec.pairs = out.get("pairs", 0)
                if out.get("error"):
                    rec.status, rec.error = "failed", out["error"]
                else:
                    rec.status = "done"
        return Report(records=[recs[r.rid] for r in requests], wall=ex.now() - t0,
                      launches=launches, peak_bytes=peak, peak_active=peak_active,
                      budget_bytes=self.budget)


class FakeExecutor:
    """Virtual-clock executor: a launch of k steps costs
    launch_s + k * (step_s + sum_active n * particle_s) seconds, systems
    advance like the C batch (k = steps_per_launch, or the smallest power of
    two covering the largest remaining need), and footprints come from
    md_query_sizes or a given function."""

    def __init__(self, steps_per_launch: int = 64, max_systems: int = 64, launch_s: float = 20e-6,
                 step_s: float = 30e-6, particle_s: float = 2e-9, footprint=None):
        self.spl = steps_per_launch
        self.max_systems = max_systems
        self.launch_s, self.step_s, self.particle_s = launch_s, step_s, particle_s
        self.t = 0.0
        self.left: dict[int, int] = {}
        self.req: dict[int, Request] = {}
        self.free = list(range(max_systems))[::-1]
        self._footprint = footprint
        self.steps_run: dict[int, int] = {}

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)

    def footprint(self, req: Request) -> int:
        if self._footprint is not None:
            return int(self._footprint(req))
        from . import md
        s = md.query_sizes(md.make_params(req.workload, "fp32"))
        return int(s.state_bytes + s.workspace_bytes)

    def admit(self, req: Request):
        if not self.free:
            return None
        h = self.free.pop()
        self.left[h] = req.workload.steps
        self.req[h] = req
        self.steps_run[h] = 0
        return h

    def step(self):
        need = max(self.left.values(), default=0)
        if need == 0:
            return
        k = self.spl
        if need < k:
            k = 1 << max(0, math.ceil(math.log2(need)))
            k = min(k, self.spl)
        work = sum(self.req[h].workload.n for h in self.left if self.left[h] > 0)
        self.t += self.launch_s + k * (self.step_s + work * self.particle_s)
        for h in self.left:
            d = min(k, self.left[h])
            self.left[h] -= d
            self.steps_run[h] += d

    def finished(self):
        return [h for h, v in self.left.items() if v == 0]

    def retire(self, h, cancelled: bool = False) -> dict:
        req = self.req.pop(h)
        del self.left[h]
        self.free.append(h)
        n = req.workload.n
        return {"pairs": int(n * req.workload.expected_neighbors() / 2), "steps": self.steps_run.pop(h)}


class GpuExecutor:
    """md_batch_* on the current HIP device.  Each admitted request gets an
    md_system whose state and workspace buffers torch allocates; they are
    released when it is retired.  After every launch the executor waits for
    the stream, so the clock measures completed GPU work."""

    def __init__(self, max_systems: int, max_particles: int, pool_bytes: int,
                 mode: str = "vertex", prec: str = "fp32", steps_per_launch: int = 64,
                 use_graph: bool = True):
        from . import md
        self.md = md
        self.prec = prec
        self.mode = mode
        self.batch = md.Batch(md.batch_params(max_systems, max_particles, pool_bytes, mode,
                                              steps_per_launch, use_graph))
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float):
        d = t - self.now()
        if d > 0:
            time.sleep(d)

    def footprint(self, req: Request) -> int:
        s = self.md.query_sizes(self.md.make_params(req.workload, self.prec))
        return int(s.state_bytes + s.workspace_bytes)

    def admit(self, req: Request):
        md = self.md
        st = make_state(req.workload, req.seed)
        g = md.System(md.make_params(req.workload, self.prec))
        g.set_state(st.x, st.v, st.q, st.angmom)
        g.build()
        slot = self.batch.try_admit(g, req.workload.steps)
        if slot is None:
            g.close()
            return None
        return slot

    def step(self):
        self.batch.step()
        self.batch.sync()

    def finished(self):
        return [s for s in list(self.batch.systems) if self.batch.steps_left(s) == 0]

    def retire(self, slot, cancelled: bool = False) -> dict:
        g = self.batch.systems.get(slot)
        out: dict = {}
        try:
            self.batch.retire(slot)
            out["pairs"] = int(g.stats()["pairs"])
        except self.md.MDError as e:
            out["error"] = str(e)
        finally:
            if g is not None:
                g.close()
        return out

    def close(self):
        self.batch.close()


class SequentialExecutor:
    """The single-system path as a server: one system at a time, all its
    steps in one md_step call (for comparison with the batch; run it with a
    Scheduler of max_slots=1)."""

    def __init__(self, mode: str = "vertex", prec: str = "fp64"):
        from . import md
        self.md = md
        self.mode, self.prec = mode, prec
        self.sys = {}
        self.next = 0
        self.t0 = time.perf_counter()

    now = GpuExecutor.now
    wait_until = GpuExecutor.wait_until

    def footprint(self, req: Request) -> int:
        return footprint_bytes(req, self.prec)

    def admit(self, req: Request):
        md = self.md
        st = make_state(req.workload, req.seed)
        g = md.System(md.make_params(req.workload, self.prec))
        g.set_state(st.x, st.v, st.q, st.angmom)
        g.build()
        g.forces(self.mode)
        h = self.next
        self.next += 1
        self.sys[h] = [g, req.workload.steps]
        return h

    def step(self):
        for item in self.sys.values():
            if item[1] > 0:
                item[0].step(item[1], self.mode)  # syncs
                item[1] = 0

    def finished(self):
        return [h for h, item in self.sys.items() if item[1] == 0]

    def retire(self, h, cancelled: bool = False) -> dict:
        g, _ = self.sys.pop(h)
        out = {"pairs": int(g.stats()["pairs"])}
        g.close()
        return out


def footprint_bytes(req: Request, prec: str = "fp32") -> int:
    """HBM footprint of one request (state + workspace, md_query_sizes)."""
    from . import md
    s = md.query_sizes(md.make_params(req.workload, prec))
    return int(s.state_bytes + s.workspace_bytes)


def latency_table(rep: Report) -> np.ndarray:
    """(rid, n, arrival, admitted, done) of the completed requests."""
    rows = [(r.rid, r.n, r.arrival, r.admitted, r.done) for r in rep.records if r.status == "done"]
    return np.array(rows, dtype=np.float64).reshape(-1, 5)
