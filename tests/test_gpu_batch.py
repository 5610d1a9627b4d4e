"""GPU tests of the batched step (md_batch_* through the C ABI): each system
gives the same result alone (md_step) and in a mix of systems of different
size, potential, density and precision -- bitwise in the vertex mode, within
1e-9 in the edge mode (FP64 atomics add in a different order) -- including
systems admitted and retired while others run, and the batch's error paths.
Every FP64 system's batched trajectory is also compared with the oracle's
velocity-Verlet run: positions, velocities (and quaternions, angular momenta)
within 1e-9 and the same number of list builds."""
import sys

import numpy as np
import pytest

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS

from _helpers import accepted_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import md as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# (workload, overrides, precision, steps): LJ and both patchy models, dense and
# dilute, small boxes (n_c = 3 and 4), FP64 and FP32 pair maths.
MIX = [
    ("lj_small", {"n": 3000, "rho": 0.8}, "fp64", 60),
    ("lj_small", {"n": 700, "rho": 0.9}, "fp64", 45),
    ("patchy", {"n": 1500, "rho": 0.5}, "fp64", 50),
    ("lj_small", {"n": 5000, "rho": 0.6}, "fp32", 64),
    ("patchy", {"n": 900, "rho": 0.4}, "fp32", 33),
    ("lj_small", {"n": 2000, "rho": 0.85}, "fp32_kahan", 20),
    ("patchy_paper", {"n": 1200, "rho": 0.3}, "fp64", 40),  # the two-patch model
]


def fresh(md, k, seed=11, edge_store=False):
    name, over, prec, steps = MIX[k]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, seed + k)
    g = md.System(md.make_params(w, prec, edge_store=edge_store))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    return g, steps


def oracle_run(k, seed=11):
    """The oracle's run of MIX[k] from the same accepted state as fresh()."""
    name, over, prec, steps = MIX[k]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, seed + k)
    if w.pot == "lj":
        return w, oracle.run(s.x, s.v, s.box, pot="lj", nsteps=steps, dt=w.dt, skin=w.skin,
                             mass=w.mass, lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    pp = oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                       delta=w.patch_delta, rpc=w.patch_rcut,
                       model=1 if w.patch_model == "polar2" else 0)
    return w, oracle.run(s.x, s.v, s.box, pot="patchy", nsteps=steps, dt=w.dt, skin=w.skin,
                         mass=w.mass, inertia=w.inertia, patchy=pp, q=s.q, angmom=s.angmom)


def check_against_oracle(k, got, gstats):
    w, ref = oracle_run(k)
    d = got["x"] - ref["x"]
    d -= w.box * np.rint(d / w.box)
    assert np.abs(d).max() < 1e-9, (k, "x")
    assert np.abs(got["v"] - ref["v"]).max() < 1e-9, (k, "v")
    if w.pot == "patchy":
        # q and -q are the same rotation
        dq = np.minimum(np.abs(got["q"] - ref["q"]).max(axis=1),
                        np.abs(got["q"] + ref["q"]).max(axis=1))
        assert dq.max() < 1e-9, (k, "q")
        assert np.abs(got["angmom"] - ref["angmom"]).max() < 1e-9, (k, "angmom")
    if ref["disp_margin"] > 1e-12:
        assert gstats["rebuilds"] == len(ref["rebuild_steps"]), k


def alone(md, k, mode):
    g, steps = fresh(md, k, edge_store=mode == "edge_det")
    g.forces(mode)
    g.step(steps, mode)
    return g.get_state(), g.stats()


def run_mix(md, mode, steps_per_launch, use_graph=True, late=(2, 5)):
    """Admits every system except `late` at once, the late ones after the
    first launch; retires each system when it is done."""
    bp = md.batch_params(8, 40000, 4 << 30, mode, steps_per_launch, use_graph)
    b = md.Batch(bp)
    pending = [k for k in range(len(MIX)) if k not in late]
    slots = {}
    store = mode == "edge_det"
    for k in pending:
        g, steps = fresh(md, k, edge_store=store)
        slots[b.admit(g, steps)] = k
    out = {}
    launches = 0
    while slots or late:
        ran = b.step()
        launches += 1
        if late:
            for k in late:
                g, steps = fresh(md, k, edge_store=store)
                slots[b.admit(g, steps)] = k
            late = ()
        for slot in [s for s in slots if b.steps_left(s) == 0]:
            k = slots.pop(slot)
            g = b.retire(slot)
            out[k] = (g.get_state(), g.stats())
        assert ran > 0 or not slots
        assert launches < 1000
    info = b.info()
    b.close()
    return out, info


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_vertex_bitwise_alone_and_in_mix(md, use_graph):
    say(f"[batch vertex] graph={use_graph}")
    mix, info = run_mix(md, "vertex", 16, use_graph)
    assert info["active"] == 0 and info["particles"] == 0 and info["bytes"] == 0
    if use_graph:
        assert info["captures"] >= 1
    for k in range(len(MIX)):
        ref, rstats = alone(md, k, "vertex")
        got, gstats = mix[k]
        for key in ref:
            assert np.array_equal(got[key], ref[key]), (k, key)
        assert gstats["steps"] == rstats["steps"] == MIX[k][3]
        assert gstats["rebuilds"] == rstats["rebuilds"]
        if use_graph and MIX[k][2] == "fp64":
            say(f"  oracle run of system {k}")
            check_against_oracle(k, got, gstats)


def test_batch_edge_alone_and_in_mix(md):
    say("[batch edge]")
    mix, _ = run_mix(md, "edge", 32)
    for k in range(len(MIX)):
        ref, _ = alone(md, k, "edge")
        got, _ = mix[k]
        box = WORKLOADS[MIX[k][0]].with_(**MIX[k][1]).box
        d = got["x"] - ref["x"]
        d -= box * np.rint(d / box)
        tol = 1e-9 if MIX[k][2] == "fp64" else 1e-6
        assert np.abs(d).max() < tol, k
        assert np.abs(got["v"] - ref["v"]).max() < tol, k
        if MIX[k][2] == "fp64":
            check_against_oracle(k, got, mix[k][1])


def test_batch_edge_det_bitwise_alone_and_in_mix(md):
    """The deterministic edge mode in the batch: per-edge records and the
    ordered gather make every system's trajectory bitwise the one it has
    alone; a system made without edge_store is refused."""
    say("[batch edge_det]")
    mix, _ = run_mix(md, "edge_det", 16)
    for k in range(len(MIX)):
        ref, rstats = alone(md, k, "edge_det")
        got, gstats = mix[k]
        for key in ref:
            assert np.array_equal(got[key], ref[key]), (k, key)
        assert gstats["rebuilds"] == rstats["rebuilds"]
        if MIX[k][2] == "fp64":
            check_against_oracle(k, got, gstats)
    b = md.Batch(md.batch_params(2, 10000, 1 << 30, "edge_det", 8, True))
    g, steps = fresh(md, 0)  # no edge_store
    with pytest.raises(md.MDError) as e:
        b.admit(g, steps)
    assert e.value.status == -1
    g.close()
    b.close()


def test_batch_thermostat_bitwise_alone(md):
    """md_batch_thermostat between batch launches gives bitwise the state of
    the same system stepped alone with md_thermostat at the same points (same
    draws: the refresh is keyed by particle id, seed and counter)."""
    say("[batch thermostat]")
    systems = [("lj_small", {"n": 3000, "rho": 0.8}, 48), ("patchy_paper", {"n": 1200, "rho": 0.3}, 48),
               ("lj_small", {"n": 900, "rho": 0.85}, 48)]
    K, T, prob = 8, 0.9, 0.3

    def make(k):
        name, over, steps = systems[k]
        w = WORKLOADS[name].with_(**over)
        s = accepted_state(w, 70 + k)
        g = md.System(md.make_params(w))
        g.set_state(s.x, s.v, s.q, s.angmom)
        g.build()
        g.forces("vertex")
        return g, w

    thermo = (0, 1)  # systems that get the thermostat
    b = md.Batch(md.batch_params(4, 20000, 1 << 30, "vertex", K, True))
    slots = {}
    for k in range(len(systems)):
        g, _ = make(k)
        slots[k] = b.admit(g, systems[k][2])
    launch = 0
    while any(b.steps_left(sl) > 0 for sl in slots.values()):
        assert b.step() == K
        for k in thermo:
            b.thermostat(slots[k], T, prob, 5 + k, launch)
        launch += 1
    got = {k: b.retire(sl).get_state() for k, sl in slots.items()}
    b.close()
    for k in range(len(systems)):
        g, w = make(k)
        for c in range(systems[k][2] // K):
            g.step(K, "vertex")
            if k in thermo:
                g.thermostat(T, prob, 5 + k, c)
        ref = g.get_state()
        g.close()
        for key in ref:
            assert np.array_equal(got[k][key], ref[key]), (k, key)
    b2 = md.Batch(md.batch_params(2, 5000, 1 << 28, "vertex", K, True))
    with pytest.raises(md.MDError):
        b2.thermostat(0, T, prob, 1, 0)  # free slot
    b2.close()


def test_batch_cancel_and_slot_reuse(md):
    say("[batch cancel]")
    b = md.Batch(md.batch_params(2, 20000, 1 << 30, "vertex", 8))
    g0, _ = fresh(md, 0)
    g1, _ = fresh(md, 1)
    s0 = b.admit(g0, 100)
    s1 = b.admit(g1, 10)
    assert s0 != s1
    g2, _ = fresh(md, 3)
    assert b.try_admit(g2, 5) is None  # no free slot
    assert b.step() == 8
    assert b.steps_left(s0) == 92 and b.steps_left(s1) == 2
    b.retire(s0)  # cancelled after 8 steps
    assert g0.stats()["steps"] == 8
    assert b.steps_left(s0) == -1
    s2 = b.admit(g2, 5)
    assert s2 == s0  # the freed slot is reused
    assert b.step() == 8  # covers max(2, 5) = 5 rounded up to a power of two
    b.retire(s1)
    b.retire(s2)
    assert g1.stats()["steps"] == 10 and g2.stats()["steps"] == 5
    # retired systems are ordinary systems again
    g0.step(3)
    assert g0.stats()["steps"] == 11
    b.close()


def test_batch_admission_limits_and_state_errors(md):
    say("[batch errors]")
    g, _ = fresh(md, 0)
    foot = g.state_bytes + g.workspace_bytes
    small = md.Batch(md.batch_params(4, 20000, foot - 1, "vertex", 4))
    assert small.try_admit(g, 10) is None  # over the footprint budget
    few = md.Batch(md.batch_params(4, 2000, 1 << 30, "vertex", 4))
    assert few.try_admit(g, 10) is None  # over max_particles (n = 3000)
    b = md.Batch(md.batch_params(4, 20000, 1 << 30, "vertex", 4))
    slot = b.admit(g, 10)
    with pytest.raises(md.MDError) as e:
        g.step(1)
    assert e.value.status == -7
    with pytest.raises(md.MDError) as e:
        b.admit(g, 10)
    assert e.value.status == -7
    other = md.Batch(md.batch_params(4, 20000, 1 << 30, "vertex", 4))
    with pytest.raises(md.MDError) as e:
        other.admit(g, 10)
    assert e.value.status == -7
    w = WORKLOADS["lj_small"].with_(n=1000)
    s = accepted_state(w, 3)
    unbuilt = md.System(md.make_params(w))
    unbuilt.set_state(s.x, s.v)
    with pytest.raises(md.MDError) as e:
        b.admit(unbuilt, 10)
    assert e.value.status == -7
    b.retire(slot)
    with pytest.raises(md.MDError) as e:
        b.retire(slot)
    assert e.value.status == -1
    for h in (small, few, b, other):
        h.close()


def test_batch_overflow_reported_at_retire(md):
    """A system whose lists overflow in the batch reports it when retired;
    the other systems are unaffected."""
    say("[batch overflow]")
    w = WORKLOADS["lj_small"].with_(n=2000, max_neighbors=16)
    s = accepted_state(w, 4)
    bad = md.System(md.make_params(w))
    bad.set_state(s.x, s.v)
    bad.build()
    b = md.Batch(md.batch_params(4, 20000, 1 << 30, "vertex", 4))
    with pytest.raises(md.MDError) as e:
        b.admit(bad, 4)  # the initial build already overflowed
    assert e.value.status == -4
    g, steps = fresh(md, 1)
    slot = b.admit(g, steps)
    while b.steps_left(slot) > 0:
        b.step()
    b.retire(slot)
    ref, _ = alone(md, 1, "vertex")
    assert np.array_equal(g.get_state()["x"], ref["x"])
    b.close()
