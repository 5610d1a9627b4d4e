"""md_forces_static (the entry point that allocates nothing) against the
existing path md_create + md_set_state + md_build_* + md_forces, through the
C ABI: two calls in a row, the second with a smaller system, so the second
runs on the scratch array the first left behind.  FP64 forces (and torques)
agree within 1e-10 per component of sum_j |F_ij,c| (the oracle's scale) with
the existing entry point and with the oracle; the device status word is
MD_OK.  Host-side rejections (a system larger than the array, a missing
pointer) enqueue nothing."""
import sys

import numpy as np
import pytest

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS

from _helpers import accepted_state, cond_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import md as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def existing_path(md, w, s, mode):
    g = md.System(md.make_params(w))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    g.forces(mode)
    out = g.get_state()
    g.close()
    return out["f"], out.get("torque")


def static_path(md, torch, w, s, mode):
    x = torch.tensor(s.x, dtype=torch.float64, device="cuda")
    q = torch.tensor(s.q, dtype=torch.float64, device="cuda") if s.q is not None else None
    f, t, status = md.forces_static(md.make_params(w), x, q, mode)
    torch.cuda.synchronize()
    return f.cpu().numpy(), (t.cpu().numpy() if t is not None else None), int(status.item())


def oracle_ref(w, s):
    if w.pot == "lj":
        F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
        return F, A, None, None
    pp = oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                       delta=w.patch_delta, rpc=w.patch_rcut,
                       model=1 if w.patch_model == "polar2" else 0)
    F, T, _, _, _, _ = oracle.patchy_forces(s.x, s.q, s.box, pp, with_abs=True)
    FA, TA = oracle.patchy_pair_scales(s.x, s.q, s.box, pp)
    return F, FA, T, TA


CASES = [
    # (workload, first n, second (smaller) n, mode)
    ("lj_small", 3000, 1000, "vertex"),
    ("lj_small", 2500, 700, "edge"),
    ("patchy_paper", 2000, 600, "vertex"),
    ("patchy", 1500, 500, "edge"),
]


@pytest.mark.parametrize("name,n1,n2,mode", CASES)
def test_static_equals_existing_entry(md, name, n1, n2, mode):
    import torch
    for call, n in enumerate((n1, n2)):
        w = WORKLOADS[name].with_(n=n)
        s = accepted_state(w, 40 + call)
        say(f"[static] {name} n={n} mode={mode} call {call + 1}")
        f, t, status = static_path(md, torch, w, s, mode)
        f0, t0 = existing_path(md, w, s, mode)
        F, FA, T, TA = oracle_ref(w, s)
        assert status == md.MD_OK
        e_same = cond_rel_err(f, f0, FA)
        e_orc = cond_rel_err(f, F, FA)
        say(f"  force error vs md_forces {e_same:.2e}, vs oracle {e_orc:.2e}")
        assert e_same <= 1e-10 and e_orc <= 1e-10
        if mode == "vertex" and w.pot == "lj":
            # same kernels, same slot order, positions wrapped exactly alike:
            # the same sums (quaternions are normalised on the host by
            # md_set_state and on the device here, which may round apart)
            assert np.array_equal(f, f0)
        if T is not None:
            et_same = cond_rel_err(t, t0, TA)
            et_orc = cond_rel_err(t, T, TA)
            say(f"  torque error vs md_forces {et_same:.2e}, vs oracle {et_orc:.2e}")
            assert et_same <= 1e-10 and et_orc <= 1e-10


def test_static_rejections(md):
    import torch
    w = WORKLOADS["lj_many"].with_(n=50000)  # needs more than the static array
    sz = md.query_sizes(md.make_params(w))
    assert sz.state_bytes + sz.workspace_bytes > md.STATIC_SCRATCH_BYTES
    x = torch.zeros((w.n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.forces_static(md.make_params(w), x)
    assert e.value.status == -2  # MD_ERR_BUFFER_TOO_SMALL
    w = WORKLOADS["patchy"].with_(n=500)
    x = torch.zeros((w.n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.forces_static(md.make_params(w), x, None)  # patchy without quaternions
    assert e.value.status == -1  # MD_ERR_INVALID_ARG
