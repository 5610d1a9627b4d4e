"""The C-ABI library loads, exports every entry point include/md.h declares,
and rejects bad parameters on the host before any HIP call (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1401_4350_amd import md as m
    return m


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(md_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("md_create", "md_build_cells", "md_build_neighbors", "md_forces",
                     "md_step", "md_energy", "md_query_sizes", "md_get_state", "md_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(md):
    lib = md.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _params(md, **kw):
    from paper_1401_4350_amd.inputs import WORKLOADS
    p = md.make_params(WORKLOADS["lj_small"])
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_query_sizes(md):
    s = md.query_sizes(_params(md))
    assert s.alignment == 256
    assert s.state_bytes >= 4096 * 3 * 32
    # workspace holds at least the full lists
    assert s.workspace_bytes >= 4096 * 4 * _params(md).max_neighbors


def test_edge_store_workspace(md):
    """The deterministic edge mode's arrays are reserved only on request: 32 B
    (LJ) per half-list entry plus 4 B per full-list slot."""
    p0 = _params(md)
    p1 = _params(md, edge_store=1)
    s0, s1 = md.query_sizes(p0), md.query_sizes(p1)
    assert s1.state_bytes == s0.state_bytes
    half = p0.n * p0.max_neighbors // 2
    assert s1.workspace_bytes - s0.workspace_bytes >= 32 * half + 4 * p0.n * p0.max_neighbors


@pytest.mark.parametrize("field,value,status", [
    ("n", 1, -1), ("box", 5.0, -5), ("dt", 0.0, -1), ("skin", -0.1, -1),
    ("rcut", 0.0, -1), ("max_neighbors", 0, -1), ("mass", -1.0, -1), ("pot", 7, -1),
    ("prec", 9, -1), ("box", float("nan"), -1), ("newton_m", -1, -1), ("newton_m", 65, -1),
    ("edge_store", 2, -1), ("edge_store", -1, -1), ("cell_order", 4, -1), ("cell_order", -1, -1),
    ("patch_model", 1, -1), ("patch_model", 2, -1), ("patch_model", -1, -1),
])
def test_invalid_params_rejected_on_host(md, field, value, status):
    p = _params(md, **{field: value})
    s = md.MDSizes()
    assert md.lib().md_query_sizes(ctypes.byref(p), ctypes.byref(s)) == status
    h = ctypes.c_void_p()
    # buffers are never touched: validation happens before any HIP call
    assert md.lib().md_create(ctypes.byref(p), 256, 1 << 40, 512, 1 << 40, None,
                              ctypes.byref(h)) == status
    assert not h.value


def test_patch_models(md):
    """Both patch models are accepted for patchy particles; a third is not."""
    from paper_1401_4350_amd.inputs import WORKLOADS
    s = md.MDSizes()
    for name, model, status in (("patchy", 0, 0), ("patchy_paper", 1, 0), ("patchy", 2, -1)):
        p = md.make_params(WORKLOADS[name].with_(n=4000))
        assert p.patch_model == (model if status == 0 else 0)
        p.patch_model = model
        assert md.lib().md_query_sizes(ctypes.byref(p), ctypes.byref(s)) == status


def test_buffer_checks_before_hip(md):
    p = _params(md)
    s = md.query_sizes(p)
    h = ctypes.c_void_p()
    lib = md.lib()
    assert lib.md_create(ctypes.byref(p), 256, s.state_bytes - 1, 512, s.workspace_bytes,
                         None, ctypes.byref(h)) == -2
    assert lib.md_create(ctypes.byref(p), 257, s.state_bytes, 512, s.workspace_bytes,
                         None, ctypes.byref(h)) == -2
    assert lib.md_create(ctypes.byref(p), None, s.state_bytes, 512, s.workspace_bytes,
                         None, ctypes.byref(h)) == -1


def test_null_handle_calls(md):
    lib = md.lib()
    for name in ("md_build_cells", "md_build_neighbors"):
        assert getattr(lib, name)(None) == -1
    assert lib.md_forces(None, 0) == -1
    assert lib.md_step(None, 1, 0) == -1
    assert lib.md_thermostat(None, 1.0, 0.5, 1, 0) == -1
    assert lib.md_status_str(-4).decode().startswith("Verlet list overflow")
    assert lib.md_last_error(None).decode() == ""


def test_batch_params_checked_on_host(md):
    lib = md.lib()
    ok = md.batch_params(8, 100000, 1 << 30)
    assert md.batch_workspace_bytes(ok) > 0
    n = ctypes.c_uint64()
    h = ctypes.c_void_p()
    for field, value in [("max_systems", 0), ("mode", 2), ("mode", 7), ("steps_per_launch", 0),
                         ("steps_per_launch", 5000), ("use_graph", 2), ("max_particles", 1),
                         ("pool_bytes", 0)]:
        p = md.batch_params(8, 100000, 1 << 30)
        setattr(p, field, value)
        assert lib.md_batch_query_sizes(ctypes.byref(p), ctypes.byref(n)) == -1, field
        assert lib.md_batch_create(ctypes.byref(p), 256, 1 << 40, None, ctypes.byref(h)) == -1
        assert not h.value
    need = md.batch_workspace_bytes(ok)
    assert lib.md_batch_create(ctypes.byref(ok), 256, need - 1, None, ctypes.byref(h)) == -2
    assert lib.md_batch_create(ctypes.byref(ok), 257, need, None, ctypes.byref(h)) == -2
    assert lib.md_batch_create(ctypes.byref(ok), None, need, None, ctypes.byref(h)) == -1
    # the workspace grows with the block-class capacities
    big = md.batch_params(8, 1000000, 1 << 30)
    assert md.batch_workspace_bytes(big) > need


def test_batch_null_handle_calls(md):
    lib = md.lib()
    k = ctypes.c_int32()
    v = ctypes.c_int64()
    assert lib.md_batch_admit(None, None, 1, ctypes.byref(k)) == -1
    assert lib.md_batch_step(None, ctypes.byref(k)) == -1
    assert lib.md_batch_steps_left(None, 0, ctypes.byref(v)) == -1
    assert lib.md_batch_retire(None, 0) == -1
    assert lib.md_batch_sync(None) == -1
    assert lib.md_batch_last_error(None).decode() == ""
    lib.md_batch_destroy(None)


def test_forces_static_rejects_on_host(md):
    """md_forces_static checks its arguments before any HIP call: bad
    parameters, a system larger than the static array, missing pointers, an
    unknown mode, the deterministic edge mode without edge_store, a curve
    cell order.  Fake non-null pointers are never dereferenced on these
    paths."""
    from paper_1401_4350_amd.inputs import WORKLOADS
    f = md.lib().md_forces_static
    fake = ctypes.c_void_p(256)

    def call(p, x=fake, q=fake, out=fake, t=fake, mode=0):
        return f(ctypes.byref(p), x, q, out, t, mode, None, None)

    assert call(_params(md, n=1)) == -1
    assert call(_params(md, box=5.0)) == -5
    big = md.make_params(WORKLOADS["lj_many"].with_(n=50000))
    assert call(big) == -2
    assert call(_params(md), x=None) == -1
    assert call(_params(md), out=None) == -1
    assert call(_params(md), mode=7) == -1
    assert call(_params(md), mode=3) == -1  # edge_store = 0
    assert call(_params(md, cell_order=2)) == -1
    patchy = md.make_params(WORKLOADS["patchy"].with_(n=500))
    assert call(patchy, q=None) == -1
    assert call(patchy, t=None) == -1
