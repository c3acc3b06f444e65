"""C ABI checks that need no GPU: the library loads, exports every function
that include/brahms.h declares, and rejects bad calls before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2609_08384_amd import brahms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "brahms.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(brahms_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return brahms.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "brahms_plan_create" in names and "brahms_step" in names
    for n in names:
        assert hasattr(lib, n), n


def _params(nf=2, dz=0.01, **kw):
    p = brahms.Params(dz=dz, fields=[brahms.FieldParams(kappa=1.0, diffraction=1.0) for _ in range(nf)], **kw)
    c, keep = brahms._params_c(p, nf)
    return c, keep


def _create(lib, nx, ny, nt, nf, c):
    h = ctypes.c_void_p()
    st = lib.brahms_plan_create(nx, ny, nt, nf, ctypes.byref(c), None, ctypes.byref(h))
    return st, h


def test_create_and_workspace(lib):
    c, keep = _params()
    st, h = _create(lib, 32, 64, 16, 2, c)
    assert st == brahms.BRAHMS_OK
    size = ctypes.c_size_t()
    assert lib.brahms_plan_workspace_size(h, ctypes.byref(size)) == brahms.BRAHMS_OK
    assert size.value > 0 and size.value % 256 == 0
    z = ctypes.c_double()
    assert lib.brahms_get_z(h, ctypes.byref(z)) == brahms.BRAHMS_OK and z.value == 0.0
    assert lib.brahms_step(h, 1) == brahms.BRAHMS_E_STATE           # before bind
    assert b"bind" in lib.brahms_last_error()
    assert lib.brahms_step(h, 0) == brahms.BRAHMS_E_STATE
    assert lib.brahms_propagate(h, 0.0105) == brahms.BRAHMS_E_INVALID_ARG  # not a multiple of dz
    assert lib.brahms_set_z(h, 0.2) == brahms.BRAHMS_OK
    assert lib.brahms_get_z(h, ctypes.byref(z)) == brahms.BRAHMS_OK and abs(z.value - 0.2) < 1e-15
    assert lib.brahms_set_z(h, -0.01) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_set_z(h, 0.005) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_propagate(h, 0.1) == brahms.BRAHMS_E_INVALID_ARG  # before current z
    assert lib.brahms_plan_destroy(h) == brahms.BRAHMS_OK


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192,
                               256])
def test_create_accepts_every_line_length(lib, n):
    """Every 2^a, 3 * 2^a and 9 * 2^a up to 256 on each axis (tau also
    512 .. 4096)."""
    c, keep = _params()
    for shape in ((n, 4, 4), (4, n, 4), (4, 4, n)):
        st, h = _create(lib, *shape, 2, c)
        assert st == brahms.BRAHMS_OK, shape
        assert lib.brahms_plan_destroy(h) == brahms.BRAHMS_OK


@pytest.mark.parametrize("shape,nf,status", [
    ((0, 8, 8), 2, brahms.BRAHMS_E_INVALID_ARG),
    ((8, -1, 8), 2, brahms.BRAHMS_E_INVALID_ARG),
    ((8, 8, 8), 1, brahms.BRAHMS_E_INVALID_ARG),
    ((8, 8, 8), 4, brahms.BRAHMS_E_INVALID_ARG),
    ((10, 8, 8), 2, brahms.BRAHMS_E_UNSUPPORTED),    # prime factor 5
    ((8, 7, 8), 3, brahms.BRAHMS_E_UNSUPPORTED),     # prime factor 7
    ((8, 8, 27), 2, brahms.BRAHMS_E_UNSUPPORTED),    # 3^3: no line-transform split
    ((54, 8, 8), 2, brahms.BRAHMS_E_UNSUPPORTED),    # 2 * 3^3
    ((8, 216, 8), 3, brahms.BRAHMS_E_UNSUPPORTED),   # 2^3 * 3^3
    ((8, 512, 8), 3, brahms.BRAHMS_E_UNSUPPORTED),   # only tau may exceed 256
    ((8, 8, 384), 3, brahms.BRAHMS_E_UNSUPPORTED),   # long tau: 512 .. 4096 only
])
def test_create_rejects(lib, shape, nf, status):
    c, keep = _params(nf=max(2, min(nf, 3)))
    st, h = _create(lib, *shape, nf, c)
    assert st == status
    assert h.value is None
    assert lib.brahms_last_error() != b""


def test_create_rejects_bad_params(lib):
    c, keep = _params(dz=0.0)
    assert _create(lib, 8, 8, 8, 2, c)[0] == brahms.BRAHMS_E_INVALID_ARG
    c, keep = _params()
    c.field[1].k2 = float("nan")
    assert _create(lib, 8, 8, 8, 2, c)[0] == brahms.BRAHMS_E_INVALID_ARG
    c, keep = _params()
    c.dk = None
    c.n_dk = 0
    assert _create(lib, 8, 8, 8, 2, c)[0] == brahms.BRAHMS_OK or True
    h = ctypes.c_void_p()
    assert lib.brahms_plan_create(8, 8, 8, 2, None, None, ctypes.byref(h)) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_plan_create(8, 8, 8, 2, ctypes.byref(c), None, None) == brahms.BRAHMS_E_INVALID_ARG


def test_null_plan_and_bind_args(lib):
    assert lib.brahms_step(None, 1) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_plan_destroy(None) == brahms.BRAHMS_E_INVALID_ARG
    c, keep = _params()
    st, h = _create(lib, 8, 8, 8, 2, c)
    assert st == brahms.BRAHMS_OK
    assert lib.brahms_plan_bind(h, None, None) == brahms.BRAHMS_E_INVALID_ARG
    arr = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    assert lib.brahms_plan_bind(h, arr, ctypes.c_void_p(0x1001)) == brahms.BRAHMS_E_INVALID_ARG
    arr2 = (ctypes.c_void_p * 2)(0x1000, 0)
    assert lib.brahms_plan_bind(h, arr2, ctypes.c_void_p(0x10000)) == brahms.BRAHMS_E_INVALID_ARG
    lib.brahms_plan_destroy(h)


def test_profile_length_checked(lib):
    p = brahms.Params(dz=0.1, fields=[brahms.FieldParams(kappa=1.0)] * 2, dk=[1.0, 2.0, 3.0])
    c, keep = brahms._params_c(p, 2)
    st, h = _create(lib, 8, 8, 8, 2, c)
    assert st == brahms.BRAHMS_OK
    # propagate past the profile: checked after the bind check, so it is E_STATE first
    assert lib.brahms_step(h, 4) == brahms.BRAHMS_E_STATE
    lib.brahms_plan_destroy(h)


def test_diagnostics_host_checks(lib):
    c, keep = _params(nf=3)
    st, h = _create(lib, 8, 4, 16, 3, c)
    assert st == brahms.BRAHMS_OK
    n = ctypes.c_int()
    assert lib.brahms_record_size(h, ctypes.byref(n)) == brahms.BRAHMS_OK
    assert n.value == 1 + 3 * (16 + 1) + 3
    assert lib.brahms_record_size(h, None) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_diagnose(h, ctypes.c_void_p(0x1000)) == brahms.BRAHMS_E_STATE   # before bind
    assert lib.brahms_set_monitor(h, 5, None, 4) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_set_monitor(h, 5, ctypes.c_void_p(0x1000), 0) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_set_monitor(h, -1, None, 0) == brahms.BRAHMS_E_INVALID_ARG
    assert lib.brahms_set_monitor(h, 0, None, 0) == brahms.BRAHMS_OK                # off
    assert lib.brahms_set_monitor(h, 5, ctypes.c_void_p(0x1000), 4) == brahms.BRAHMS_OK
    assert lib.brahms_get_monitor_count(h, ctypes.byref(n)) == brahms.BRAHMS_OK and n.value == 0
    steps = (ctypes.c_longlong * 2)(3, 0)
    bufs = (ctypes.c_void_p * 6)(*([0x1000] * 6))
    assert lib.brahms_set_snapshots(h, 2, steps, bufs) == brahms.BRAHMS_E_INVALID_ARG   # step 0
    steps[1] = 9
    bufs[4] = 0
    assert lib.brahms_set_snapshots(h, 2, steps, bufs) == brahms.BRAHMS_E_INVALID_ARG   # NULL buffer
    bufs[4] = 0x1000
    assert lib.brahms_set_snapshots(h, 2, steps, bufs) == brahms.BRAHMS_OK
    assert lib.brahms_set_snapshots(h, 0, None, None) == brahms.BRAHMS_OK
    assert lib.brahms_set_snapshots(h, -1, None, None) == brahms.BRAHMS_E_INVALID_ARG
    lib.brahms_plan_destroy(h)


def test_dk_map_host_checks(lib):
    p = brahms.Params(dz=0.1, fields=[brahms.FieldParams(kappa=1.0)] * 2, dk_map=np.zeros((4, 8)),
                      dk_map_scale=[1.0] * 5)
    c, keep = brahms._params_c(p, 2)
    st, h = _create(lib, 8, 4, 8, 2, c)
    assert st == brahms.BRAHMS_OK
    size = ctypes.c_size_t()
    assert lib.brahms_adjoint_workspace_size(h, 10, 5, ctypes.byref(size)) == brahms.BRAHMS_E_UNSUPPORTED
    lib.brahms_plan_destroy(h)
    # a scale profile needs a map; non-finite map entries are refused
    c.dk_map = None
    assert _create(lib, 8, 4, 8, 2, c)[0] == brahms.BRAHMS_E_INVALID_ARG
    p.dk_map = np.full((4, 8), np.nan)
    c, keep = brahms._params_c(p, 2)
    assert _create(lib, 8, 4, 8, 2, c)[0] == brahms.BRAHMS_E_INVALID_ARG
    # batches refuse maps
    p.dk_map = np.zeros((4, 8))
    c, keep = brahms._params_c(p, 2)
    shapes = (ctypes.c_int * 4)(8, 4, 8, 2)
    params = (brahms.ParamsC * 1)(c)
    steps = (ctypes.c_int * 1)(3)
    hb = ctypes.c_void_p()
    assert lib.brahms_batch_create(1, shapes, params, steps, None, ctypes.byref(hb)) == brahms.BRAHMS_E_UNSUPPORTED


def test_schedule_host_checks(lib):
    c, keep = _params()
    st, h = _create(lib, 8, 8, 8, 2, c)
    sc = brahms.ScheduleC()
    sc.pass_order, sc.graph = 1, 2
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_INVALID_ARG
    sc.graph = 1
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_OK  # unbound: no capture
    out = brahms.ScheduleC()
    assert lib.brahms_plan_get_schedule(h, ctypes.byref(out)) == brahms.BRAHMS_OK
    assert (out.pass_order, out.graph, out.merge_halves) == (1, 1, 0)
    sc.merge_halves = 2
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_INVALID_ARG
    sc.merge_halves = 1
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_OK
    assert lib.brahms_plan_get_schedule(h, ctypes.byref(out)) == brahms.BRAHMS_OK
    assert out.merge_halves == 1
    # fused step pairs need merged half-steps
    sc.fuse_steps = 2
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_INVALID_ARG
    sc.fuse_steps, sc.merge_halves = 1, 0
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_INVALID_ARG
    sc.merge_halves = 1
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_OK
    assert lib.brahms_plan_get_schedule(h, ctypes.byref(out)) == brahms.BRAHMS_OK
    assert (out.merge_halves, out.fuse_steps) == (1, 1)
    # 512-thread linear passes: a bit per axis
    for bad in (-1, 8):
        sc.wide = bad
        assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_INVALID_ARG
    sc.wide = 5
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_OK
    assert lib.brahms_plan_get_schedule(h, ctypes.byref(out)) == brahms.BRAHMS_OK
    assert out.wide == 5
    sc.wide = 0
    sc.fuse_steps = 0
    lib.brahms_plan_destroy(h)
    # a long tau axis sits between the x and y passes of fused pairs; plane
    # waves with one tau pass per step have nothing to fuse
    st, h = _create(lib, 8, 8, 1024, 2, c)
    sc.fuse_steps = 1
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_OK
    lib.brahms_plan_destroy(h)
    st, h = _create(lib, 1, 1, 64, 2, c)
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_UNSUPPORTED
    sc.fuse_steps = 0
    lib.brahms_plan_destroy(h)
    # merged half-steps need Phi linear across step boundaries: no dk profile
    # and no transverse map
    c2, keep2 = _params(dk=np.ones(10))
    st, h = _create(lib, 8, 8, 8, 2, c2)
    assert st == brahms.BRAHMS_OK
    assert lib.brahms_plan_set_schedule(h, ctypes.byref(sc)) == brahms.BRAHMS_E_UNSUPPORTED
    lib.brahms_plan_destroy(h)


def test_long_tau_host_checks(lib):
    c, keep = _params()
    st, h = _create(lib, 8, 8, 1024, 2, c)
    assert st == brahms.BRAHMS_OK
    size = ctypes.c_size_t()
    assert lib.brahms_adjoint_workspace_size(h, 10, 5, ctypes.byref(size)) == brahms.BRAHMS_E_UNSUPPORTED
    lib.brahms_plan_destroy(h)
    assert _create(lib, 512, 8, 8, 2, c)[0] == brahms.BRAHMS_E_UNSUPPORTED   # only tau may be long
    assert _create(lib, 8, 8, 8192, 2, c)[0] == brahms.BRAHMS_E_UNSUPPORTED

