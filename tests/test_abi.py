"""The C-ABI library loads, exports every function include/vl.h declares, and
rejects bad arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2109_06743_amd import build as B
from paper_2109_06743_amd import vl, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB):
        B.build()
    return vl.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vl_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_exported(lib):
    names = declared_functions()
    assert len(names) >= 15, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(vl.EXPORTS) <= set(names)


def test_status_strings(lib):
    for code in range(7):
        assert lib.vl_status_str(code)
    assert b"gfx950" in lib.vl_version()


def _create(cfg, dtype="f32"):
    c = vl.make_config(cfg, dtype)
    h = ctypes.c_void_p()
    st = vl.load().vl_create(ctypes.byref(c), ctypes.byref(h))
    return st, h


def test_create_validates_on_host(lib):
    cfg, _ = workloads.landau(nx=16, nv=16)
    st, h = _create(cfg)
    assert st == 0 and h.value
    assert lib.vl_yee_size(h) == 0
    assert lib.vl_step_work_size(h) > 0
    assert lib.vl_destroy(h) == 0
    bad = dict(cfg, nx=0)
    assert _create(bad)[0] == 1
    bad = dict(cfg, v_hi=cfg["v_lo"])
    assert _create(bad)[0] == 1
    bad = dict(cfg, m=-1.0)
    assert _create(bad)[0] == 1


def test_create_2x3v_checks(lib):
    cfg, _, _ = workloads.gem(nx=4, ny=2, nv=4, dtype="float64")
    st, h = _create(cfg, "f64")
    assert st == 0
    assert lib.vl_yee_size(h) == 4 * (3 * 2 + 3 * 3)
    lib.vl_destroy(h)
    sp = [dict(s) for s in cfg["species"]]
    sp[0]["v_lo"] = [-1.0, -2.0, -1.0]          # v_y grid not symmetric: reflecting walls impossible
    assert _create(dict(cfg, species=sp))[0] == 1
    sp = [dict(s) for s in cfg["species"]]
    sp[1]["nv"] = [40, 4, 4]                    # longer pencils than the velocity kernel supports
    assert _create(dict(cfg, species=sp))[0] == 3


def test_entry_points_reject_bad_arguments_before_device_use(lib):
    cfg, _ = workloads.landau(nx=16, nv=16)
    st, h = _create(cfg)
    p = ctypes.c_void_p(0x1000)                 # never dereferenced: validation fails first
    q = ctypes.c_void_p(0x2000)
    assert lib.vl_pfc_advect_x(h, 0, None, p, 0.1, None) == 1
    assert lib.vl_pfc_advect_x(h, 0, p, q, -0.1, None) == 1
    assert lib.vl_pfc_advect_x(h, 0, p, q, float("nan"), None) == 1
    assert lib.vl_pfc_advect_x(h, 0, p, p, 0.1, None) == 2
    assert lib.vl_pfc_advect_x(h, 1, p, q, 0.1, None) == 1
    assert lib.vl_pfc_advect_v(h, 0, p, p, q, None, 0.1, None) == 2
    assert lib.vl_pfc_advect_v(h, 0, p, q, None, None, 0.1, None) == 1
    assert lib.vl_moments(h, 0, None, p, None) == 1
    assert lib.vl_moment_fit(h, 0, p, p, None, q, None, None, None) == 1
    assert lib.vl_maxwell_half_step(h, p, ctypes.c_void_p(0x3000), 0.1, None) == 3
    s = vl.State()
    assert lib.vl_step(h, ctypes.byref(s), 0.1, None) == 1
    assert lib.vl_step(h, None, 0.1, None) == 1
    fs = vl.FluidClosureState()
    assert lib.vl_fluid_closure_step(h, ctypes.byref(fs), 0, 0.1, None) == 3    # 1X1V: no ten-moment fluid
    assert lib.vl_fluid_closure_work_size(h) == 0
    assert b"" != lib.vl_last_error(h)
    lib.vl_destroy(h)


def test_cube34_grids(lib):
    cfg = dict(kind="2x3v", nx=4, ny=2, x_lo=0.0, x_hi=1.0, y_lo=-1.0, y_hi=1.0, c=20.0, fit=True,
               species=[dict(q=-1.0, m=0.04, v_lo=[-1.0] * 3, v_hi=[1.0] * 3, nv=[34] * 3)])
    for dt in ("f32", "f64"):
        st, h = _create(cfg, dt)
        assert st == 0
        lib.vl_destroy(h)
    st, h = _create(dict(cfg, vsplit="backsub"), "f32")
    assert st == 0                                  # the FP32 block fills one CU's LDS
    lib.vl_destroy(h)
    st, h = _create(dict(cfg, vsplit="backsub"), "f64")
    assert st == 3                                  # the FP64 block does not fit the LDS
    cfg["species"][0]["nv"] = [34, 34, 33]           # non-cubic beyond the generic limits
    st, h = _create(cfg, "f32")
    assert st == 3


def test_periodic_y_and_the_network_closure(lib):
    cfg, _, _ = workloads.orszag_tang(n=8, nv=4)
    st, h = _create(cfg)
    assert st == 0
    lib.vl_destroy(h)
    st, h = _create(dict(cfg, closure="mlp", closure_tol=0.5))
    assert st == 3                                  # the network's features mirror at walls
    c = vl.make_config(cfg)
    c.bc_y = 7
    h = ctypes.c_void_p()
    assert lib.vl_create(ctypes.byref(c), ctypes.byref(h)) == 1


def test_fluid_closure_step_rejects_bad_arguments(lib):
    cfg, _, _ = workloads.gem_fluid(nx=8, ny=4)
    st, h = _create(cfg)
    assert lib.vl_fluid_closure_work_size(h) > 0
    fs = vl.FluidClosureState()
    fs.U[0], fs.U[1], fs.fields, fs.work = 0x1000, 0x2000, 0x3000, 0x4000
    assert lib.vl_fluid_closure_step(h, ctypes.byref(fs), 7, 0.1, None) == 1        # unknown closure
    assert lib.vl_fluid_closure_step(h, ctypes.byref(fs), 0, -0.1, None) == 1
    assert lib.vl_fluid_closure_step(h, ctypes.byref(fs), 1, 0.1, None) == 1        # network closure, no params
    fs.U[1] = 0x1000
    assert lib.vl_fluid_closure_step(h, ctypes.byref(fs), 0, 0.1, None) == 2        # U[0] aliases U[1]
    fs.U[1], fs.work = 0x2000, None
    assert lib.vl_fluid_closure_step(h, ctypes.byref(fs), 0, 0.1, None) == 1
    assert lib.vl_fluid_closure_step(h, None, 0, 0.1, None) == 1
    lib.vl_destroy(h)


def test_create_rejects_rows_of_4_gib(lib):
    """A row of f (nx velocity blocks) is addressed with 32-bit byte offsets."""
    sp = [dict(q=-1.0, m=0.04, v_lo=[-1.0] * 3, v_hi=[1.0] * 3, nv=[16] * 3)]
    cfg = dict(kind="2x3v", nx=131071, ny=2, x_lo=0.0, x_hi=1.0, y_lo=-1.0, y_hi=1.0, c=20.0, fit=True, species=sp)
    st, h = _create(cfg, "f64")                      # 131071 * 4096 * 8 B < 4 GiB
    assert st == 0
    lib.vl_destroy(h)
    assert _create(dict(cfg, nx=131072), "f64")[0] == 3
    st, h = _create(dict(cfg, nx=262143), "f32")
    assert st == 0
    lib.vl_destroy(h)
    assert _create(dict(cfg, nx=262144), "f32")[0] == 3


def test_mlp_train_epoch_rejects_bad_arguments(lib):
    cfg, _ = workloads.landau(nx=16, nv=16)
    st, h = _create(cfg)
    p = ctypes.c_void_p(0x1000)                 # never dereferenced: validation fails first
    y = ctypes.c_void_p(0x2000)
    f = lib.vl_mlp_train_epoch
    assert f(h, None, p, p, 1, 1e-3, p, y, 10, p, 4, 2, p, p, None) == 1          # null params
    assert f(h, p, p, p, 1, 1e-3, p, y, 10, None, 4, 2, p, p, None) == 1          # null indices
    assert f(h, p, p, p, 1, 1e-3, p, y, 10, p, 4, 0, p, p, None) == 1             # no steps
    assert f(h, p, p, p, 0, 1e-3, p, y, 10, p, 4, 2, p, p, None) == 1             # Adam steps count from 1
    assert f(h, p, p, p, 1, float("nan"), p, y, 10, p, 4, 2, p, p, None) == 1     # learning rate
    assert f(h, p, p, p, 1, 1e-3, ctypes.c_void_p(0x1001), y, 10, p, 4, 2, p, p, None) == 1   # x alignment
    lib.vl_destroy(h)


def test_noalloc_fit_rejects_oversized_grid_on_host(lib):
    """vl_moment_fit_noalloc holds the scratch of at most 49152 spatial cells:
    a larger context is refused before any device call."""
    cfg, f, _ = workloads.gem(nx=8, ny=4, nv=8)
    big = dict(cfg, nx=256, ny=256)                      # 65536 cells
    st, h = _create(big)
    assert st == 0
    p = ctypes.c_void_p(256)
    assert lib.vl_moment_fit_noalloc(h, 0, p, p, p, p, None, None, None) == 1
    assert b"49152" in lib.vl_last_error(h)
    assert lib.vl_moment_fit_noalloc(h, 0, None, p, p, p, None, None, None) == 1
    assert lib.vl_moment_fit_noalloc(h, 2, p, p, p, p, None, None, None) == 1
    assert lib.vl_destroy(h) == 0
