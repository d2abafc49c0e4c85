"""Periodic y (the Orszag-Tang set-up, Sec. 3.2) against the oracle: the
fused X operator on a ragged grid (x strips, and 128-row segments of both
cyclic pencils with a short last one), full steps with moment fitting, and the fluid
model alone with the Eq. 5 closure."""
import numpy as np
import pytest

from gpu_util import TOL_STEP, TOL_SWEEP, dev, host, rel_l2, storage_round
from oracle import fields as OF
from oracle import moments as OM
from oracle import step as OS
from oracle import vlasov as OV
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu


def _yee(F0, nx, ny):
    F = OF.Yee(nx, ny)
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
    return F


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_x_operator_periodic(dtype):
    import torch
    from gpu_util import ensure_lib
    from paper_2109_06743_amd import vl
    ensure_lib()
    cfg, f, _ = W.orszag_tang(n=20, ny=140, nv=8, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    ctx = vl.Context(cfg, dtype)
    tau = 2.0 * cfg["dt"]
    for s, sp in enumerate(cfg["species"]):
        v, _ = OS._grids(cfg, sp)
        fin = storage_round(f[s], dtype)
        ref = OV.x_advect_2x3v(fin, v[0], v[1], dx, dy, tau, f_inf=float(fin.max()), bc_y="periodic")
        fi = dev(fin, dtype)
        fo = torch.empty_like(fi)
        ctx.pfc_advect_x(s, fi, fo, tau)
        ctx.sync()
        got = host(fo, ref.shape)
        assert rel_l2(got, ref) < 2 * TOL_SWEEP[dtype], (dtype, s)
        assert abs(got.sum() - fin.sum()) <= (1e-6 if dtype == "f32" else 1e-12) * fin.sum()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_periodic(dtype):
    from gpu_util import ensure_lib
    from paper_2109_06743_amd import vl
    ensure_lib()
    cfg, f, F0 = W.orszag_tang(n=12, nv=8, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    F = _yee(F0, nx, ny)
    f = [storage_round(x, dtype) for x in f]
    moms, Us = [], []
    for k, sp in enumerate(cfg["species"]):
        v, dv = OS._grids(cfg, sp)
        mm = OM.raw_moments_3v(f[k], v, dv, sp["m"])
        moms.append(mm)
        Us.append(mm[..., :10].copy())
    ctx = vl.Context(cfg, dtype)
    st = vl.StepState(ctx, f, vl.yee_pack(F), U_list=Us, mom_post_list=moms)
    ref = dict(f=f, U=[u.copy() for u in Us], mom_post=moms, F=F)
    for k in range(3):
        print(f"{dtype} step {k}", flush=True)
        ctx.step(st, cfg["dt"])
        ref = OS.step_2x3v(ref, cfg, cfg["dt"])
        ctx.sync()
        for s in range(2):
            got = host(st.f[s], ref["f"][s].shape)
            assert rel_l2(got, ref["f"][s]) < TOL_STEP[dtype] * (k + 1), (k, s)
            assert rel_l2(host(st.U[s], ref["U"][s].shape), ref["U"][s]) < (1e-5 if dtype == "f32" else 1e-12)
        yee = vl.yee_unpack(host(st.fields), nx, ny)
        for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            r = getattr(ref["F"], c)
            np.testing.assert_allclose(yee[c], r, rtol=0, atol=(1e-6 if dtype == "f32" else 1e-12), err_msg=c)


def test_fluid_closure_periodic():
    from gpu_util import ensure_lib
    from paper_2109_06743_amd import vl
    ensure_lib()
    cfg, f, F0 = W.orszag_tang(n=16, ny=12, nv=8, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    F = _yee(F0, nx, ny)
    Us = []
    for k, sp in enumerate(cfg["species"]):
        v, dv = OS._grids(cfg, sp)
        Us.append(OM.raw_moments_3v(f[k], v, dv, sp["m"])[..., :10].copy())
    ctx = vl.Context(cfg, "f64")
    fs = vl.FluidState(ctx, Us, vl.yee_pack(F))
    ref = {"U": [u.copy() for u in Us], "F": F}
    for k in range(3):
        ctx.fluid_closure_step(fs, cfg["dt"], "gradient")
        ref = OS.fluid_step_2x3v(ref, cfg, cfg["dt"], "gradient")
        ctx.sync()
        for s in range(2):
            assert rel_l2(host(fs.U[s], ref["U"][s].shape), ref["U"][s]) < 1e-12 * (k + 1), (k, s)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_periodic_34(dtype):
    """The Orszag-Tang configuration itself at a small grid: periodic y with
    34^3 velocity blocks (FP32: the block fills one CU's LDS; FP64: half its
    v_x planes at a time), two full steps against the oracle."""
    from gpu_util import ensure_lib
    from paper_2109_06743_amd import vl
    ensure_lib()
    cfg, f, F0 = W.orszag_tang(n=4, nv=34, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    F = _yee(F0, nx, ny)
    f = [storage_round(x, dtype) for x in f]
    moms, Us = [], []
    for k, sp in enumerate(cfg["species"]):
        v, dv = OS._grids(cfg, sp)
        mm = OM.raw_moments_3v(f[k], v, dv, sp["m"])
        moms.append(mm)
        Us.append(mm[..., :10].copy())
    ctx = vl.Context(cfg, dtype)
    st = vl.StepState(ctx, f, vl.yee_pack(F), U_list=Us, mom_post_list=moms)
    ref = dict(f=f, U=[u.copy() for u in Us], mom_post=moms, F=F)
    for k in range(2):
        print(f"{dtype} 34^3 periodic step {k}", flush=True)
        ctx.step(st, cfg["dt"])
        ref = OS.step_2x3v(ref, cfg, cfg["dt"])
        ctx.sync()
        for s in range(2):
            got = host(st.f[s], ref["f"][s].shape)
            assert rel_l2(got, ref["f"][s]) < TOL_STEP[dtype] * (k + 1), (k, s)
            assert rel_l2(host(st.U[s], ref["U"][s].shape), ref["U"][s]) < (1e-5 if dtype == "f32" else 1e-12)
        yee = vl.yee_unpack(host(st.fields), nx, ny)
        for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            np.testing.assert_allclose(yee[c], getattr(ref["F"], c), rtol=0,
                                       atol=(1e-6 if dtype == "f32" else 1e-12), err_msg=c)
