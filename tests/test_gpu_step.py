"""GPU parity of the full time step (vl_step, Algorithm 1) against the CPU
oracle's step: both trajectories start from the same state and are compared
after every step (f by rel-L2, moments per group, fields, fluid state), plus
conservation and determinism properties of the GPU path.

Workloads: Landau damping 64x64 (Sec. 3.1 set-up, the cfg of the headline
small case), two-stream 96x128, GEM-like 2X3V grids (Sec. 3.3 geometry at
reduced size) with FP32 and FP64 storage, moment fitting on and off."""
import numpy as np
import pytest

from gpu_util import TOL_STEP, ensure_lib, host, rel_l2, storage_round
from oracle import fields as OF
from oracle import moments as OM
from oracle import step as OS
from oracle import vlasov as OV
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_lib()


def _start_1x1v(cfg, f, dtype):
    from paper_2109_06743_amd import vl
    f = storage_round(f, dtype)
    v, dv = OV.centres(cfg["v_lo"], cfg["v_hi"], cfg["nv"])
    mom = OM.raw_moments_1v(f, v, dv, cfg["m"])
    ctx = vl.Context(cfg, dtype)
    st = vl.StepState(ctx, [f], np.zeros(cfg["nx"]), U_list=[mom[:, :3]], mom_post_list=[mom])
    ref = {"f": f, "mom_post": mom, "U": mom[:, :3].copy()}
    return ctx, st, ref


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("fit", [False, True])
@pytest.mark.parametrize("which", ["landau", "twostream"])
def test_step_1x1v(dtype, fit, which):
    if which == "landau":
        cfg, f = W.landau(fit=fit)
        steps = 8
    else:
        cfg, f = W.twostream(nx=96, nv=128, fit=fit)
        steps = 5
    ctx, st, ref = _start_1x1v(cfg, f, dtype)
    dt = cfg["dt"]
    for k in range(steps):
        ctx.step(st, dt)
        ref = OS.step_1x1v(ref, cfg, dt)
        ctx.sync()
        got = host(st.f[0], ref["f"].shape)
        assert rel_l2(got, ref["f"]) < TOL_STEP[dtype] * (k + 1), k
        # E is the small fluctuation of the density: its FP32 error is the density's
        # rounding (1e-7 of n) over the perturbation amplitude
        E = host(st.fields)
        assert rel_l2(E, ref["E_half"]) < (2e-5 if dtype == "f32" else 1e-11), k
        mp = host(st.mom_post[0], ref["mom_post"].shape)
        assert rel_l2(mp, ref["mom_post"]) < (1e-5 if dtype == "f32" else 1e-12)
        if fit:
            assert rel_l2(host(st.U[0], ref["U"].shape), ref["U"]) < (1e-5 if dtype == "f32" else 1e-12)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("fit", [False, True])
@pytest.mark.parametrize("nx", [1, 2, 3])
def test_step_1x1v_degenerate_grids(dtype, fit, nx):
    """One to three periodic cells: the x windows and the fluid's ghost cells
    wrap onto the same cells, and at nx <= 2 the spectral Poisson solve has
    no mode below the Nyquist one (E = 0)."""
    cfg, f = W.landau(nx=nx, nv=16, fit=fit)
    ctx, st, ref = _start_1x1v(cfg, f, dtype)
    for k in range(4):
        ctx.step(st, cfg["dt"])
        ref = OS.step_1x1v(ref, cfg, cfg["dt"])
        ctx.sync()
        got = host(st.f[0], ref["f"].shape)
        assert rel_l2(got, ref["f"]) < TOL_STEP[dtype] * (k + 1), k
        assert (got >= 0).all()
        # FP32 storage rounds the density to 1e-7 of n: E (about 1.6e-2 at nx = 3)
        # within 1e-6 absolute, as in the rel-L2 bound of the Landau steps
        np.testing.assert_allclose(host(st.fields), ref["E_half"], rtol=0,
                                   atol=(1e-6 if dtype == "f32" else 1e-12))
        if fit:
            assert rel_l2(host(st.U[0], ref["U"].shape), ref["U"]) < (1e-5 if dtype == "f32" else 1e-12)


def _start_2x3v(cfg, f, F0, dtype):
    from paper_2109_06743_amd import vl
    F = OF.Yee(cfg["nx"], cfg["ny"])
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
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
    return ctx, st, ref


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("fit", [False, True])
@pytest.mark.parametrize("shape", [(8, 4, 8), (12, 6, 12), (40, 20, 8)])
def test_step_2x3v(dtype, fit, shape):
    """(40, 20, 8): several x strips of the fused X operator and full plus
    partial tiles of fluid faces in both directions."""
    from paper_2109_06743_amd import vl
    nx, ny, nv = shape
    cfg, f, F0 = W.gem(nx=nx, ny=ny, nv=nv, dt=0.003, fit=fit, dtype=np.float64)
    ctx, st, ref = _start_2x3v(cfg, f, F0, dtype)
    for k in range(3):
        ctx.step(st, cfg["dt"])
        ref = OS.step_2x3v(ref, cfg, cfg["dt"])
        ctx.sync()
        for s in range(2):
            got = host(st.f[s], ref["f"][s].shape)
            assert rel_l2(got, ref["f"][s]) < TOL_STEP[dtype] * (k + 1), (k, s)
            if fit:
                assert rel_l2(host(st.U[s], ref["U"][s].shape), ref["U"][s]) < (1e-5 if dtype == "f32" else 1e-12)
        # fields are O(1) in B0 and v_A B0 units; E itself stays ~1e-7 here because
        # j almost balances curl B, so the bound is absolute on the field scale
        yee = vl.yee_unpack(host(st.fields), nx, ny)
        for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            r = getattr(ref["F"], c)
            np.testing.assert_allclose(yee[c], r, rtol=0, atol=(1e-6 if dtype == "f32" else 1e-12), err_msg=c)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("fit", [False, True])
@pytest.mark.parametrize("nx,ny", [(1, 2), (2, 3), (3, 2)])
def test_step_2x3v_degenerate_grids(dtype, fit, nx, ny):
    """The smallest grids the library accepts: one to three cells along x (the
    x windows and the fluid faces' ghosts wrap onto the same few cells) and
    two or three rows between the walls (the mirrored pencils and ghost rows
    cover the whole grid).  f, the fluid state and the fields follow the
    oracle over three steps."""
    from paper_2109_06743_amd import vl
    cfg, f, F0 = W.gem(nx=nx, ny=ny, nv=8, dt=0.003, fit=fit, dtype=np.float64)
    ctx, st, ref = _start_2x3v(cfg, f, F0, dtype)
    for k in range(3):
        ctx.step(st, cfg["dt"])
        ref = OS.step_2x3v(ref, cfg, cfg["dt"])
        ctx.sync()
        for s in range(2):
            got = host(st.f[s], ref["f"][s].shape)
            assert rel_l2(got, ref["f"][s]) < TOL_STEP[dtype] * (k + 1), (k, s)
            assert (got >= 0).all()
            if fit:
                assert rel_l2(host(st.U[s], ref["U"][s].shape), ref["U"][s]) < (1e-5 if dtype == "f32" else 1e-12)
        yee = vl.yee_unpack(host(st.fields), nx, ny)
        for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            np.testing.assert_allclose(yee[c], getattr(ref["F"], c), rtol=0,
                                       atol=(1e-6 if dtype == "f32" else 1e-12), err_msg=c)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("nv", [(8, 12, 10), (6, 4, 20)])
def test_step_2x3v_general_blocks(dtype, nv):
    """Non-cubic velocity blocks (the general V operator, moments and fit
    kernels) through full moment-fitting steps on a 10 x 6 grid."""
    from paper_2109_06743_amd import vl
    nx, ny = 10, 6
    cfg, f, F0 = W.gem(nx=nx, ny=ny, nv=8, dt=0.003, fit=True, dtype=np.float64)
    cfg["species"] = [dict(sp, nv=list(nv)) for sp in cfg["species"]]
    f = []
    for sp in cfg["species"]:
        v, dv = OS._grids(cfg, sp)
        u = np.zeros((ny, nx, 3))
        u[..., 2] = 0.05 * sp["v_hi"][2]
        # thermal speed sqrt(T/m) about a third of the velocity box
        T = np.broadcast_to(np.eye(3) * (0.12 * sp["m"] * sp["v_hi"][0] ** 2), (ny, nx, 3, 3))
        n = 1.0 + 0.1 * np.cos(2 * np.pi * (np.arange(nx) + 0.5) / nx)[None, :] * np.ones((ny, 1))
        f.append(np.stack([np.stack([OM.maxwellian_3v(n[j, i], u[j, i], T[j, i], sp["m"], v, dv)
                                     for i in range(nx)]) for j in range(ny)]))
    ctx, st, ref = _start_2x3v(cfg, f, F0, dtype)
    for k in range(3):
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


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_conserves_mass_and_is_deterministic(dtype):
    import torch
    from paper_2109_06743_amd import vl
    cfg, f, F0 = W.gem(nx=16, ny=8, nv=8, dt=0.003, fit=True, dtype=np.float64)
    runs = []
    for rep in range(2):
        ctx, st, _ = _start_2x3v(cfg, f, F0, dtype)
        m0 = [x.double().sum().item() for x in st.f]
        for _ in range(4):
            ctx.step(st, cfg["dt"])
        ctx.sync()
        for s in range(2):
            m1 = st.f[s].double().sum().item()
            assert abs(m1 - m0[s]) / m0[s] < (2e-6 if dtype == "f32" else 1e-13)
            assert (st.f[s] >= 0).all().item()
        runs.append([x.clone() for x in st.f] + [st.fields.clone()])
    for a, b in zip(*runs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_kept_maximum_matches_recomputed(dtype):
    """The limiter bound max f of each step comes from the per-block maxima of
    the kernel that wrote f (reduced in two launches once there are more than
    8192 partials: 128 x 72 cells).  Steps that take the kept maximum and
    steps told to recompute it from f (f_max_valid = 0) give the same f and
    fields bit for bit."""
    import torch
    cfg, f, F0 = W.gem(nx=128, ny=72, nv=8, dt=0.003, fit=True, dtype=np.float64)
    runs = []
    for recompute in (False, True):
        ctx, st, _ = _start_2x3v(cfg, f, F0, dtype)
        for _ in range(3):
            if recompute:
                st.c.f_max_valid = 0
            ctx.step(st, cfg["dt"])
        ctx.sync()
        runs.append([x.clone() for x in st.f] + [st.fields.clone()])
    for a, b in zip(*runs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_2x3v_one_species(dtype):
    """Electrons alone (the fluid kernels launched for a set of one species
    inside the step), three steps with moment fitting against the oracle."""
    from paper_2109_06743_amd import vl
    cfg, f, F0 = W.gem(nx=12, ny=6, nv=8, dt=0.003, fit=True, dtype=np.float64)
    cfg = dict(cfg, species=cfg["species"][:1])
    ctx, st, ref = _start_2x3v(cfg, f[:1], F0, dtype)
    for k in range(3):
        ctx.step(st, cfg["dt"])
        ref = OS.step_2x3v(ref, cfg, cfg["dt"])
        ctx.sync()
        got = host(st.f[0], ref["f"][0].shape)
        assert rel_l2(got, ref["f"][0]) < TOL_STEP[dtype] * (k + 1), k
        assert rel_l2(host(st.U[0], ref["U"][0].shape), ref["U"][0]) < (1e-5 if dtype == "f32" else 1e-12), k
