"""34^3 velocity grids (the paper's resolution in Sec. 3.2) on the GEM
set-up, in FP32 and FP64 storage: the V operator (FP32: one cell per CU, the
block filling its LDS; FP64: the block is twice the LDS, so the in-plane
sweeps run on half the v_x planes at a time), the moments (one block per
cell), the moment fit (FP64: two pencils per thread in registers, the rest in
LDS) and full steps against the oracle.  The V cases include shifts of
several cells (the v_x pencils' whole-cell path through the output block)."""
import numpy as np
import pytest

from gpu_util import TOL_MOM, TOL_STEP, TOL_SWEEP, dev, host, rel_l2, storage_round
from oracle import fields as OF
from oracle import moments as OMo
from oracle import step as OS
from oracle import vlasov as OV
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu
N = 34


def _grid(sp):
    v, dv = [], []
    for d in range(3):
        c, h = OV.centres(sp["v_lo"][d], sp["v_hi"][d], sp["nv"][d])
        v.append(c)
        dv.append(h)
    return v, dv


@pytest.fixture(scope="module")
def gem34():
    from gpu_util import ensure_lib
    ensure_lib()
    return W.gem(nx=4, ny=2, nv=N, dt=0.003, fit=True, dtype=np.float64)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("escale,bscale", [(0.1, 1.0), (40.0, 10.0)])
def test_v_operator_34(gem34, dtype, escale, bscale):
    """(0.1, 1): sub-cell shifts; (40, 10): electron shifts of about two
    cells from E and up to six from v x B at the box edge (whole-cell
    paths)."""
    from paper_2109_06743_amd import vl
    cfg, f, _ = gem34
    ny, nx = cfg["ny"], cfg["nx"]
    ctx = vl.Context(cfg, dtype)
    rng = np.random.default_rng(3)
    E = escale * rng.normal(size=(ny, nx, 3))
    B = bscale * rng.normal(size=(ny, nx, 3))
    for s, sp in enumerate(cfg["species"]):
        print(f"species {s} {dtype} E x{escale}", flush=True)
        v, dv = _grid(sp)
        fs = storage_round(f[s], dtype)
        fin = dev(fs, dtype)
        fout = fin.new_empty(fin.shape)
        ctx.pfc_advect_v(s, fin, fout, dev(E, "f64"), dev(B, "f64"), cfg["dt"])
        ctx.sync()
        ref = OV.v_advect_3v(fs, E, B, sp["q"], sp["m"], v, dv, cfg["dt"], f_inf=float(fs.max()))
        got = host(fout, ref.shape)
        for j in range(ny):
            for i in range(nx):
                assert rel_l2(got[j, i], ref[j, i]) < 3 * TOL_SWEEP[dtype], (s, j, i)
        assert abs(got.sum() - fs.sum()) <= (1e-6 if dtype == "f32" else 1e-13) * fs.sum()
        assert (got >= 0).all()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_moments_and_fit_34(gem34, dtype):
    import torch
    from paper_2109_06743_amd import vl
    cfg, f, _ = gem34
    ny, nx = cfg["ny"], cfg["nx"]
    ctx = vl.Context(cfg, dtype)
    for s, sp in enumerate(cfg["species"]):
        print(f"species {s} {dtype}", flush=True)
        v, dv = _grid(sp)
        f32 = storage_round(f[s], dtype)
        fin = dev(f32, dtype)
        mom = torch.zeros(nx * ny * 20, dtype=torch.float64, device="cuda")
        ctx.moments(s, fin, mom)
        ctx.sync()
        m_ref = OMo.raw_moments_3v(f32, v, dv, sp["m"])
        got = host(mom, m_ref.shape)
        for a, b in [(0, 1), (1, 4), (4, 10), (10, 20)]:
            den = max(np.linalg.norm(m_ref[..., a:b]), 1e-3 * np.abs(m_ref[..., 0]).max())
            assert np.linalg.norm(got[..., a:b] - m_ref[..., a:b]) / den < TOL_MOM[dtype], (s, a)
        # fluid state: shifted mean velocity, 5 % hotter
        d = OMo.derived_3v(m_ref, sp["m"])
        U = np.zeros((ny, nx, 10))
        for j in range(ny):
            for i in range(nx):
                n, u, T = d["n"][j, i], d["u"][j, i], d["T"][j, i]
                vt = np.sqrt(np.trace(T) / (3 * sp["m"]))
                u2 = u + np.array([0.05, -0.03, 0.02]) * vt
                P2 = n * 1.05 * T + sp["m"] * n * np.outer(u2, u2)
                U[j, i] = [n, *(n * u2), P2[0, 0], P2[0, 1], P2[0, 2], P2[1, 1], P2[1, 2], P2[2, 2]]
        fout = torch.empty_like(fin)
        post = torch.zeros_like(mom)
        ctx.moment_fit(s, fin, fout, mom, torch.from_numpy(U.reshape(-1).copy()).cuda(), post)
        ctx.sync()
        gotf = host(fout, f32.shape)
        gotp = host(post, m_ref.shape)
        for j in range(ny):
            for i in range(nx):
                ref, _, _, _ = OMo.fit_cell_3v(f32[j, i], m_ref[j, i], U[j, i], sp["m"], v, dv)
                assert rel_l2(gotf[j, i], ref) < (1e-5 if dtype == "f32" else 1e-12), (s, j, i)
                if dtype == "f64":
                    mp = OMo.raw_moments_3v(ref[None, None], v, dv, sp["m"])[0, 0]
                    assert np.linalg.norm(gotp[j, i] - mp) / np.linalg.norm(mp) < 1e-12, (s, j, i)


@pytest.mark.parametrize("dtype,vsplit", [("f32", "strang"), ("f64", "strang"), ("f32", "backsub")])
def test_step_34(gem34, dtype, vsplit):
    """Two full steps against the oracle; FP32 also with the backsubstitution
    velocity split (34^3 blocks: FP32 only)."""
    from paper_2109_06743_amd import vl
    cfg, f, F0 = gem34
    if vsplit == "backsub":
        cfg = dict(cfg, vsplit="backsub")
    nx, ny = cfg["nx"], cfg["ny"]
    F = OF.Yee(nx, ny)
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
    f = [storage_round(x, dtype) for x in f]
    moms, Us = [], []
    for k, sp in enumerate(cfg["species"]):
        v, dv = OS._grids(cfg, sp)
        mm = OMo.raw_moments_3v(f[k], v, dv, sp["m"])
        moms.append(mm)
        Us.append(mm[..., :10].copy())
    ctx = vl.Context(cfg, dtype)
    st = vl.StepState(ctx, f, vl.yee_pack(F), U_list=Us, mom_post_list=moms)
    ref = dict(f=f, U=[u.copy() for u in Us], mom_post=moms, F=F)
    for k in range(2):
        print(f"step {k} {dtype} {vsplit}", flush=True)
        ctx.step(st, cfg["dt"])
        ref = OS.step_2x3v(ref, cfg, cfg["dt"])
        ctx.sync()
        for s in range(2):
            got = host(st.f[s], ref["f"][s].shape)
            assert rel_l2(got, ref["f"][s]) < TOL_STEP[dtype] * (k + 1), (k, s)
            assert rel_l2(host(st.U[s], ref["U"][s].shape), ref["U"][s]) < (1e-5 if dtype == "f32" else 1e-12)
