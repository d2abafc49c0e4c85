"""vl_moment_fit_noalloc (the allocation-free variant of vl_moment_fit, its
scratch in a static device array) against vl_moment_fit through the C ABI:
two calls in a row, the second with a smaller grid (the static array then
still holds the first call's larger contents), FP32 and FP64, 16^3, 12^3
and 1V grids; f, the rescaled fluid state, the post-fit moments and the
clip/skip counters agree bitwise (the same kernels, fixed-order sums), and f
matches the oracle's fit within the per-call bound."""
import numpy as np
import pytest

from gpu_util import TOL_SWEEP, dev, ensure_lib, host, rel_l2, storage_round
from oracle import moments as OM
from oracle import step as OS
from oracle import vlasov as OV
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_lib()


def _fluid_from(mom, m, du, tscale):
    d = OM.derived_3v(mom, m)
    n = d["n"] * 1.01
    u = d["u"] + du
    T = d["T"] * tscale
    U = np.zeros(mom.shape[:-1] + (10,))
    U[..., 0] = n
    U[..., 1:4] = n[..., None] * u
    for k, (a, b) in enumerate(OM.PAIRS):
        U[..., 4 + k] = n * T[..., a, b] + m * n * u[..., a] * u[..., b]
    return U


def _run_pair(cfg, dtype, s, f, U, mom):
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(cfg, dtype)
    cells = cfg["nx"] * cfg.get("ny", 1)
    k = mom.shape[-1]
    out = {}
    for name in ("alloc", "noalloc"):
        fin = dev(f, dtype)
        fout = torch.empty_like(fin)
        Ud = dev(U, "f64")
        post = torch.full((cells * k,), -7.0, dtype=torch.float64, device="cuda")
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        call = ctx.moment_fit if name == "alloc" else ctx.moment_fit_noalloc
        call(s, fin, fout, dev(mom, "f64"), Ud, post, cnt)
        ctx.sync()
        out[name] = (fout.cpu().numpy(), Ud.cpu().numpy(), post.cpu().numpy(), cnt.cpu().numpy())
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("nv", [16, 12])
def test_noalloc_fit_matches_fit_3v(dtype, nv):
    for nx, ny in ((40, 30), (11, 5)):                  # the second call on a smaller grid
        cfg, f0, _ = W.gem(nx=nx, ny=ny, nv=nv, dtype=np.float64)
        for s, sp in enumerate(cfg["species"]):
            v, dv = OS._grids(cfg, sp)
            f = storage_round(f0[s] * (1 + 0.3 * W.random_block(f0[s].shape, seed=70 + s + nx, kind="rough")),
                              dtype)
            mom = OM.raw_moments_3v(f, v, dv, sp["m"])
            vt = np.sqrt(0.5 / sp["m"]) * 0.3
            U = _fluid_from(mom, sp["m"], np.array([0.3, -0.2, 0.1]) * vt, 1.1)
            U[1, 2, 4] = -1.0                            # one skipped cell
            out = _run_pair(cfg, dtype, s, f, U, mom)
            a, b = out["alloc"], out["noalloc"]
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
            assert b[3][1] == 1
            ref_f, ref_U, _, _ = OM.moment_fit_3v(f, mom, U, sp["m"], v, dv)
            assert rel_l2(b[0].astype(np.float64).reshape(ref_f.shape), ref_f) < TOL_SWEEP[dtype] * 3


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_fit_matches_fit_1v(dtype):
    cfg, f0 = W.twostream(nx=16, nv=80)
    f = storage_round(f0, dtype)
    v, dv = OV.centres(cfg["v_lo"], cfg["v_hi"], 80)
    mom = OM.raw_moments_1v(f, v, dv, cfg["m"])
    d = OM.derived_1v(mom, cfg["m"])
    n, u, T = d["n"] * 1.02, d["u"] + 0.2, d["T"] * 0.8
    U = np.stack([n, n * u, n * T + cfg["m"] * n * u * u], axis=-1)
    out = _run_pair(cfg, dtype, 0, f, U, mom)
    for x, y in zip(out["alloc"], out["noalloc"]):
        np.testing.assert_array_equal(x, y)
