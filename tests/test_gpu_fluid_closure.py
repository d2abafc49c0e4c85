"""The ten-moment fluid model run with a heat-flux closure
(vl_fluid_closure_step) against the oracle, step by step: the Eq. 5
gradient closure (FP64 throughout, so the fluid states and fields agree to
rounding) and the network closure (BF16 network on the device, the same
BF16-valued network in FP64 in the oracle), on the GEM set-up at 40 x 18 (a
full and a partial tile of x faces per row, three tile rows of y faces)."""
import numpy as np
import pytest

from gpu_util import host, rel_l2
from oracle import fields as OF
from oracle import step as OS
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(nx, ny):
    cfg, U, F0 = W.gem_fluid(nx=nx, ny=ny)
    F = OF.Yee(nx, ny)
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
    return cfg, U, F


@pytest.mark.parametrize("closure,tol_u,tol_f", [("gradient", 1e-12, 1e-12), ("mlp", 2e-5, 1e-6)])
def test_fluid_closure_step_matches_oracle(closure, tol_u, tol_f):
    from gpu_util import ensure_lib
    from paper_2109_06743_amd import vl
    ensure_lib()
    nx, ny = 40, 18
    cfg, U, F = _setup(nx, ny)
    params = W.mlp_init(0) if closure == "mlp" else None
    ctx = vl.Context(cfg, "f64")
    fs = vl.FluidState(ctx, U, vl.yee_pack(F), mlp_params=params)
    ref = {"U": [u.copy() for u in U], "F": F}
    for k in range(3):
        print(f"{closure} step {k}", flush=True)
        ctx.fluid_closure_step(fs, cfg["dt"], closure)
        ref = OS.fluid_step_2x3v(ref, cfg, cfg["dt"], closure, params)
        ctx.sync()
        for s in range(2):
            got = host(fs.U[s], ref["U"][s].shape)
            assert rel_l2(got, ref["U"][s]) < tol_u * (k + 1), (closure, k, s)
        yee = vl.yee_unpack(host(fs.fields), nx, ny)
        for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            r = getattr(ref["F"], c)
            assert np.abs(yee[c] - r).max() <= tol_f * (k + 1) * max(np.abs(r).max(), 1.0), (closure, k, c)


def test_gradient_closure_changes_the_step():
    """The closure term is live: the same step without heat flux (network
    closure with a zero network) differs from the gradient-closure step."""
    from gpu_util import ensure_lib
    from paper_2109_06743_amd import vl
    ensure_lib()
    nx, ny = 40, 18
    cfg, U, F = _setup(nx, ny)
    ctx = vl.Context(cfg, "f64")
    a = vl.FluidState(ctx, U, vl.yee_pack(F))
    b = vl.FluidState(ctx, U, vl.yee_pack(F), mlp_params=np.zeros(vl.MLP_NPARAM, dtype=np.float32))
    ctx.fluid_closure_step(a, cfg["dt"], "gradient")
    ctx.fluid_closure_step(b, cfg["dt"], "mlp")
    ctx.sync()
    ref = OS.fluid_step_2x3v({"U": [u.copy() for u in U], "F": F}, cfg, cfg["dt"], "gradient")
    for s in range(2):
        ga, gb = host(a.U[s], U[s].shape), host(b.U[s], U[s].shape)
        assert rel_l2(ga, ref["U"][s]) < 1e-12
        assert rel_l2(ga, gb) > 1e-9, s
