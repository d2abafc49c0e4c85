"""GPU parity of the learned heat-flux closure (features, BF16-MFMA forward
and backward, Adam, the closure inside vl_step) against the FP64 oracle
(oracle/mlp.py), and the test of what the trained network gains over the
temperature-gradient closure of Eq. 5 on held-out data that the Vlasov solver
itself generated.

Tolerances: the network multiplies BF16 operands (8 significant bits) with
FP32 accumulation and rounds its hidden activations to BF16; the oracle runs
the same BF16-valued weights and features exactly in FP64.  Forward outputs
agree to rel-L2 1e-2 and gradients to 2e-2 (the BF16 bound: three layers of
2^-9 relative rounding on activations and on the back-propagated errors)."""
import math

import numpy as np
import pytest

from gpu_util import ensure_lib, host, rel_l2, storage_round
from oracle import fields as OF
from oracle import mlp as OM
from oracle import moments as OMo
from oracle import step as OS
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_lib()


def _t(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).contiguous().cuda()


def _bf16_values(bits):
    """uint16 BF16 patterns (as an int16 tensor) -> float64 numpy."""
    b = bits.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def _perturbed_gem_moments(nx, ny, nv, seed):
    """Raw moments of GEM-like f with a seeded modulation (non-Maxwellian,
    non-zero heat flux) for both species."""
    cfg, f, _ = W.gem(nx=nx, ny=ny, nv=nv, dt=0.003, fit=True, dtype=np.float64)
    rng = np.random.default_rng(seed)
    moms = []
    for k, sp in enumerate(cfg["species"]):
        v, dv = OS._grids(cfg, sp)
        mod = 1.0 + 0.3 * rng.uniform(-1, 1, size=f[k].shape)
        moms.append(OMo.raw_moments_3v(f[k] * mod, v, dv, sp["m"]))
    return cfg, moms


@pytest.mark.parametrize("nx,ny", [(13, 7), (150, 9)])
def test_features_and_targets_match_oracle(nx, ny):
    """13 x 7: one tile of the features kernel (64 columns x 4 rows) with
    ragged rows and columns; 150 x 9: three tiles per row and three rows of
    tiles, ragged at both ends, with the x wrap and the y mirror crossing
    tile edges."""
    import torch
    from paper_2109_06743_amd import vl
    nv = 8
    cfg, moms = _perturbed_gem_moments(nx, ny, nv, 3)
    ctx = vl.Context(cfg, "f32")
    cells = nx * ny
    Bf = np.random.default_rng(4).normal(size=(ny, nx, 3))
    Bf[2, 3] = 0.0                                       # a cell without field
    for s, sp in enumerate(cfg["species"]):
        for stride, arr, B in ((20, moms[s], None), (10, moms[s][..., :10], Bf), (20, moms[s], Bf)):
            x = torch.zeros(cells * 64, dtype=torch.int16, device="cuda")
            sc = torch.zeros(cells, dtype=torch.float64, device="cuda")
            ctx.mlp_features(s, _t(arr.reshape(-1), torch.float64), stride, x, sc,
                             B=None if B is None else _t(B.reshape(-1), torch.float64))
            ctx.sync()
            xr, scr = OM.features_bf16(arr, sp["m"], s, B)
            xg = _bf16_values(x).reshape(cells, 64)
            # FP64 rounding order may differ: allow one BF16 unit, and require
            # nearly every feature to be identical
            ulp = np.abs(xr) * 2.0 ** -8 + 1e-30
            assert np.all(np.abs(xg - xr) <= ulp), (s, stride)
            assert np.mean(xg == xr) > 0.99
            np.testing.assert_allclose(host(sc), scr, rtol=1e-13)
        y = torch.zeros(cells * 16, dtype=torch.float32, device="cuda")
        ctx.mlp_targets(s, _t(moms[s].reshape(-1), torch.float64), y)
        ctx.sync()
        yr = OM.targets(moms[s], sp["m"])
        assert np.abs(yr).max() > 1e-3
        np.testing.assert_allclose(host(y).reshape(cells, 16), yr, rtol=2e-6, atol=1e-9)


def _params(seed, w4_scale=1.0):
    p = W.mlp_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    d = OM.unpack(p)
    for k in ("b1", "b2", "b3"):
        d[k][:] = rng.normal(scale=0.1, size=d[k].shape)
    d["b4"][:10] = rng.normal(scale=0.1, size=10)
    d["W4"] *= w4_scale
    return OM.pack(d).astype(np.float32)


def _random_x(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(scale=0.7, size=(n, 64))
    x[:, 61:] = 0.0
    return OM.bf16_round(x.astype(np.float32)), OM.bf16_bits(x.astype(np.float32))


@pytest.mark.parametrize("n", [1, 16, 1000, 4099])
def test_forward_matches_oracle(n):
    import torch
    from paper_2109_06743_amd import vl
    cfg, _ = W.landau()
    ctx = vl.Context(dict(W.gem(nx=4, ny=2, nv=8)[0]), "f32")
    p = _params(1)
    xv, xb = _random_x(n, 2)
    y = torch.full((n * 16,), float("nan"), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(_t(p, torch.float32), _t(xb.view(np.int16), torch.int16).reshape(n, 64), y)
    ctx.sync()
    yr, _ = OM.forward(p, xv)
    yg = host(y).reshape(n, 16)
    assert rel_l2(yg[:, :10], yr[:, :10]) < 1e-2
    assert np.abs(yg[:, 10:] - yr[:, 10:]).max() < 1e-6      # padding rows: zero weights, bias b4[10:]


def test_parameters_off_16_byte_alignment_give_the_same_results():
    """The kernels stage the network into LDS with 16-byte loads when the
    parameter array allows it and element by element otherwise: both paths
    give bitwise the same outputs and gradients."""
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(dict(W.gem(nx=4, ny=2, nv=8)[0]), "f32")
    p = _params(3)
    n = 1000
    xv, xb = _random_x(n, 4)
    x = _t(xb.view(np.int16), torch.int16).reshape(n, 64)
    t = _t(np.random.default_rng(5).normal(size=(n, 16)).astype(np.float32), torch.float32)
    pa = _t(p, torch.float32)
    buf = torch.zeros(p.size + 1, dtype=torch.float32, device="cuda")
    pm = buf[1:]                                   # 4 bytes past a 16-byte boundary
    pm.copy_(pa)
    assert pa.data_ptr() % 16 == 0 and pm.data_ptr() % 16 == 4
    out = []
    for P in (pa, pm):
        y = torch.zeros(n * 16, dtype=torch.float32, device="cuda")
        ctx.mlp_forward(P, x, y)
        work = torch.zeros(ctx.mlp_work_size(n), dtype=torch.float32, device="cuda")
        gl = torch.zeros(vl.MLP_NPARAM + 1, dtype=torch.float32, device="cuda")
        ctx.mlp_gradient(P, x, t, work, gl)
        ctx.sync()
        out.append((host(y), host(gl)))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("n", [7, 777, 5000])
def test_gradient_matches_oracle(n):
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(dict(W.gem(nx=4, ny=2, nv=8)[0]), "f32")
    p = _params(4)
    xv, xb = _random_x(n, 5)
    rng = np.random.default_rng(6)
    t = np.zeros((n, 16), dtype=np.float32)
    t[:, :10] = rng.normal(scale=0.5, size=(n, 10))
    work = torch.zeros(ctx.mlp_work_size(n), dtype=torch.float32, device="cuda")
    gl = torch.zeros(OM.N_PARAM + 1, dtype=torch.float32, device="cuda")
    ctx.mlp_gradient(_t(p, torch.float32), _t(xb.view(np.int16), torch.int16).reshape(n, 64), _t(t, torch.float32),
                     work, gl)
    ctx.sync()
    L, g = OM.gradient(p, xv, t.astype(np.float64))
    got = host(gl)
    assert abs(got[-1] - L) / L < 1e-2
    for name, off, shape in OM._LAYOUT:
        size = int(np.prod(shape))
        a, b = got[off:off + size], g[off:off + size]
        if name in ("W4", "b4"):
            assert np.all(a.reshape(shape)[10:] == 0.0)
        assert rel_l2(a, b) < 2e-2, name
    # deterministic: a second evaluation is bitwise identical
    gl2 = torch.zeros_like(gl)
    ctx.mlp_gradient(_t(p, torch.float32), _t(xb.view(np.int16), torch.int16).reshape(n, 64), _t(t, torch.float32),
                     work, gl2)
    ctx.sync()
    assert torch.equal(gl, gl2)


def test_adam_step_matches_oracle_and_training_descends():
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(dict(W.gem(nx=4, ny=2, nv=8)[0]), "f32")
    n = 2048
    xv, xb = _random_x(n, 8)
    rng = np.random.default_rng(9)
    A = rng.normal(scale=0.15, size=(10, 64))
    t = np.zeros((n, 16), dtype=np.float32)
    t[:, :10] = np.tanh(xv @ A.T)
    P = _t(W.mlp_init(3), torch.float32)
    m1 = torch.zeros_like(P)
    m2 = torch.zeros_like(P)
    X = _t(xb.view(np.int16), torch.int16).reshape(n, 64)
    T = _t(t, torch.float32)
    work = torch.zeros(ctx.mlp_work_size(n), dtype=torch.float32, device="cuda")
    gl = torch.zeros(OM.N_PARAM + 1, dtype=torch.float32, device="cuda")
    p0 = host(P)
    ctx.mlp_train_step(P, m1, m2, 1, 1e-3, X, T, work, gl)
    ctx.sync()
    g = host(gl)[:-1]
    pr, _, _ = OM.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    np.testing.assert_allclose(host(P), pr, rtol=1e-5, atol=1e-7)
    losses = [host(gl)[-1]]
    for k in range(2, 301):
        ctx.mlp_train_step(P, m1, m2, k, 1e-3, X, T, work, gl)
        if k % 50 == 0:
            ctx.sync()
            losses.append(host(gl)[-1])
    assert losses[-1] < 0.2 * losses[0], losses
    d = OM.unpack(host(P))
    assert np.all(d["W4"][10:] == 0.0) and np.all(d["b4"][10:] == 0.0)


@pytest.mark.parametrize("n,batch,nsteps", [(3000, 512, 4), (12000, 5000, 2)])
def test_train_epoch_equals_train_steps_on_gathered_batches(n, batch, nsteps):
    """vl_mlp_train_epoch gathers the batch rows inside the gradient kernel:
    its parameters after the steps equal those of as many vl_mlp_train_step
    calls on the gathered batches (same kernels, same order: bitwise), and an
    index outside the rows counts as a padding row.  Batches of 512 rows give
    one 16-row tile per gradient block; 5000 rows give two per block (the
    next tile's rows are prefetched) and a half tile at the end."""
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(dict(W.gem(nx=4, ny=2, nv=8)[0]), "f32")
    xv, xb = _random_x(n, 11)
    rng = np.random.default_rng(12)
    t = np.zeros((n, 16), dtype=np.float32)
    t[:, :10] = np.tanh(xv @ rng.normal(scale=0.15, size=(10, 64)).T)
    X = _t(xb.view(np.int16), torch.int16).reshape(n, 64)
    T = _t(t, torch.float32)
    idx = torch.as_tensor(rng.permutation(n)[:nsteps * batch].astype(np.int64)).cuda()
    work = torch.zeros(ctx.mlp_work_size(batch), dtype=torch.float32, device="cuda")
    runs = []
    for mode in ("steps", "epoch"):
        P = _t(W.mlp_init(3), torch.float32)
        m1, m2 = torch.zeros_like(P), torch.zeros_like(P)
        gl = torch.zeros(OM.N_PARAM + 1, dtype=torch.float32, device="cuda")
        if mode == "steps":
            for k in range(nsteps):
                sel = idx[k * batch:(k + 1) * batch]
                ctx.mlp_train_step(P, m1, m2, 1 + k, 1e-3, X[sel].contiguous(), T[sel].contiguous(), work, gl)
        else:
            assert ctx.mlp_train_epoch(P, m1, m2, 1, 1e-3, X, T, idx, batch, work, gl) == nsteps
        ctx.sync()
        runs.append((host(P), host(gl)))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    # an out-of-range index is a padding row: no loss and no gradient of its own; a batch of
    # padding only gives exactly zero, one padding row leaves the gradient of the other rows scaled
    # by (batch - 1) / batch for the mean (up to the BF16 rounding of the scaled errors)
    P = _t(W.mlp_init(3), torch.float32)
    gl_0 = torch.full((OM.N_PARAM + 1,), 7.0, dtype=torch.float32, device="cuda")
    pad = torch.full((batch,), -1, dtype=torch.int64, device="cuda")
    pad[::2] = n + 3
    ctx.mlp_train_epoch(P.clone(), torch.zeros_like(P), torch.zeros_like(P), 1, 1e-3, X, T, pad, batch, work, gl_0)
    sel = idx[:batch].clone()
    sel[5] = n + 7
    gl_a = torch.zeros(OM.N_PARAM + 1, dtype=torch.float32, device="cuda")
    ctx.mlp_train_epoch(P.clone(), torch.zeros_like(P), torch.zeros_like(P), 1, 1e-3, X, T, sel, batch, work, gl_a)
    keep = torch.cat([sel[:5], sel[6:]])
    gl_b = torch.zeros(OM.N_PARAM + 1, dtype=torch.float32, device="cuda")
    ctx.mlp_gradient(P, X[keep].contiguous(), T[keep].contiguous(), work, gl_b)
    ctx.sync()
    assert not host(gl_0).any()
    ga, gb = host(gl_a), host(gl_b) * ((batch - 1) / batch)
    assert rel_l2(ga[:-1], gb[:-1]) < 2e-2
    assert abs(ga[-1] - gb[-1]) <= 1e-5 * gb[-1]


# ------------------------------------------------------ closure in a step --
def _start(cfg, f, F0, dtype, params):
    from paper_2109_06743_amd import vl
    F = OF.Yee(cfg["nx"], cfg["ny"])
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
    st = vl.StepState(ctx, f, vl.yee_pack(F), U_list=Us, mom_post_list=moms, mlp_params=params)
    ref = dict(f=f, U=[u.copy() for u in Us], mom_post=moms, F=F, mlp_params=params.astype(np.float64))
    return ctx, st, ref


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_closure_step_matches_oracle(dtype):
    """The network's third moment drives the fluid (tolerance so large that the
    judge never falls back); the GPU's fallback flags are fed to the oracle."""
    nx, ny, nv = 8, 4, 16
    cfg, f, F0 = W.gem(nx=nx, ny=ny, nv=nv, dt=0.003, fit=True, dtype=np.float64)
    cfg = dict(cfg, closure="mlp", closure_tol=1e30)
    params = _params(11, w4_scale=0.05)
    ctx, st, ref = _start(cfg, f, F0, dtype, params)
    for k in range(2):
        ctx.step(st, cfg["dt"])
        ctx.sync()
        fb = host(st.closure_fallback).astype(bool).tolist()
        assert fb == [False, False]
        ref = OS.step_2x3v(dict(ref, fallback=fb), cfg, cfg["dt"])
        ref["mlp_params"] = params.astype(np.float64)
        np.testing.assert_allclose(host(st.closure_err), ref["closure_err"], rtol=2e-2)
        for s in range(2):
            # the network's BF16 rounding enters U through dt div(Q): its
            # relative effect on U and f stays within a few 1e-6 per step
            tol = (2e-5 if dtype == "f32" else 1e-5) * (k + 1)
            assert rel_l2(host(st.U[s], ref["U"][s].shape), ref["U"][s]) < tol, (k, s)
            assert rel_l2(host(st.f[s], ref["f"][s].shape), ref["f"][s]) < tol, (k, s)


def test_closure_fallback_equals_kinetic_step():
    """closure_tol = 0: every step falls back, and the result is bitwise that of
    the kinetic-closure step."""
    import torch
    nx, ny, nv = 8, 4, 8
    cfg, f, F0 = W.gem(nx=nx, ny=ny, nv=nv, dt=0.003, fit=True, dtype=np.float64)
    params = _params(12)
    ctx_k, st_k, _ = _start(cfg, f, F0, "f32", params)
    ctx_m, st_m, _ = _start(dict(cfg, closure="mlp", closure_tol=0.0), f, F0, "f32", params)
    for _ in range(3):
        ctx_k.step(st_k, cfg["dt"])
        ctx_m.step(st_m, cfg["dt"])
    ctx_k.sync()
    ctx_m.sync()
    assert host(st_m.closure_fallback).tolist() == [1.0, 1.0]
    assert np.all(host(st_m.closure_err) > 0)
    for s in range(2):
        assert torch.equal(st_k.f[s], st_m.f[s])
        assert torch.equal(st_k.U[s], st_m.U[s])
    assert torch.equal(st_k.fields, st_m.fields)


# ------------------------------------------------------------- the gain ----
def _gem_snapshots(nx, ny, nv, steps, every, start, psi0=0.1):
    """Run the GEM set-up (initial perturbation psi0) on the GPU (FP32 f,
    fitting on) and collect the post-step raw moments of both species and the
    cell-centred B every `every` steps."""
    import torch
    from paper_2109_06743_amd import vl
    cfg, f, F0 = W.gem(nx=nx, ny=ny, nv=nv, dt=0.003, fit=True, dtype=np.float32, psi0=psi0)
    ctx = vl.Context(cfg, "f32")
    st = vl.StepState(ctx, f, vl.yee_pack(F0))
    cells = nx * ny
    E = torch.zeros(cells * 3, dtype=torch.float64, device="cuda")
    snaps = []
    for k in range(1, steps + 1):
        ctx.step(st, cfg["dt"])
        if k >= start and k % every == 0:
            B = torch.zeros(cells * 3, dtype=torch.float64, device="cuda")
            ctx.cell_fields(st.fields, E, B)
            snaps.append(([m.clone() for m in st.mom_pre], B))
    ctx.sync()
    return cfg, ctx, snaps


def _features(ctx, snaps, cells):
    import torch
    xs, ys, ss = [], [], []
    for mom, B in snaps:
        for s in range(2):
            x = torch.zeros(cells, 64, dtype=torch.int16, device="cuda")
            sc = torch.zeros(cells, dtype=torch.float64, device="cuda")
            y = torch.zeros(cells, 16, dtype=torch.float32, device="cuda")
            ctx.mlp_features(s, mom[s], 20, x, sc, B=B)
            ctx.mlp_targets(s, mom[s], y)
            xs.append(x)
            ys.append(y)
            ss.append(sc)
    return xs, ys, ss


def test_trained_network_beats_gradient_closure():
    """Train on the solver's own moments and kinetic heat flux (GEM set-up,
    32x16 x 16^3, both species, 1500 steps), with batches drawn with
    probability proportional to n m v_t^3 (the weight the heat flux carries),
    then evaluate on a run held out whole: the same set-up with another
    initial perturbation (psi0 0.15 instead of 0.1).  Per species, the error
    of the heat-flux divergence (the term the fluid update uses) and of the
    heat-flux vector q_i = Q_ijj (the in-step judge's measure) is compared
    with four predictors that need no training data or only its mean: zero
    (error 1 exactly), the per-component mean of the normalised training
    targets, and Eq. 5's temperature-gradient closure (divergence only)."""
    import torch
    nx, ny, nv = 32, 16, 16
    cells = nx * ny
    cfg, ctx, train = _gem_snapshots(nx, ny, nv, steps=1500, every=15, start=60)
    _, _, held = _gem_snapshots(nx, ny, nv, steps=600, every=30, start=60, psi0=0.15)
    xs, ys, ss = _features(ctx, train, cells)
    X = torch.cat(xs).contiguous()
    Y = torch.cat(ys).contiguous()
    w = torch.cat(ss).float()
    w = w / w.mean() + 1e-3
    mean_y = host(Y[:, :10].double().mean(0))
    n = X.shape[0]
    P = _t(W.mlp_init(0), torch.float32)
    m1 = torch.zeros_like(P)
    m2 = torch.zeros_like(P)
    batch = 4096
    work = torch.zeros(ctx.mlp_work_size(batch), dtype=torch.float32, device="cuda")
    gl = torch.zeros(OM.N_PARAM + 1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    step = 0
    epochs = 96
    for epoch in range(epochs):
        idx = torch.multinomial(w, n, replacement=True, generator=gen)
        step += ctx.mlp_train_epoch(P, m1, m2, step + 1, 2e-3 * 0.5 ** (epoch // (epochs // 4)), X, Y, idx, batch,
                                    work, gl)
    ctx.sync()
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    J = np.zeros((10, 3))
    for c, d in ((0, 0), (3, 0), (5, 0), (1, 1), (6, 1), (8, 1), (2, 2), (7, 2), (9, 2)):
        J[c, d] = 1.0                      # q_i = Q_ijj over the ten ordered triples
    res = {}
    for s, sp in enumerate(cfg["species"]):
        e = {k: [] for k in ("div_net", "div_grad", "div_mean", "q_net", "q_mean")}
        for momt, B in held:
            x = torch.zeros(cells, 64, dtype=torch.int16, device="cuda")
            sc = torch.zeros(cells, dtype=torch.float64, device="cuda")
            y = torch.zeros(cells, 16, dtype=torch.float32, device="cuda")
            ctx.mlp_features(s, momt[s], 20, x, sc, B=B)
            ctx.mlp_forward(P, x, y)
            ctx.sync()
            mom = host(momt[s]).reshape(ny, nx, 20)
            scale = host(sc).reshape(ny, nx, 1)
            Qk = OM.heat_flux(mom, sp["m"])
            Qn = scale * host(y).reshape(ny, nx, 16)[..., :10]
            Qm = scale * mean_y
            dk = OM.divergence_heat_flux(Qk, dx, dy)
            e["div_net"].append(rel_l2(OM.divergence_heat_flux(Qn, dx, dy), dk))
            e["div_mean"].append(rel_l2(OM.divergence_heat_flux(Qm, dx, dy), dk))
            e["div_grad"].append(rel_l2(OM.gradient_closure_divergence(mom[..., :10], sp["m"], sp["q"], dx, dy), dk))
            e["q_net"].append(rel_l2(Qn @ J, Qk @ J))
            e["q_mean"].append(rel_l2(Qm @ J, Qk @ J))
        res[s] = {k: float(np.mean(v)) for k, v in e.items()}
        print(f"species {s} held-out run: " + ", ".join(f"{k} {v:.3f}" for k, v in res[s].items()), flush=True)
    # measured on the held-out run: electrons div 0.60, q 0.51 (Eq. 5: div 1.25; mean predictor: div 1.11,
    # q 1.36); ions div 0.27, q 0.30 (Eq. 5: div 13.6; mean predictor: div 0.99, q 1.10)
    bars = {0: (0.75, 0.65), 1: (0.4, 0.45)}
    for s in range(2):
        r = res[s]
        assert r["div_net"] < bars[s][0] and r["q_net"] < bars[s][1], (s, r)     # zero predictor: 1, 1
        assert r["div_net"] < r["div_grad"], (s, r)
        assert r["div_net"] < r["div_mean"] - 0.2 and r["q_net"] < r["q_mean"] - 0.3, (s, r)
