"""Throughput of the full moment-fitting Vlasov step on one MI355X.

A step is one vl_step (Algorithm 1: Maxwell half step, X(dt/2), V(dt),
X(dt/2), moments, ten-moment fluid RK3, moment fitting, Maxwell half step)
over all phase-space cells of both species, with inputs resident in HBM.

Headline workload: the large-domain magnetotail-like reconnection set-up
(Sec. 4.1 geometry) on 1024 x 512 spatial cells x 12^3 velocity cells x 2
species (m_i/m_e = 100, guide field 0.1), FP32 f with FP64 moments, fitting
and fields, the largest of the benchmark configurations (1.81e9 phase-space
cells).  The same workload runs with FP64 f for the FP32 speed-up.  The GEM
set-up (Sec. 3.3 geometry, 256 x 128 x 16^3) is reported beside it, and the
learned heat-flux closure is trained and run on that geometry.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "phase-space cell-updates/s per full step (FP32 vs FP64) + % of HBM peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name):
    from paper_2109_06743_amd import workloads as W
    if name == "gem":
        cfg, f, F = W.gem(nx=256, ny=128, nv=16, dt=0.003, fit=True, dtype=np.float32)
        label = "GEM 2X3V 256x128 x 16^3 x 2 species, mi/me=25, moment fitting"
    elif name == "gem34":
        cfg, f, F = W.gem(nx=128, ny=64, nv=34, dt=0.003, fit=True, dtype=np.float32)
        label = "GEM 2X3V 128x64 x 34^3 x 2 species, mi/me=25, moment fitting"
    elif name == "ot":
        # the paper's Orszag-Tang grid, 41 GB of f per species: generated on the GPU
        cfg, f, F = W.orszag_tang_device(n=512, nv=34, dtype="f32")
        label = "Orszag-Tang 2X3V 512x512 x 34^3 x 2 species, periodic, mi/me=100, moment fitting"
    elif name == "tail":
        cfg, f, F = W.tail(nx=1024, ny=512, nv=12, dt=0.0012, fit=True, dtype=np.float32)
        label = "magnetotail 2X3V 1024x512 x 12^3 x 2 species, mi/me=100, Bg=0.1, moment fitting"
    else:
        raise SystemExit(f"unknown workload {name}")
    return cfg, f, F, label


def _nelem(x):
    """Element count of a numpy array or a torch tensor."""
    return x.numel() if hasattr(x, "numel") else x.size


def total_energy(ctx, st):
    """(mass per species, kinetic+thermal energy, field energy) of a step state."""
    import torch
    me = torch.zeros(2, dtype=torch.float64, device="cuda")
    fe = torch.zeros(1, dtype=torch.float64, device="cuda")
    mass, kin = [], 0.0
    for s in range(len(st.f)):
        ctx.mass_energy(s, st.f[s], st.mom_post[s], me)
        mass.append(me[0].item())
        kin += me[1].item()
    ctx.field_energy(st.fields, fe)
    return mass, kin, fe.item()


def run_gpu(cfg, f, F, dtype, steps, warmup, mlp_params=None):
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(cfg, dtype)
    st = vl.StepState(ctx, f, vl.yee_pack(F), mlp_params=mlp_params)
    torch.cuda.synchronize()
    ncells = sum(x.numel() for x in st.f)
    mass0, kin0, fld0 = total_energy(ctx, st)
    # The first warm-up step (code-object loading, the initial max f) runs
    # untimed; the others run with every kernel category timed: the
    # per-category breakdown, and which f-pass kernel dominates.
    nb = max(warmup - 1, 1)                              # warm-up steps in the breakdown
    if warmup > 1:
        ctx.step(st, cfg["dt"])
        ctx.sync()
    ctx.timing_enable(True)
    for _ in range(nb):
        ctx.step(st, cfg["dt"])
    ctx.sync()
    breakdown = ctx.timing_read()
    dominant = max(ALG_BYTES_PER_CELL, key=lambda k: breakdown[k][0])
    # The library launches every kernel on the stream it is given (torch's
    # current stream here) and brackets the launches of the timed category
    # with HIP events on that same stream; only the dominant kernel is timed
    # inside the timed region, so the step is perturbed by two event records
    # per launch of that kernel and no more.
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.timing_enable([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        ctx.step(st, cfg["dt"])
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = a.elapsed_time(b) / steps
    ctx.sync()
    tim = ctx.timing_read()
    ctx.timing_enable(False)
    mass1, kin1, fld1 = total_energy(ctx, st)
    cnt = st.counters.cpu().numpy().tolist()
    e0, e1 = kin0 + fld0, kin1 + fld1
    res = dict(ms=ms, wall=wall, ncells=ncells, timing=tim, breakdown=breakdown, breakdown_steps=nb,
               warmup=warmup, dominant=dominant,
               energy_rel_drift=(e1 - e0) / e0, mass_rel_drift=max(abs(b - a) / a for a, b in zip(mass0, mass1)),
               steps_run=max(warmup, 1) + steps, counters=cnt, elem=4 if dtype == "f32" else 8)
    if mlp_params is not None:
        res["closure_err"] = st.closure_err.cpu().numpy().tolist()
        res["closure_fallback"] = st.closure_fallback.cpu().numpy().tolist()
    del st, ctx
    torch.cuda.empty_cache()
    return res


# kernel category -> (source files of its kernels, kernel name in the profiles)
KERNEL_SOURCES = {
    "pfc_x": ("pfc_kernels.hip", "pfc_xy_kernel"),    # 2X3V: x and y sweeps fused
    "pfc_v": ("pfc_kernels.hip", "pfc_v3_cube_kernel"),
    "fit": ("moment_kernels.hip", "fit3_cube_kernel"),
    "moments": ("moment_kernels.hip", "moments3_cube_kernel"),
}


def kernel_source_hash(category):
    """Hash of the sources a kernel category is built from (its .hip file and
    the shared device headers): a change invalidates recorded counters."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2109_06743_amd", "csrc")
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[category][0], "vl_common.h", "vl_internal.h"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(category, workload):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE runs
    (scaled by the copy-kernel calibration), or None when there is no record
    for this kernel and workload or its sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    for r in rec.get("records", []):
        if r.get("category") == category and r.get("workload") == workload:
            return r["bytes_per_launch"] if r.get("source_hash") == kernel_source_hash(category) else None
    return None


# Algorithmic bytes per phase-space cell and launch, in units of the f
# element size: one read and one write of one species' f (moments: one read);
# halo re-reads and the small spatial arrays are not counted.
ALG_BYTES_PER_CELL = {"pfc_x": 2, "pfc_v": 2, "fit": 2, "moments": 1}


def roofline(res, workload):
    """Dominant f-pass kernel: algorithmic bytes per launch / mean launch time
    of its launches inside the timed region."""
    k = res["dominant"]
    tot, n = res["timing"][k]
    avg_s = tot / n * 1e-3
    alg = ALG_BYTES_PER_CELL[k] * res["elem"] * res["cells_per_launch"]
    achieved = alg / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(k, workload), "kernel": k,
            "avg_launch_ms": round(tot / n, 4), "algorithmic_bytes_per_launch": alg}


def calibrate_copy(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters: FETCH_SIZE / WRITE_SIZE of this copy are compared with nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def _closure_snapshots(ctx, st, cfg, steps, start, every, keep, after_step=None):
    """Run `steps` steps of the kinetic (moment-fitting) solver and, every
    `every` steps from `start`, store the network features, the normalised
    kinetic heat flux and the scale n m v_t^3 of every cell and species
    (keep(k) says whether snapshot k is stored).  Returns lists of tensors
    and (step, species) labels."""
    import torch
    cells = cfg["nx"] * cfg["ny"]
    Ec = torch.zeros(cells * 3, dtype=torch.float64, device="cuda")
    Bc = torch.zeros(cells * 3, dtype=torch.float64, device="cuda")
    X, Y, S, K = [], [], [], []
    for k in range(1, steps + 1):
        ctx.step(st, cfg["dt"])
        if after_step is not None:
            after_step()
        if k >= start and k % every == 0 and keep(k):
            ctx.cell_fields(st.fields, Ec, Bc)
            for s in range(2):
                x = torch.zeros(cells, 64, dtype=torch.int16, device="cuda")
                sc = torch.zeros(cells, dtype=torch.float64, device="cuda")
                y = torch.zeros(cells, 16, dtype=torch.float32, device="cuda")
                ctx.mlp_features(s, st.mom_pre[s], 20, x, sc, B=Bc)
                ctx.mlp_targets(s, st.mom_pre[s], y)
                X.append(x)
                Y.append(y)
                S.append(sc)
                K.append((k, s))
    return X, Y, S, K


def _heat_flux_vector_error(ctx, P, X, Y, S):
    """Relative L2 error over the rows of the heat-flux vector q_i = Q_ijj
    (the in-step judge's measure) of the network against the kinetic targets,
    and the same for the per-component mean of the targets as predictor."""
    import torch
    # q_i = Q_ijj over the ten ordered triples (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz)
    J = torch.zeros(10, 3, dtype=torch.float64, device="cuda")
    for c, d in ((0, 0), (3, 0), (5, 0), (1, 1), (6, 1), (8, 1), (2, 2), (7, 2), (9, 2)):
        J[c, d] = 1.0
    yh = torch.zeros_like(Y)
    ctx.mlp_forward(P, X, yh)
    qk = (Y[:, :10].double() * S[:, None]) @ J
    qn = (yh[:, :10].double() * S[:, None]) @ J
    qm = (Y[:, :10].double().mean(0)[None, :] * S[:, None]) @ J
    den = qk.norm().item()
    return (qn - qk).norm().item() / den, (qm - qk).norm().item() / den


def _train_network(ctx, X, Y, w, epochs, batch, lr, seed):
    """Adam on the library's BF16-MFMA gradient: `epochs` passes of len(X)
    samples drawn with probability proportional to w (inverse of the
    cumulative weights), lr halved every quarter of the epochs."""
    import torch
    from paper_2109_06743_amd import vl, workloads as W
    P = torch.as_tensor(W.mlp_init(seed)).cuda()
    m1, m2 = torch.zeros_like(P), torch.zeros_like(P)
    work = torch.zeros(ctx.mlp_work_size(batch), dtype=torch.float32, device="cuda")
    gl = torch.zeros(vl.MLP_NPARAM + 1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = X.shape[0]
    cdf = torch.cumsum(w.double(), 0)
    step = 0
    losses = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for ep in range(epochs):
        lr_ep = lr * 0.5 ** (ep // (epochs // 4))
        u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen) * cdf[-1]
        idx = torch.searchsorted(cdf, u).clamp_(max=n - 1)
        # one call per epoch: the batches idx[k*batch:(k+1)*batch] are gathered in the gradient kernel
        step += ctx.mlp_train_epoch(P, m1, m2, step + 1, lr_ep, X, Y, idx, batch, work, gl)
        losses.append(gl[-1].item())
    b.record()
    torch.cuda.synchronize()
    return P, losses, step, a.elapsed_time(b)


def train_closure(cfg, f, F, gen_steps=3000, start=60, every=15, epochs=96, batch=16384, lr=2e-3, seed=0,
                  closure_steps=600, other_psi0=0.15, other_steps=600):
    """Learned heat-flux closure on the benchmark geometry.  The solver
    generates its own training data: features (with the cell-centred field
    direction) and normalised kinetic heat flux of every cell and species
    every `every` steps after `start` over a `gen_steps`-step run; every fifth
    snapshot is held out.  The network is trained with the library's
    BF16-MFMA gradient and Adam calls on batches drawn with probability
    proportional to each sample's scale n m v_t^3 (the in-step judge weighs
    cells by their heat flux, which scales so).  Then the solver runs
    `closure_steps` steps from the data run's end with that network as its
    closure (judge tolerance 1, so the states are the ones the closure
    produces; the targets stay the kinetic heat flux of f), those snapshots
    join the training set and the network is trained again from its initial
    weights.  A run with a different initial perturbation (psi0 = other_psi0)
    is held out whole.  Returns the parameters, figures, and the solver state
    at the end of the kinetic data run."""
    import torch
    from paper_2109_06743_amd import vl, workloads as W
    ctx = vl.Context(cfg, "f32")
    st = vl.StepState(ctx, f, vl.yee_pack(F))
    t0 = time.perf_counter()
    snaps = [k for k in range(start, gen_steps + 1) if k % every == 0]
    held = {k for i, k in enumerate(snaps) if i % 5 == 2}
    X, Y, S, K = _closure_snapshots(ctx, st, cfg, gen_steps, start, every, lambda k: True)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    tr = [i for i, (k, s) in enumerate(K) if k not in held]
    ho = [i for i, (k, s) in enumerate(K) if k in held]
    Xh = torch.cat([X[i] for i in ho]).contiguous()
    Yh = torch.cat([Y[i] for i in ho]).contiguous()
    Sh = torch.cat([S[i] for i in ho])
    Xtr, Ytr, Str = [X[i] for i in tr], [Y[i] for i in tr], [S[i] for i in tr]
    del X, Y, S
    end = dict(f=[x.clone() for x in st.f], fields=st.fields.clone(), U=[u.clone() for u in st.U],
               mom_post=[m.clone() for m in st.mom_post], t=gen_steps * cfg["dt"])
    del st

    def heldout_Q(P):
        yh = torch.zeros_like(Yh)
        ctx.mlp_forward(P, Xh, yh)
        torch.cuda.synchronize()
        d = (yh[:, :10] - Yh[:, :10]).double()
        return (d.norm() / Yh[:, :10].double().norm()).item()

    # round 1: the kinetic run's snapshots
    Xt, Yt = torch.cat(Xtr).contiguous(), torch.cat(Ytr).contiguous()
    w = torch.cat(Str).float()
    P1, _, steps1, ms1 = _train_network(ctx, Xt, Yt, w / w.mean() + 1e-3, epochs, batch, lr, seed)
    q1 = heldout_Q(P1)
    del Xt, Yt
    # the states the closure produces, with kinetic targets
    ctx_c = vl.Context(dict(cfg, closure="mlp", closure_tol=1.0), "f32")
    st_c = vl.StepState(ctx_c, end["f"], end["fields"], U_list=end["U"], mom_post_list=end["mom_post"],
                        mlp_params=P1.cpu().numpy())
    fb = torch.zeros(2, dtype=torch.int64, device="cuda")

    def count_fallbacks():
        fb.add_(st_c.closure_fallback.to(torch.int64))
    t1 = time.perf_counter()
    Xc, Yc, Sc, _ = _closure_snapshots(ctx_c, st_c, cfg, closure_steps, every, every, lambda k: True,
                                       after_step=count_fallbacks)
    torch.cuda.synchronize()
    closure_s = time.perf_counter() - t1
    fb1 = fb.cpu().numpy().tolist()
    del st_c, ctx_c
    # round 2: both sets, from the initial weights
    Xt, Yt = torch.cat(Xtr + Xc).contiguous(), torch.cat(Ytr + Yc).contiguous()
    w = torch.cat(Str + Sc).float()
    n_train = Xt.shape[0]
    del Xtr, Ytr, Xc, Yc
    P, losses, step, train_ms = _train_network(ctx, Xt, Yt, w / w.mean() + 1e-3, epochs, batch, lr, seed)
    del Xt, Yt
    n_held = Xh.shape[0]
    heldout = heldout_Q(P)
    cells = cfg["nx"] * cfg["ny"]
    same = {}
    for s, name in enumerate(("electrons", "ions")):
        rows = torch.cat([torch.arange(j * cells, (j + 1) * cells, device="cuda")
                          for j, i in enumerate(ho) if K[i][1] == s])
        e_net, e_mean = _heat_flux_vector_error(ctx, P, Xh[rows].contiguous(), Yh[rows].contiguous(), Sh[rows])
        same[name] = {"network": round(e_net, 4), "mean_predictor": round(e_mean, 4), "zero_predictor": 1.0}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    yh = torch.zeros_like(Yh)
    a.record()
    for _ in range(5):
        ctx.mlp_forward(P, Xh, yh)
    b.record()
    torch.cuda.synchronize()
    inf_ms = a.elapsed_time(b) / 5
    # a run with another initial perturbation, held out whole
    cfg_o, f_o, F_o = W.gem(nx=cfg["nx"], ny=cfg["ny"], nv=cfg["species"][0]["nv"][0], dt=cfg["dt"], fit=True,
                            dtype=np.float32, psi0=other_psi0)
    st_o = vl.StepState(ctx, f_o, vl.yee_pack(F_o))
    Xo, Yo, So, Ko = _closure_snapshots(ctx, st_o, cfg_o, other_steps, 60, 60, lambda k: True)
    other = {}
    for s, name in enumerate(("electrons", "ions")):
        rows = [i for i, (k, sp) in enumerate(Ko) if sp == s]
        e_net, e_mean = _heat_flux_vector_error(ctx, P, torch.cat([Xo[i] for i in rows]).contiguous(),
                                                torch.cat([Yo[i] for i in rows]).contiguous(),
                                                torch.cat([So[i] for i in rows]))
        other[name] = {"network": round(e_net, 4), "mean_predictor": round(e_mean, 4), "zero_predictor": 1.0}
    del st_o, Xo, Yo, So, Xh, Yh, ctx
    torch.cuda.empty_cache()
    return P.cpu().numpy(), {
        "samples": n_train + n_held, "train_samples": n_train, "heldout_samples": n_held, "data_steps": gen_steps,
        "data_seconds": round(gen_s, 2), "closure_data_steps": closure_steps,
        "closure_data_seconds": round(closure_s, 2), "closure_data_fallback_steps": fb1,
        "round1_heldout_rel_l2_Q": round(q1, 4), "round1_train_ms": round(ms1, 1), "round1_adam_steps": steps1,
        "epochs": epochs, "batch": batch, "adam_steps": step,
        "sampling": "probability proportional to n m v_t^3",
        "train_ms": round(train_ms, 1), "train_samples_per_s": round(step * batch / (train_ms * 1e-3)),
        "loss_per_epoch": [round(x, 6) for x in losses[::max(len(losses) // 16, 1)]], "heldout_rel_l2_Q": round(heldout, 4),
        "heldout_rel_l2_heat_flux_vector": same,
        "heldout_other_run": {"psi0": other_psi0, "steps": other_steps, "snapshot_every": 60,
                              "rel_l2_heat_flux_vector": other},
        "forward_samples_per_s": round(n_held / (inf_ms * 1e-3))}, end


def run_closure(cfg, end, params, steps, warmup):
    """The step with the learned closure from the state the data run ended in
    (the conditions the network was trained on)."""
    import torch
    from paper_2109_06743_amd import vl
    ctx = vl.Context(cfg, "f32")
    st = vl.StepState(ctx, end["f"], end["fields"], U_list=end["U"], mom_post_list=end["mom_post"],
                      mlp_params=params)
    ncells = sum(x.numel() for x in st.f)
    mass0, kin0, fld0 = total_energy(ctx, st)
    for _ in range(warmup):
        ctx.step(st, cfg["dt"])
    torch.cuda.synchronize()
    fb = torch.zeros(2, dtype=torch.int64, device="cuda")
    errs = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        ctx.step(st, cfg["dt"])
        fb += st.closure_fallback.to(torch.int64)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    mass1, kin1, fld1 = total_energy(ctx, st)
    err = st.closure_err.cpu().numpy().tolist()
    e0, e1 = kin0 + fld0, kin1 + fld1
    del st, ctx
    torch.cuda.empty_cache()
    return dict(ms=ms, ncells=ncells, closure_err=err, fallback_steps=fb.cpu().numpy().tolist(),
                energy_rel_drift=(e1 - e0) / e0, mass_rel_drift=max(abs(b - a) / a for a, b in zip(mass0, mass1)))


def run_fluid_closure(nx, ny, closure, params, steps, warmup):
    """The ten-moment fluid model alone (vl_fluid_closure_step) on the GEM
    set-up with the Eq. 5 gradient closure or the network's heat flux: time
    per step, per-category breakdown and mass drift."""
    import torch
    from paper_2109_06743_amd import vl
    from paper_2109_06743_amd import workloads as W
    cfg, U, F = W.gem_fluid(nx=nx, ny=ny)
    # explicit limits: the Yee solver (c dt <= h / sqrt 2) and the parabolic
    # Eq. 5 term (RK3 with the 5-point Laplacian: D dt <= 0.3 h^2, D = chi d_s v_t)
    h = min((cfg["x_hi"] - cfg["x_lo"]) / nx, (cfg["y_hi"] - cfg["y_lo"]) / ny)
    chi = 2.0 * math.sqrt(2.0 / math.pi)
    D = max(chi * math.sqrt(sp["m"]) / abs(sp["q"])
            * math.sqrt(float(np.max((u[..., 4] + u[..., 7] + u[..., 9]) / (3.0 * u[..., 0] * sp["m"]))))
            for sp, u in zip(cfg["species"], U))
    dt = 0.5 * min(h / (cfg["c"] * math.sqrt(2.0)), 0.3 * h * h / D)
    cfg["dt"] = dt
    ctx = vl.Context(cfg, "f64")
    fs = vl.FluidState(ctx, U, vl.yee_pack(F), mlp_params=params if closure == "mlp" else None)
    mass0 = [u.view(-1, 10)[:, 0].sum().item() for u in fs.U]
    ctx.fluid_closure_step(fs, cfg["dt"], closure)
    ctx.sync()
    ctx.timing_enable(True)
    nb = max(warmup - 1, 1)
    for _ in range(nb):
        ctx.fluid_closure_step(fs, cfg["dt"], closure)
    ctx.sync()
    br = ctx.timing_read()
    ctx.timing_enable(False)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        ctx.fluid_closure_step(fs, cfg["dt"], closure)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    mass1 = [u.view(-1, 10)[:, 0].sum().item() for u in fs.U]
    finite = all(bool(torch.isfinite(u).all()) for u in fs.U)
    del fs, ctx
    torch.cuda.empty_cache()
    return dict(ms=ms, cells=nx * ny * len(U), breakdown={k: round(v[0] / nb, 4) for k, v in br.items() if v[1]},
                mass_rel_drift=max(abs(q - p) / p for p, q in zip(mass0, mass1)), steps_run=1 + nb + steps,
                dt=dt, finite=finite)


def fluid_closure_report(args, trained_params):
    """Both closures of the fluid-only model on the GEM set-up at --fluid-grid."""
    from paper_2109_06743_amd import workloads as W
    fnx, fny = args.fluid_grid
    net = trained_params if trained_params is not None else W.mlp_init(0)
    runs = []
    for closure in ("gradient", "mlp"):
        rf = run_fluid_closure(fnx, fny, closure, net, args.steps, args.warmup)
        log(f"fluid-only {fnx}x{fny} {closure} closure: {rf['ms']:.3f} ms/step {rf['breakdown']}")
        runs.append({"closure": closure, "value": rf["cells"] / (rf["ms"] * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": round(rf["ms"], 4), "kernel_ms_per_step": rf["breakdown"],
                     "mass_rel_drift": rf["mass_rel_drift"], "steps_run": rf["steps_run"], "dt": rf["dt"],
                     "state_finite": rf["finite"]})
    which = "trained above" if trained_params is not None else "untrained, Glorot init"
    return {"workload": f"GEM ten-moment two-fluid model {fnx}x{fny} x 2 species, FP64, closures: Eq. 5 "
                        f"temperature gradient / network ({which})",
            "runs": runs}


def _oracle_slab(cfg, f, F, i0, j0, snx, sny):
    """A snx x sny window of a 2X3V workload (f of every species and the Yee
    fields) as a problem of its own with the same cell sizes: the same
    per-cell work as the full grid, on the full grid's own values."""
    from oracle import fields as OF
    dx = (cfg["x_hi"] - cfg["x_lo"]) / cfg["nx"]
    dy = (cfg["y_hi"] - cfg["y_lo"]) / cfg["ny"]
    c = dict(cfg, nx=snx, ny=sny, x_lo=cfg["x_lo"] + i0 * dx, x_hi=cfg["x_lo"] + (i0 + snx) * dx,
             y_lo=cfg["y_lo"] + j0 * dy, y_hi=cfg["y_lo"] + (j0 + sny) * dy)
    fs = [np.ascontiguousarray(x[j0:j0 + sny, i0:i0 + snx], dtype=np.float64) for x in f]
    G = OF.Yee(snx, sny)
    for k in ("Ex", "Ez", "By"):
        setattr(G, k, np.ascontiguousarray(getattr(F, k)[j0:j0 + sny, i0:i0 + snx], dtype=np.float64))
    for k in ("Ey", "Bx", "Bz"):
        setattr(G, k, np.ascontiguousarray(getattr(F, k)[j0:j0 + sny + 1, i0:i0 + snx], dtype=np.float64))
    return c, fs, G


YEE = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def _oracle_steps(job):
    """Worker of the CPU baseline: the FP64 numpy oracle's full 2X3V step on
    one slab, repeated until `seconds` have passed (at least `capture` steps,
    at least one), on one thread.  Returns (phase-space cells, steps, seconds,
    state) with state = f of every species and the Yee fields (plain arrays)
    after the first `capture` steps, or None when capture is 0."""
    cfg, f, F, seconds, capture = job
    from threadpoolctl import threadpool_limits
    from oracle import moments as OM, step as OS
    with threadpool_limits(limits=1):
        moms, Us = [], []
        for k, sp in enumerate(cfg["species"]):
            v, dv = OS._grids(cfg, sp)
            mm = OM.raw_moments_3v(f[k], v, dv, sp["m"])
            moms.append(mm)
            Us.append(mm[..., :10].copy())
        st = dict(f=f, U=Us, mom_post=moms, F=F)
        t0 = time.perf_counter()
        n = 0
        state = None
        while n < max(capture, 1) or time.perf_counter() - t0 < seconds:
            st = OS.step_2x3v(st, cfg, cfg["dt"])
            n += 1
            if n == capture:
                state = dict(f=[np.array(x) for x in st["f"]], fields={k: np.array(getattr(st["F"], k)) for k in YEE})
        dt = time.perf_counter() - t0
    return sum(x.size for x in f), n, dt, state


def cpu_baseline(cfg, f, F, label, seconds=8.0, snx=16, sny=8, check_steps=2):
    """The FP64 numpy oracle's full step on windows of the benchmark
    workload's own initial state (snx x sny spatial cells with every velocity
    cell of both species: the per-cell work of the full grid).  Timed once on
    one thread, and once with one worker process per host core (at most 16,
    the host share of one GPU), each on its own window, all at the same time:
    throughput = all workers' cell-updates / the wall time of the slowest."""
    import multiprocessing as mp
    ny, nx = cfg["ny"], cfg["nx"]
    ncores = max(1, min(os.cpu_count() or 1, 16))
    # windows along the middle rows (the current sheet) at distinct x
    wins = [(((k * nx) // ncores) // snx * snx % (nx - snx + 1), (ny - sny) // 2) for k in range(ncores)]
    ctx = mp.get_context("spawn")              # workers never touch the GPU
    cw, fw, Fw = _oracle_slab(cfg, f, F, *wins[0], snx, sny)
    with ctx.Pool(1) as pool:
        c, n1, t1, ref = pool.apply(_oracle_steps, ((cw, fw, Fw, seconds, check_steps),))
    v1 = c * n1 / t1
    # the oracle's state after check_steps steps of window 0, and that window's
    # start, for the GPU's error against it (plain arrays)
    check = dict(cfg=cw, f0=fw, F0={k: np.array(getattr(Fw, k)) for k in YEE}, ref=ref, steps=check_steps,
                 window=f"{snx}x{sny} spatial cells at x index {wins[0][0]}, y index {wins[0][1]}")
    jobs = [(*_oracle_slab(cfg, f, F, i0, j0, snx, sny), seconds, 0) for i0, j0 in wins]
    t0 = time.perf_counter()
    with ctx.Pool(ncores) as pool:
        res = pool.map(_oracle_steps, jobs)
    wall = time.perf_counter() - t0
    tot = sum(c * n for c, n, _, _ in res)
    slowest = max(t for _, _, t, _ in res)
    vall = tot / slowest
    nv = cfg["species"][0]["nv"][0]
    return {"value": vall, "unit": "cell-updates/s", "cores": ncores, "kind": "oracle",
            "sample": f"{label}: the numpy FP64 oracle's full step (fit on, both species, {nv}^3 velocity cells) on "
                      f"{ncores} windows of {snx}x{sny} spatial cells of the workload's own initial state, one "
                      f"single-threaded worker process per core, {min(n for _, n, _, _ in res)}-"
                      f"{max(n for _, n, _, _ in res)} steps each in {slowest:.1f} s ({wall:.1f} s wall with start-up)",
            "one_thread": {"value": v1, "cores": 1, "steps": n1, "seconds": round(t1, 2)}}, check


def oracle_error(check):
    """The GPU step against the FP64 oracle: the same window of the workload
    (its own problem, as in the CPU baseline) stepped `steps` times by the
    library in FP32 and in FP64 storage, compared with the oracle's state
    that the CPU-baseline leg recorded: relative L2 error of f per species and
    the largest field difference relative to the largest field value."""
    import types
    import torch
    from paper_2109_06743_amd import vl
    cfg, ref, steps = check["cfg"], check["ref"], check["steps"]
    F0 = types.SimpleNamespace(**check["F0"])
    out = {"window": check["window"], "steps": steps, "reference": "FP64 numpy oracle, same initial state"}
    for dt in ("f32", "f64"):
        ctx = vl.Context(cfg, dt)
        st = vl.StepState(ctx, check["f0"], vl.yee_pack(F0))
        for _ in range(steps):
            ctx.step(st, cfg["dt"])
        ctx.sync()
        errs = []
        for s, fr in enumerate(ref["f"]):
            g = st.f[s].double().cpu().numpy().reshape(fr.shape)
            errs.append(float(np.linalg.norm(g - fr) / np.linalg.norm(fr)))
        fg = st.fields.cpu().numpy()
        fo = vl.yee_pack(types.SimpleNamespace(**ref["fields"]))
        out[dt] = {"f_rel_l2_per_species": errs,
                   "fields_max_abs_rel": float(np.abs(fg - fo).max() / np.abs(fo).max())}
        del st, ctx
    return out


def step_fractions(res):
    """Whole-step HBM fractions: bytes per phase-space cell per step under the
    passes this implementation runs (two fused X passes, V, one moments read,
    fit: 9 f-element transfers = 36 B in FP32) and the two models of separate
    (48 B) and fully fused (32 B) passes, over the step time."""
    e = res["elem"]
    rate = res["ncells"] / (res["ms"] * 1e-3)
    return {name: {"bytes_per_cell": k * e, "frac": round(k * e * rate / 1e9 / HBM_PEAK_GBS, 4)}
            for name, k in (("moved", 9), ("model_six_passes", 12), ("model_four_passes", 8))}


def kernel_fractions(res):
    """Per f-pass kernel: algorithmic bytes per launch / mean launch time in
    the warm-up breakdown (every category timed), as a fraction of peak."""
    out = {}
    for k, n_el in ALG_BYTES_PER_CELL.items():
        tot, n = res["breakdown"][k]
        if n:
            alg = n_el * res["elem"] * res["cells_per_launch"]
            out[k] = {"ms_per_launch": round(tot / n, 4), "frac": round(alg / (tot / n * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def measure(name, args, fp64=True, built=None, backsub=True):
    """FP32 (and FP64) steps of one workload: value, roofline, fractions, drifts."""
    t0 = time.perf_counter()
    cfg, f, F, label = built if built is not None else build_workload(name)
    log(f"workload {label}: built in {time.perf_counter() - t0:.1f} s")
    r32 = run_gpu(cfg, f, F, "f32", args.steps, args.warmup)
    r32["cells_per_launch"] = sum(_nelem(x) for x in f) / len(f)
    log(f"{name} fp32: {r32['ms']:.3f} ms/step  warm-up breakdown {r32['breakdown']}  timed {r32['timing']}")
    r64 = None
    if fp64 and name != "ot":
        r64 = run_gpu(cfg, [x.astype(np.float64) for x in f], F, "f64", args.steps, args.warmup)
        r64["cells_per_launch"] = r32["cells_per_launch"]
        log(f"{name} fp64: {r64['ms']:.3f} ms/step")
    half = None
    if fp64 and name == "ot":
        # FP64 f of the 512^2 box is 165 GB per copy and the step holds two:
        # both precisions on half the box, 512 x 256, for the speed-up
        import torch
        from paper_2109_06743_amd import workloads as W
        half = {}
        for dt in ("f32", "f64"):
            cfg_h, f_h, F_h = W.orszag_tang_device(n=512, ny=256, nv=34, dtype=dt)
            half[dt] = run_gpu(cfg_h, f_h, F_h, dt, args.steps, args.warmup)
            half[dt]["cells_per_launch"] = sum(_nelem(x) for x in f_h) / len(f_h)
            log(f"{name} 512x256 {dt}: {half[dt]['ms']:.3f} ms/step")
            del f_h
            torch.cuda.empty_cache()
    value = r32["ncells"] / (r32["ms"] * 1e-3)
    out = {"workload": label, "value": value, "ms_per_step": round(r32["ms"], 4),
           "cells": r32["ncells"], "species": len(f), "dt": cfg["dt"],
           "roofline": roofline(r32, label), "step_hbm_frac": step_fractions(r32),
           "kernel_hbm_frac": kernel_fractions(r32),
           "kernel_ms_per_step": {k: round(v[0] / r32["breakdown_steps"], 4) for k, v in r32["breakdown"].items()
                                  if v[1]},
           "energy_rel_drift": {"f32": r32["energy_rel_drift"], "steps": r32["steps_run"]},
           "mass_rel_drift": {"f32": r32["mass_rel_drift"]}}
    if r64 is not None:
        v64 = r64["ncells"] / (r64["ms"] * 1e-3)
        out["fp64"] = {"value": v64, "ms_per_step": round(r64["ms"], 4), "speedup_fp32_over_fp64": round(value / v64, 3),
                       "step_hbm_frac": step_fractions(r64)}
    if half is not None:
        v32h = half["f32"]["ncells"] / (half["f32"]["ms"] * 1e-3)
        v64h = half["f64"]["ncells"] / (half["f64"]["ms"] * 1e-3)
        out["fp64"] = {"grid": "512x256 x 34^3 x 2 species (half the box: the FP64 step on 512^2 needs 330 GB)",
                       "value": v64h, "ms_per_step": round(half["f64"]["ms"], 4),
                       "fp32_same_grid": {"value": v32h, "ms_per_step": round(half["f32"]["ms"], 4),
                                          "kernel_hbm_frac": kernel_fractions(half["f32"])},
                       "speedup_fp32_over_fp64": round(v32h / v64h, 3), "step_hbm_frac": step_fractions(half["f64"]),
                       "kernel_hbm_frac": kernel_fractions(half["f64"]),
                       "kernel_ms_per_step": {k: round(v[0] / half["f64"]["breakdown_steps"], 4)
                                              for k, v in half["f64"]["breakdown"].items() if v[1]},
                       "energy_rel_drift": {"f32": half["f32"]["energy_rel_drift"], "f64": half["f64"]["energy_rel_drift"],
                                            "steps": half["f64"]["steps_run"]},
                       "mass_rel_drift": {"f32": half["f32"]["mass_rel_drift"], "f64": half["f64"]["mass_rel_drift"]}}
    if backsub:             # 34^3 blocks: FP32 (the affine sweeps hold the block in LDS)
        rb = run_gpu(dict(cfg, vsplit="backsub"), f, F, "f32", args.steps, args.warmup)
        log(f"{name} fp32 backsubstitution split: {rb['ms']:.3f} ms/step")
        vb, va = rb["breakdown"]["pfc_v"], r32["breakdown"]["pfc_v"]
        out["backsub_split"] = {
            "value": rb["ncells"] / (rb["ms"] * 1e-3), "ms_per_step": round(rb["ms"], 4),
            "pfc_v_ms_per_launch": round(vb[0] / vb[1], 4), "strang_pfc_v_ms_per_launch": round(va[0] / va[1], 4),
            "energy_rel_drift": rb["energy_rel_drift"], "mass_rel_drift": rb["mass_rel_drift"]}
    if r64 is not None:
        out["energy_rel_drift"]["f64"] = r64["energy_rel_drift"]
        out["energy_rel_drift"]["f64_steps"] = r64["steps_run"]
        out["mass_rel_drift"]["f64"] = r64["mass_rel_drift"]
    return out, (cfg, f, F, label)


def v_operator_report(steps=5):
    """The V operator alone with the two velocity splittings (Strang shear
    sweeps and backsubstitution) on random f and random cell fields, on the
    GEM 16^3 and magnetotail 12^3 grids: average time per launch (one
    species' block) from the library's HIP-event timing."""
    import torch
    from paper_2109_06743_amd import vl, workloads as W
    out = {}
    for name, builder, (nx, ny, nv), dt in (("gem", W.gem, (256, 128, 16), 0.003),
                                           ("tail", W.tail, (1024, 512, 12), 0.0012)):
        cfg, _, _ = builder(nx=8, ny=4, nv=nv, dt=dt, dtype=np.float32)
        cfg = dict(cfg, nx=nx, ny=ny)
        cells = nx * ny
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        fin = torch.rand((ny, nx, nv, nv, nv), dtype=torch.float32, device="cuda", generator=g)
        fout = torch.empty_like(fin)
        E = (torch.rand(cells * 3, dtype=torch.float64, device="cuda", generator=g) - 0.5) * 0.2
        B = (torch.rand(cells * 3, dtype=torch.float64, device="cuda", generator=g) - 0.5) * 2.0
        for split in ("strang", "backsub"):
            ctx = vl.Context(dict(cfg, vsplit=split), "f32")
            for s in range(2):
                ctx.pfc_advect_v(s, fin, fout, E, B, dt)
            ctx.sync()
            ctx.timing_enable(["pfc_v"])
            for _ in range(steps):
                for s in range(2):
                    ctx.pfc_advect_v(s, fin, fout, E, B, dt)
            ctx.sync()
            ms, n = ctx.timing_read()["pfc_v"]
            out[f"{name}_{split}"] = {"grid": f"{nx}x{ny} x {nv}^3", "ms_per_launch": round(ms / n, 4),
                                     "launches": n}
            log(f"V operator {name} {split}: {ms / n:.4f} ms per launch")
            del ctx
        del fin, fout
        torch.cuda.empty_cache()
    return out


def graph_replay_report(nx=32, ny=16, nv=8, steps=200):
    """A small GEM grid, where a step is bound by its ~60 kernel launches
    rather than by HBM: eager vl_step calls against replays of one captured
    step (a HIP graph through torch's graph API), two contexts from the same
    state, both trajectories compared bit for bit at the end."""
    import torch
    from paper_2109_06743_amd import vl
    from paper_2109_06743_amd import workloads as W
    cfg, f, F = W.gem(nx=nx, ny=ny, nv=nv, dt=0.003, fit=True, dtype=np.float32)
    pair = []
    for _ in range(2):
        ctx = vl.Context(cfg, "f32")
        st = vl.StepState(ctx, f, vl.yee_pack(F))
        ctx.step(st, cfg["dt"])                     # allocates the context's scratch
        pair.append((ctx, st))
    (ca, sa), (cb, sb) = pair
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        cb.step(sb, cfg["dt"])                      # recorded, not run
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    for _ in range(steps):
        ca.step(sa, cfg["dt"])
    ev[1].record(stream)
    ev[2].record(stream)
    for _ in range(steps):
        g.replay()
    ev[3].record(stream)
    torch.cuda.synchronize()
    eager, graph = ev[0].elapsed_time(ev[1]) / steps, ev[2].elapsed_time(ev[3]) / steps
    same = all(torch.equal(x, y) for x, y in zip(sa.f + sa.U + [sa.fields], sb.f + sb.U + [sb.fields]))
    del g, pair, ca, sa, cb, sb
    torch.cuda.empty_cache()
    return {"workload": f"GEM 2X3V {nx}x{ny} x {nv}^3 x 2 species, moment fitting", "steps": steps,
            "eager_ms_per_step": round(eager, 4), "graph_ms_per_step": round(graph, 4),
            "speedup": round(eager / graph, 3), "bitwise_equal": bool(same)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tail", choices=["gem", "gem34", "ot", "tail"],
                    help="headline workload (default: magnetotail 1024x512x12^3)")
    ap.add_argument("--secondary", default="gem", choices=["gem", "gem34", "ot", "tail", "none"],
                    help="workload reported beside the headline")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-backsub", action="store_true", help="skip the step with the backsubstitution velocity split")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-closure form")
    ap.add_argument("--closure-tol", type=float, nargs="+", default=[0.25, 0.5, 1.0],
                    help="judge tolerances of the learned-closure runs (one run each)")
    ap.add_argument("--no-fluid-closure", action="store_true", help="skip the fluid-only closure runs")
    ap.add_argument("--graph", action="store_true",
                    help="add the eager-against-graph-replay comparison (not under rocprofv3 --pmc: graph "
                         "replays there do not return)")
    ap.add_argument("--fluid-grid", type=int, nargs=2, default=[2048, 1024], metavar=("NX", "NY"))
    ap.add_argument("--only-fluid-closure", action="store_true",
                    help="only the fluid-only closure runs (one JSON object), e.g. for profiling")
    ap.add_argument("--only-v-operator", action="store_true",
                    help="only the V operator with both velocity splittings (one JSON object), e.g. for profiling")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this implementation runs on one GPU: the data-parallel path is measured on a single MI355X "
              "and has no multi-GPU code; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        torch.cuda.set_device(0)
        calibrate_copy()
        return
    from paper_2109_06743_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    if args.only_fluid_closure:
        torch.cuda.set_device(0)
        print(json.dumps({"fluid_closure": fluid_closure_report(args, None)}), flush=True)
        return
    if args.only_v_operator:
        torch.cuda.set_device(0)
        print(json.dumps({"v_operator": v_operator_report()}), flush=True)
        return
    t0 = time.perf_counter()
    built = build_workload(args.workload)
    cfg, f, F, label = built
    log(f"workload {label}: built in {time.perf_counter() - t0:.1f} s")
    cpu = check = None
    if not args.no_cpu and cfg["kind"] == "2x3v" and args.workload != "ot":
        # before any GPU call: the worker processes are started from a process
        # that has not initialised the GPU
        log("timing the CPU oracle on windows of the workload ...")
        cpu, check = cpu_baseline(cfg, f, F, label)
        log(f"  {cpu}")
    torch.cuda.set_device(0)
    head, _ = measure(args.workload, args, fp64=not args.no_fp64, built=built, backsub=not args.no_backsub)
    del built, f, F
    out = {
        "metric": METRIC, "value": head["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": label, "cells": head["cells"], "species": head["species"], "dt": head["dt"],
                   "moments_fields_fluid": "f64"},
        "roofline": head["roofline"],
    }
    for k in ("step_hbm_frac", "kernel_hbm_frac", "fp64", "backsub_split", "energy_rel_drift", "mass_rel_drift",
              "kernel_ms_per_step"):
        if k in head:
            out[k] = head[k]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if check is not None:
        out["oracle_error"] = oracle_error(check)
        log(f"error against the oracle: {out['oracle_error']}")
    if args.secondary != "none" and args.secondary != args.workload:
        sec, _ = measure(args.secondary, args, fp64=not args.no_fp64, backsub=not args.no_backsub)
        out["secondary"] = sec
    if args.graph:
        out["graph_replay"] = graph_replay_report()
        log(f"graph replay: {out['graph_replay']}")
    mlp_geom = "gem"
    params = None
    if not args.no_mlp:
        cfg_m0, f_m, F_m, label_m = build_workload(mlp_geom)
        log("learned closure: generating data and training ...")
        params, tr, end = train_closure(cfg_m0, f_m, F_m)
        log(f"  {tr}")
        runs = []
        for tol in args.closure_tol:
            cfg_m = dict(cfg_m0, closure="mlp", closure_tol=tol)
            rm = run_closure(cfg_m, dict(end, f=[x.clone() for x in end["f"]], fields=end["fields"].clone(),
                                         U=[u.clone() for u in end["U"]], mom_post=[m.clone() for m in end["mom_post"]]),
                             params, args.steps, args.warmup)
            log(f"mlp closure tol {tol}: {rm['ms']:.3f} ms/step, err {rm['closure_err']}, "
                f"fallback steps {rm['fallback_steps']}")
            runs.append({"closure_tol": tol, "value": rm["ncells"] / (rm["ms"] * 1e-3), "unit": "cell-updates/s",
                         "ms_per_step": round(rm["ms"], 4), "closure_err_last_step": rm["closure_err"],
                         "fallback_steps_per_species": rm["fallback_steps"], "timed_steps": args.steps,
                         "energy_rel_drift": rm["energy_rel_drift"], "mass_rel_drift": rm["mass_rel_drift"]})
        out["mlp_closure"] = {
            "workload": label_m + " + learned heat-flux closure (64-64-64-64-16 tanh MLP, BF16 MFMA)",
            "start_time": end["t"], "runs": runs, "training": tr}
        del end
    if not args.no_fluid_closure:
        out["fluid_closure"] = fluid_closure_report(args, params)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
