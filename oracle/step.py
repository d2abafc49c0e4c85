"""Full time steps of the moment-fitting Vlasov solver, FP64 CPU oracle.
Test infrastructure only.

Algorithm 1 of the paper (time stepping of the moment-fitting Vlasov-Maxwell
solver), with these readings where it is silent:
* "Full Vlasov Leapfrog Step": Strang order X(dt/2) V(dt) X(dt/2), the
  fields for V taken at t+1/2.  V is the Strang shear sequence
  (oracle.vlasov.v_advect_3v), or with cfg["vsplit"] == "backsub" the
  backsubstitution split (oracle.vlasov.v_advect_3v_backsub).
* Electromagnetic (2X3V): the first Maxwell half step uses j^t (current of the
  fitted f^t), the second j^{t+1} (current of the fitted f^{t+1}); V uses the
  cell-centred E, B after the first half step.  The fluid's stage fields are
  (E, B)^t, 2 (E, B)^{t+1/2} - (E, B)^t and (E, B)^{t+1/2}.
* Electrostatic (1X1V, Sec. 3.1): E for V comes from Poisson of the electron
  density after X(dt/2); the fluid's stage fields are E(n^t), E(n^{t+1}) and
  their mean.
* Q-calligraphic at t is that of the fitted f^t, at t+1 that of f^{t+1}
  before fitting, at t+1/2 their mean (Algorithm 1, "interpolate").
* With fitting switched off the step is the standard PFC Vlasov step (the
  fluid is not advanced).
* Learned closure (cfg["closure"] == "mlp", 2X3V; not in the paper): the
  network (oracle.mlp) is judged on the moments of f^{t+1} before fitting
  with the field direction of (E, B)^{t+1} (the extrapolated stage field);
  if its heat-flux error exceeds cfg["closure_tol"] (or when st["fallback"]
  says so for that species) the step is the kinetic one, otherwise the fluid
  RK3 takes each stage's Q-calligraphic from the network applied to that
  stage's state.
"""
import numpy as np

from . import fields, fluid, mlp, moments, vlasov


# ---------------------------------------------------------------- 1X1V ----
def step_1x1v(st, cfg, dt):
    """st: dict(f[nx,nv], mom_post[nx,4], U[nx,3] or None).  Returns new dict."""
    q, m = cfg["q"], cfg["m"]
    v, dv = vlasov.centres(cfg["v_lo"], cfg["v_hi"], cfg["nv"])
    dx = (cfg["x_hi"] - cfg["x_lo"]) / cfg["nx"]
    f = vlasov.x_advect_1x1v(st["f"], v, dx, 0.5 * dt)
    E_half = fields.efield_1x1v(moments.raw_moments_1v(f, v, dv, m)[:, 0], dx, q)
    f = vlasov.v_advect_1x1v(f, E_half, q, m, dv, dt)
    f = vlasov.x_advect_1x1v(f, v, dx, 0.5 * dt)
    mom_pre = moments.raw_moments_1v(f, v, dv, m)
    out = {"f": f, "mom_pre": mom_pre, "E_half": E_half, "U": st.get("U"),
           "clipped": 0, "skipped": 0}
    if cfg.get("fit"):
        E_t = fields.efield_1x1v(st["mom_post"][:, 0], dx, q)
        E_t1 = fields.efield_1x1v(mom_pre[:, 0], dx, q)
        U = fluid.rk3_1v(st["U"], st["mom_post"][:, 3], mom_pre[:, 3], E_t, E_t1, q, m, dx, dt)
        f, U, c, s = moments.moment_fit_1v(f, mom_pre, U, m, v, dv)
        out.update(f=f, U=U, clipped=c, skipped=s)
        out["mom_post"] = moments.raw_moments_1v(f, v, dv, m)
    else:
        out["mom_post"] = mom_pre
    return out


def energy_1x1v(f, cfg):
    """Kinetic energy sum(m v^2 f / 2) plus field energy sum(E^2 / 2) (eps0 = 1)."""
    v, dv = vlasov.centres(cfg["v_lo"], cfg["v_hi"], cfg["nv"])
    dx = (cfg["x_hi"] - cfg["x_lo"]) / cfg["nx"]
    mom = moments.raw_moments_1v(f, v, dv, cfg["m"])
    E = fields.efield_1x1v(mom[:, 0], dx, cfg["q"])
    kin = 0.5 * mom[:, 2].sum() * dx
    fld = 0.5 * (E * E).sum() * dx
    return kin, fld


# ---------------------------------------------------------------- 2X3V ----
def _grids(cfg, sp):
    v, dv = [], []
    for d in range(3):
        c, h = vlasov.centres(sp["v_lo"][d], sp["v_hi"][d], sp["nv"][d])
        v.append(c)
        dv.append(h)
    return v, dv


def step_2x3v(st, cfg, dt):
    """st: dict(f=[f_s], U=[U_s], mom_post=[m_s], F=Yee).  Returns new dict."""
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    c = cfg["c"]
    species = cfg["species"]
    bc = cfg.get("bc_y", "reflect")
    F_t = st["F"]
    j_t = sum(sp["q"] * st["mom_post"][k][..., 1:4] for k, sp in enumerate(species))
    F = fields.maxwell_half_step(F_t, j_t, dt, c, dx, dy, bc)
    E_h, B_h = fields.cell_centred(F)
    E_0, B_0 = fields.cell_centred(F_t)
    fields_t1 = (2.0 * E_h - E_0, 2.0 * B_h - B_0)
    out = {"f": [], "U": [], "mom_pre": [], "mom_post": [], "clipped": 0, "skipped": 0,
           "closure_err": [], "fallback": []}
    for k, sp in enumerate(species):
        q, m = sp["q"], sp["m"]
        v, dv = _grids(cfg, sp)
        f = vlasov.x_advect_2x3v(st["f"][k], v[0], v[1], dx, dy, 0.5 * dt, bc_y=bc)
        if cfg.get("vsplit") == "backsub":
            f = vlasov.v_advect_3v_backsub(f, E_h, B_h, q, m, v, dv, dt)
        else:
            f = vlasov.v_advect_3v(f, E_h, B_h, q, m, v, dv, dt)
        f = vlasov.x_advect_2x3v(f, v[0], v[1], dx, dy, 0.5 * dt, bc_y=bc)
        mom_pre = moments.raw_moments_3v(f, v, dv, m)
        U = st["U"][k]
        if cfg.get("fit"):
            use_net = False
            if cfg.get("closure") == "mlp":
                if bc != "reflect":
                    raise ValueError("the network closure is defined for reflecting y walls")
                err = mlp.judge_error(mom_pre, m, k, st["mlp_params"], fields_t1[1])
                fb = st["fallback"][k] if st.get("fallback") is not None else not (err <= cfg["closure_tol"])
                out["closure_err"].append(err)
                out["fallback"].append(bool(fb))
                use_net = not fb
            if use_net:
                U = fluid.rk3_3v_stagewise(U, lambda V, Bs, k=k, m=m: mlp.closure_qcal(V, m, k, st["mlp_params"], Bs),
                                           (E_0, B_0), fields_t1, (E_h, B_h), q, m, dx, dy, dt)
            else:
                U = fluid.rk3_3v(U, st["mom_post"][k][..., 10:], mom_pre[..., 10:],
                                 (E_0, B_0), fields_t1, (E_h, B_h), q, m, dx, dy, dt, bc)
            f, U, cl, sk = moments.moment_fit_3v(f, mom_pre, U, m, v, dv)
            out["clipped"] += cl
            out["skipped"] += sk
            mom_post = moments.raw_moments_3v(f, v, dv, m)
        else:
            mom_post = mom_pre
        out["f"].append(f)
        out["U"].append(U)
        out["mom_pre"].append(mom_pre)
        out["mom_post"].append(mom_post)
    j_t1 = sum(sp["q"] * out["mom_post"][k][..., 1:4] for k, sp in enumerate(species))
    out["F"] = fields.maxwell_half_step(F, j_t1, dt, c, dx, dy, bc)
    out["E_half"], out["B_half"] = E_h, B_h
    return out


def fluid_step_2x3v(st, cfg, dt, closure, params=None):
    """The ten-moment multi-fluid model on its own (Sec. 2.3): st =
    dict(U=[U_s], F=Yee).  The field half steps and stage fields are those of
    step_2x3v with the currents q n u of the fluid states; every RK stage
    takes its third moment from a closure of the stage state:
    'gradient': zero heat flux in Q-calligraphic and Eq. 5 as the source
    -div Q of the second-moment equation; 'mlp': the network's heat flux
    (params) from the stage state and magnetic field."""
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    c = cfg["c"]
    species = cfg["species"]
    bc = cfg.get("bc_y", "reflect")
    F_t = st["F"]
    j_t = sum(sp["q"] * st["U"][k][..., 1:4] for k, sp in enumerate(species))
    F = fields.maxwell_half_step(F_t, j_t, dt, c, dx, dy, bc)
    E_h, B_h = fields.cell_centred(F)
    E_0, B_0 = fields.cell_centred(F_t)
    fields_t1 = (2.0 * E_h - E_0, 2.0 * B_h - B_0)
    out = {"U": []}
    for k, sp in enumerate(species):
        q, m = sp["q"], sp["m"]
        if closure == "gradient":
            def qcal_of(V, Bs, m=m):
                return mlp.qcal_from_closure(V, np.zeros(V.shape[:-1] + (10,)), 0.0, m)

            def source_of(V, m=m, q=q):
                S = np.zeros(V.shape)
                S[..., 4:10] = -mlp.gradient_closure_divergence(V, m, q, dx, dy, bc)
                return S
        elif closure == "mlp":
            if bc != "reflect":
                raise ValueError("the network closure is defined for reflecting y walls")

            def qcal_of(V, Bs, m=m, k=k):
                return mlp.closure_qcal(V, m, k, params, Bs)
            source_of = None
        else:
            raise ValueError(closure)
        out["U"].append(fluid.rk3_3v_closure(st["U"][k], qcal_of, source_of, (E_0, B_0), fields_t1, (E_h, B_h),
                                             q, m, dx, dy, dt, bc))
    j_t1 = sum(sp["q"] * out["U"][k][..., 1:4] for k, sp in enumerate(species))
    out["F"] = fields.maxwell_half_step(F, j_t1, dt, c, dx, dy, bc)
    return out


def energy_2x3v(st, cfg):
    """Total energy: sum_s tr(P_s)/2 over cells (kinetic + thermal, Sec. 3.2's
    energy split summed) plus the Yee field energy."""
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    kin = 0.0
    for k, sp in enumerate(cfg["species"]):
        v, dv = _grids(cfg, sp)
        mom = moments.raw_moments_3v(st["f"][k], v, dv, sp["m"])
        kin += 0.5 * (mom[..., 4] + mom[..., 7] + mom[..., 9]).sum() * dx * dy
    return kin, fields.field_energy(st["F"], cfg["c"], dx, dy)
