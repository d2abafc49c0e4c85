"""Seeded synthetic workloads (initial conditions and run parameters).

This module holds only the problem set-ups: analytic initial distributions
sampled at cell centres, initial fields, grid extents, time steps.  It
contains none of the solver's arithmetic (no sweeps, quadratures, fitting or
field updates), so both the HIP path and the CPU reference can start from
the same arrays.

Set-ups (paper sections cited by name):
* landau    - linear Landau damping (Sec. 3.1): f0 = (1 + a cos kx) e^{-v^2/2}/sqrt(2 pi)
* twostream - two drifting Maxwellians at +-2.4, v_t 0.5, k 0.2 (a beam
              variant of the two-stream set-up of Sec. 3.1)
* gem       - Harris sheet with the GEM perturbation (Sec. 3.3)
* tail      - Harris sheet plus background populations, guide field,
              seeded random B_x noise (magnetotail set-up, Sec. 4.1)
Units: electrostatic runs in omega_p^-1, lambda_D, v_t, m_e (Sec. 3.1);
electromagnetic runs in Omega_i^-1, d_i, v_A, m_i, q_i, mu0 = k_B = 1 (Sec. 2.1).
"""
import math

import numpy as np


def _centres(lo, hi, n):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


# ------------------------------------------------------------ 1X1V ------
def landau(nx=64, nv=64, vmax=6.0, alpha=0.01, k=0.5, dt=0.1, steps=100, fit=False):
    L = 2 * math.pi / k
    cfg = dict(kind="1x1v", nx=nx, x_lo=-L / 2, x_hi=L / 2, nv=nv, v_lo=-vmax, v_hi=vmax,
               q=-1.0, m=1.0, fit=fit, dt=dt, steps=steps, name=f"landau {nx}x{nv}")
    x = _centres(cfg["x_lo"], cfg["x_hi"], nx)
    v = _centres(-vmax, vmax, nv)
    f = (1.0 + alpha * np.cos(k * x))[:, None] * (np.exp(-0.5 * v * v) / math.sqrt(2 * math.pi))[None, :]
    return cfg, f


def twostream(nx=256, nv=256, vmax=8.0, alpha=1e-3, k=0.2, vd=2.4, vt=0.5, dt=0.1, steps=500, fit=False):
    L = 2 * math.pi / k
    cfg = dict(kind="1x1v", nx=nx, x_lo=0.0, x_hi=L, nv=nv, v_lo=-vmax, v_hi=vmax,
               q=-1.0, m=1.0, fit=fit, dt=dt, steps=steps, name=f"twostream {nx}x{nv}")
    x = _centres(0.0, L, nx)
    v = _centres(-vmax, vmax, nv)
    g = lambda w: np.exp(-0.5 * (w / vt) ** 2) / (math.sqrt(2 * math.pi) * vt)
    f = (1.0 + alpha * np.cos(k * x))[:, None] * (0.5 * (g(v - vd) + g(v + vd)))[None, :]
    return cfg, f


# ------------------------------------------------------------ 2X3V ------
def _maxwellian_block(n, uz, T, m, v):
    """Analytic isotropic Maxwellian n (m/2piT)^{3/2} exp(-m |v-u|^2/(2T)), u = (0,0,uz),
    for arrays n, uz of shape [...]; returns [..., nvx, nvy, nvz]."""
    vx, vy, vz = v
    pre = n * (m / (2 * math.pi * T)) ** 1.5
    ex = np.exp(-0.5 * m * vx * vx / T)[:, None, None] * np.exp(-0.5 * m * vy * vy / T)[None, :, None]
    ez = np.exp(-0.5 * m * (vz[None, :] - np.asarray(uz)[..., None]) ** 2 / T)
    return pre[..., None, None, None] * ex * ez[..., None, None, :]


def _vgrid_name(nv):
    return f"{nv}^3" if np.isscalar(nv) else "x".join(str(k) for k in nv)


def _species(q, m, vmax, nv):
    """nv: cells per velocity axis, one number (a cube) or three."""
    return dict(q=q, m=m, v_lo=[-vmax] * 3, v_hi=[vmax] * 3, nv=[nv] * 3 if np.isscalar(nv) else list(nv))


class Yee0:
    """Initial Yee-grid fields (same placement as the solver's)."""

    def __init__(self, nx, ny):
        self.Ex = np.zeros((ny, nx)); self.Ey = np.zeros((ny + 1, nx)); self.Ez = np.zeros((ny, nx))
        self.Bx = np.zeros((ny + 1, nx)); self.By = np.zeros((ny, nx)); self.Bz = np.zeros((ny + 1, nx))


def _gem_setup(nx, ny, nv, mass_ratio, c, lam, nb, Ti_Te, psi0, ve_max, vi_max, dt, steps, fit):
    """GEM configuration, density, per-species (u_z, T) profiles and Yee fields."""
    Lx, Ly = 8 * math.pi, 4 * math.pi
    Te = 0.5 / (1.0 + Ti_Te)
    Ti = Ti_Te * Te
    me = 1.0 / mass_ratio
    sp = [_species(-1.0, me, ve_max, nv), _species(1.0, 1.0, vi_max, nv)]
    cfg = dict(kind="2x3v", nx=nx, ny=ny, x_lo=-Lx / 2, x_hi=Lx / 2, y_lo=-Ly / 2, y_hi=Ly / 2,
               c=c, species=sp, fit=fit, dt=dt, steps=steps,
               name=f"gem {nx}x{ny}x{_vgrid_name(nv)} mi/me={mass_ratio:g}")
    x = _centres(-Lx / 2, Lx / 2, nx)
    y = _centres(-Ly / 2, Ly / 2, ny)
    X, Y = np.meshgrid(x, y)          # [ny, nx]
    n = 1.0 / np.cosh(Y / lam) ** 2 + nb
    jz = (psi0 * ((2 * math.pi / Lx) ** 2 + (math.pi / Ly) ** 2)
          * np.cos(2 * math.pi * X / Lx) * np.cos(math.pi * Y / Ly)
          - (1.0 / lam) / np.cosh(Y / lam) ** 2)
    uzi = jz * Ti / (n * (Ti + Te))
    uze = -uzi * Te / Ti
    F = Yee0(nx, ny)
    dx, dy = Lx / nx, Ly / ny
    xc = -Lx / 2 + (np.arange(nx) + 0.5) * dx      # integer i
    xf = -Lx / 2 + (np.arange(nx) + 1.0) * dx      # i + 1/2
    yc = -Ly / 2 + (np.arange(ny) + 0.5) * dy      # integer j
    yf = -Ly / 2 + np.arange(ny + 1) * dy          # j - 1/2 (walls included)
    XF, YF = np.meshgrid(xc, yf)
    F.Bx = np.tanh(YF / lam) - psi0 * (math.pi / Ly) * np.cos(2 * math.pi * XF / Lx) * np.sin(math.pi * YF / Ly)
    XB, YB = np.meshgrid(xf, yc)
    F.By = psi0 * (2 * math.pi / Lx) * np.sin(2 * math.pi * XB / Lx) * np.cos(math.pi * YB / Ly)
    return cfg, n, ((uze, Te), (uzi, Ti)), F


def gem(nx=256, ny=128, nv=16, mass_ratio=25.0, c=20.0, lam=0.5, nb=0.2, Ti_Te=5.0, psi0=0.1,
        ve_max=12.5, vi_max=5.0, dt=0.003, steps=200, fit=True, dtype=np.float32):
    """GEM reconnection set-up (Sec. 3.3) on an nx x ny x nv^3 grid (nv one
    number, or three for a non-cubic velocity grid)."""
    cfg, n, prof, F = _gem_setup(nx, ny, nv, mass_ratio, c, lam, nb, Ti_Te, psi0, ve_max, vi_max, dt, steps, fit)
    f = []
    for s, (uz, T) in zip(cfg["species"], prof):
        v = [_centres(s["v_lo"][d], s["v_hi"][d], s["nv"][d]) for d in range(3)]
        f.append(_maxwellian_block(n, uz, T, s["m"], v).astype(dtype))
    return cfg, f, F


def gem_fluid(nx=256, ny=128, mass_ratio=25.0, c=20.0, lam=0.5, nb=0.2, Ti_Te=5.0, psi0=0.1, dt=0.003,
              steps=200):
    """The GEM set-up for the ten-moment fluid model alone: per species the
    fluid record U[ny, nx, 10] = (n, n u, P) of the drifting Maxwellian,
    P = n T I + m n u u (u along z), and the same Yee fields."""
    cfg, n, prof, F = _gem_setup(nx, ny, 4, mass_ratio, c, lam, nb, Ti_Te, psi0, 12.5, 5.0, dt, steps, False)
    cfg["name"] = f"gem fluid {nx}x{ny} mi/me={mass_ratio:g}"
    U = []
    for s, (uz, T) in zip(cfg["species"], prof):
        V = np.zeros((ny, nx, 10))
        V[..., 0] = n
        V[..., 3] = n * uz
        V[..., 4] = V[..., 7] = n * T
        V[..., 9] = n * T + s["m"] * n * uz * uz
        U.append(V)
    return cfg, U, F


def _maxwellian_drift(n, u, T, m, v):
    """Analytic isotropic Maxwellian n (m/2piT)^{3/2} exp(-m |v-u|^2/(2T)) with a
    drift u[..., 3]; n, T of shape [...]; returns [..., nvx, nvy, nvz]."""
    vx, vy, vz = v
    T = np.asarray(T, dtype=np.float64) * np.ones_like(n)
    pre = n * (m / (2 * math.pi * T)) ** 1.5
    g = [np.exp(-0.5 * m * (vd[None, :] - u[..., k].reshape(-1, 1)) ** 2 / T.reshape(-1, 1))
         for k, vd in enumerate((vx, vy, vz))]
    out = pre.reshape(-1, 1, 1, 1) * g[0][:, :, None, None] * g[1][:, None, :, None] * g[2][:, None, None, :]
    return out.reshape(n.shape + (len(vx), len(vy), len(vz)))


def _ot_setup(nx, ny, nv, mass_ratio, c, beta_i, du, dB, ve_max, vi_max, dt, steps, fit):
    """Orszag-Tang configuration, per-species (n, u[3], T) at cell centres and Yee fields."""
    me = 1.0 / mass_ratio
    L = 0.5 * math.sqrt(me) * nx                   # two cells per electron inertial length (d_i = 1)
    Ly = L * ny / nx
    T = 0.5 * beta_i                               # beta_i = 2 n0 T_i / B0^2 with n0 = B0 = mu0 = 1; T_e = T_i
    sp = [_species(-1.0, me, ve_max, nv), _species(1.0, 1.0, vi_max, nv)]
    cfg = dict(kind="2x3v", nx=nx, ny=ny, x_lo=0.0, x_hi=L, y_lo=0.0, y_hi=Ly, c=c, species=sp, fit=fit, dt=dt,
               steps=steps, bc_y="periodic", name=f"orszag-tang {nx}x{ny}x{nv}^3 mi/me={mass_ratio:g}")
    dx, dy = L / nx, Ly / ny
    xc = (np.arange(nx) + 0.5) * dx                # integer i
    xf = (np.arange(nx) + 1.0) * dx                # i + 1/2
    yc = (np.arange(ny) + 0.5) * dy                # integer j
    yf = np.arange(ny + 1) * dy                    # j - 1/2 (rows 0 and ny are the same points)
    k1 = 2 * math.pi / L
    F = Yee0(nx, ny)
    XC, YF = np.meshgrid(xc, yf)
    F.Bx = -dB * np.sin(k1 * YF)
    XF, YC = np.meshgrid(xf, yc)
    F.By = dB * np.sin(2 * k1 * XF)
    F.Bz = np.ones((ny + 1, nx))
    F.Ex = -du * np.sin(k1 * XF)                   # E = -u x B with B_z = B0
    F.Ey = -du * np.sin(k1 * YF)
    # electron density from Gauss's law on the grid: div E = (n_i - n_e) / eps0, eps0 = 1/c^2
    divE = (F.Ex - np.roll(F.Ex, 1, axis=1)) / dx + (F.Ey[1:] - F.Ey[:-1]) / dy
    X, Y = np.meshgrid(xc, yc)
    u = np.zeros((ny, nx, 3))
    u[..., 0] = -du * np.sin(k1 * Y)
    u[..., 1] = du * np.sin(k1 * X)
    ue = u.copy()
    ue[..., 2] = -k1 * dB * (2 * np.cos(2 * k1 * X) + np.cos(k1 * Y))   # the electrons carry j_z
    ne = 1.0 - divE / (c * c)
    ni = np.ones((ny, nx))
    return cfg, ((ne, ue, T), (ni, u, T)), F


def orszag_tang(n=512, nv=34, mass_ratio=100.0, c=18.174, beta_i=0.1, du=0.2, dB=0.2, ve_max=14.0, vi_max=1.5,
                dt=0.0015, steps=20, fit=True, dtype=np.float32, ny=None):
    """Orszag-Tang turbulence (Sec. 3.2): periodic box, B = (-dB sin 2pi y/L,
    dB sin 4pi x/L, B0), u = (-du sin 2pi y/L, du sin 2pi x/L, u_z) with the
    electrons carrying j_z, E = -u x B, T_i = T_e, beta_i = 0.1, m_i/m_e = 100,
    c = 18.174 v_A, electrons on +-14 v_A, ions on +-1.5 v_A; n x ny cells
    (ny = n: the square box)."""
    ny = n if ny is None else ny
    cfg, prof, F = _ot_setup(n, ny, nv, mass_ratio, c, beta_i, du, dB, ve_max, vi_max, dt, steps, fit)
    f = []
    for s, (ns, us, Ts) in zip(cfg["species"], prof):
        v = [_centres(s["v_lo"][d], s["v_hi"][d], s["nv"][d]) for d in range(3)]
        f.append(_maxwellian_drift(ns, us, Ts, s["m"], v).astype(dtype))
    return cfg, f, F


def orszag_tang_device(n=512, nv=34, dtype="f32", rows_per_chunk=16, **kw):
    """The same set-up with f generated on the current GPU (torch tensors), a
    few rows at a time: the full 512^2 x 34^3 grid is 41 GB per species."""
    import torch
    ny = kw.pop("ny", n)
    cfg, prof, F = _ot_setup(n, ny, nv, kw.get("mass_ratio", 100.0), kw.get("c", 18.174), kw.get("beta_i", 0.1),
                             kw.get("du", 0.2), kw.get("dB", 0.2), kw.get("ve_max", 14.0), kw.get("vi_max", 1.5),
                             kw.get("dt", 0.0015), kw.get("steps", 20), kw.get("fit", True))
    tdt = torch.float32 if dtype == "f32" else torch.float64
    f = []
    for s, (ns, us, Ts) in zip(cfg["species"], prof):
        v = [torch.as_tensor(_centres(s["v_lo"][d], s["v_hi"][d], s["nv"][d]), device="cuda") for d in range(3)]
        out = torch.empty((ny, n, nv, nv, nv), dtype=tdt, device="cuda")
        m = s["m"]
        for j0 in range(0, ny, rows_per_chunk):
            j1 = min(j0 + rows_per_chunk, ny)
            nn = torch.as_tensor(ns[j0:j1], device="cuda")
            uu = torch.as_tensor(us[j0:j1], device="cuda")
            pre = nn * (m / (2 * math.pi * Ts)) ** 1.5
            g = [torch.exp(-0.5 * m * (v[k][None, None, :] - uu[..., k, None]) ** 2 / Ts) for k in range(3)]
            blk = (pre[..., None, None, None] * g[0][..., :, None, None] * g[1][..., None, :, None]
                   * g[2][..., None, None, :])
            out[j0:j1] = blk.to(tdt)
        f.append(out)
    return cfg, f, F


def tail(nx=1024, ny=512, nv=12, mass_ratio=100.0, c=30.0, lam=0.6, Ti_Te=3.0, Bg=0.1, noise=1e-4,
         ve_max=20.0, vi_max=5.0, dt=0.0012, steps=20, fit=True, seed=0, dtype=np.float32):
    """Magnetotail-like set-up (Sec. 4.1): Harris sheet carrying the current,
    static background at n0/3 and T0/3, guide field -Bg, seeded noise on B_x."""
    Lx, Ly = 120.0, 40.0
    Te = 0.5 / (1.0 + Ti_Te)
    Ti = Ti_Te * Te
    me = 1.0 / mass_ratio
    nbg = 1.0 / 3.0
    sp = [_species(-1.0, me, ve_max, nv), _species(1.0, 1.0, vi_max, nv)]
    cfg = dict(kind="2x3v", nx=nx, ny=ny, x_lo=-Lx / 2, x_hi=Lx / 2, y_lo=-Ly / 2, y_hi=Ly / 2,
               c=c, species=sp, fit=fit, dt=dt, steps=steps,
               name=f"tail {nx}x{ny}x{nv}^3 mi/me={mass_ratio:g}")
    x = _centres(-Lx / 2, Lx / 2, nx)
    y = _centres(-Ly / 2, Ly / 2, ny)
    X, Y = np.meshgrid(x, y)
    ns = 1.0 / np.cosh(Y / lam) ** 2
    uzi = np.full_like(ns, -Ti / (lam * (Ti + Te)))
    uze = -uzi * Te / Ti
    f = []
    for s, (uz, T) in zip(sp, ((uze, Te), (uzi, Ti))):
        v = [_centres(s["v_lo"][d], s["v_hi"][d], s["nv"][d]) for d in range(3)]
        blk = _maxwellian_block(ns, uz, T, s["m"], v)
        blk += _maxwellian_block(np.full_like(ns, nbg), np.zeros_like(ns), T / 3.0, s["m"], v)
        f.append(blk.astype(dtype))
    F = Yee0(nx, ny)
    dy = Ly / ny
    yf = -Ly / 2 + np.arange(ny + 1) * dy
    rng = np.random.default_rng(seed)
    F.Bx = np.tanh(yf / lam)[:, None] + noise * rng.uniform(-1.0, 1.0, size=(ny + 1, nx))
    F.Bz[:] = -Bg
    return cfg, f, F


def random_block(shape, seed, kind="smooth"):
    """Seeded non-negative test data for sweep/moment parity: 'smooth'
    (Maxwellian-like with a seeded modulation), 'rough' (uniform random) or
    'step' (piecewise constant with jumps)."""
    rng = np.random.default_rng(seed)
    if kind == "rough":
        return rng.uniform(0.0, 1.0, size=shape)
    if kind == "step":
        a = (rng.uniform(size=shape) > 0.5).astype(np.float64)
        return a * rng.uniform(0.5, 1.0, size=shape)
    out = np.ones(shape)
    for ax, n in enumerate(shape):
        c = (np.arange(n) + 0.5) / n - 0.5
        w = rng.uniform(0.15, 0.35)
        sh = [1] * len(shape)
        sh[ax] = n
        out = out * np.exp(-0.5 * (c / w) ** 2).reshape(sh)
    return out * (1.0 + 0.3 * rng.uniform(-1, 1, size=shape))


CONFIGS = {
    "landau": dict(builder="landau", kwargs=dict()),
    "twostream": dict(builder="twostream", kwargs=dict()),
    "gem": dict(builder="gem", kwargs=dict()),
    "tail": dict(builder="tail", kwargs=dict()),
}


def mlp_init(seed=0):
    """Initial parameters of the heat-flux network (13520 FP32 values, layout
    W1[64][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[16][64] b4[16]):
    Glorot-uniform weights, zero biases, the six padding output rows zero.
    Random numbers only; the network itself lives elsewhere."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((64, 64), (64, 64), (64, 64), (16, 64)):
        lim = math.sqrt(6.0 / (fan_in + (10 if fan_out == 16 else fan_out)))
        W = rng.uniform(-lim, lim, size=(fan_out, fan_in))
        if fan_out == 16:
            W[10:] = 0.0
        parts += [W.ravel(), np.zeros(fan_out)]
    return np.concatenate(parts).astype(np.float32)
