"""Pins of the oracle's periodic-y path (the Orszag-Tang set-up, Sec. 3.2).

* the y sweep of every v_y cell is a cyclic pencil: integer Courant numbers
  give rolls (to rounding of the flux form), and mass is conserved;
* with no current the Yee half steps keep the discrete divergence of E
  (Gauss's law residual) constant across the periodic seam;
* the Orszag-Tang initial state satisfies the discrete Gauss law exactly
  (the electron density is built from it);
* the ten-moment fluid with no fields conserves n and both in-plane momenta
  (the y flux leaves through the seam and comes back);
* the full step conserves the mass of both species.
"""
import numpy as np

from oracle import fields as OF
from oracle import fluid
from oracle import moments as OM
from oracle import step as OS
from oracle import vlasov as OV
from paper_2109_06743_amd import workloads as W


def _yee(F0, nx, ny):
    F = OF.Yee(nx, ny)
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
    return F


def test_periodic_y_sweep_integer_shift_is_a_roll():
    rng = np.random.default_rng(5)
    ny, nx, nv = 9, 4, 7
    f = rng.random((ny, nx, nv, nv, nv))
    vy = OV.centres(-3.5, 3.5, nv)[0]               # cell centres -3 .. 3
    dy, tau = 1.0, 1.0                               # every v_y cell moves a whole number of rows
    out = OV.y_sweep_2x3v(f, vy, dy, tau, f.max(), "periodic")
    for jy in range(nv):
        k = int(round(vy[jy] * tau / dy))
        np.testing.assert_allclose(out[:, :, :, jy, :], np.roll(f[:, :, :, jy, :], k, axis=0), rtol=0, atol=1e-14)
    assert abs(out.sum() - f.sum()) <= 1e-12 * f.sum()


def test_gauss_residual_constant_across_the_seam():
    cfg, _, F0 = W.orszag_tang(n=12, nv=4, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    F = _yee(F0, nx, ny)
    F.Bz = F.Bz + 0.05 * np.cos(2 * np.pi * np.arange(ny + 1)[:, None] / ny)   # a field that changes E at the seam

    def div(F):
        return (F.Ex - np.roll(F.Ex, 1, axis=1)) / dx + (F.Ey[1:] - F.Ey[:-1]) / dy
    d0 = div(F)
    for _ in range(5):
        F = OF.maxwell_half_step(F, np.zeros((ny, nx, 3)), cfg["dt"], cfg["c"], dx, dy, "periodic")
    np.testing.assert_allclose(div(F), d0, atol=1e-11)
    np.testing.assert_allclose(F.Ey[0], F.Ey[ny], atol=1e-15)      # the seam rows stay one set of points
    np.testing.assert_allclose(F.Bx[0], F.Bx[ny], atol=1e-15)


def test_orszag_tang_initial_state_satisfies_gauss():
    cfg, f, F = W.orszag_tang(n=16, nv=20, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    divE = (F.Ex - np.roll(F.Ex, 1, axis=1)) / dx + (F.Ey[1:] - F.Ey[:-1]) / dy
    _, prof, _ = W._ot_setup(nx, ny, 20, 100.0, cfg["c"], 0.1, 0.2, 0.2, 14.0, 1.5, cfg["dt"], 1, True)
    ne, ni = prof[0][0], prof[1][0]
    np.testing.assert_allclose(divE, (ni - ne) * cfg["c"] ** 2, rtol=1e-12, atol=1e-12)


def test_periodic_fluid_conserves_n_and_momentum():
    cfg, f, _ = W.orszag_tang(n=12, nv=8, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    dx = (cfg["x_hi"] - cfg["x_lo"]) / nx
    dy = (cfg["y_hi"] - cfg["y_lo"]) / ny
    sp = cfg["species"][1]
    v, dv = OS._grids(cfg, sp)
    mom = OM.raw_moments_3v(f[1], v, dv, sp["m"])
    U = mom[..., :10].copy()
    zero = (np.zeros((ny, nx, 3)), np.zeros((ny, nx, 3)))
    U1 = fluid.rk3_3v(U, mom[..., 10:], mom[..., 10:], zero, zero, zero, sp["q"], sp["m"], dx, dy, 0.01, "periodic")
    for k in (0, 1, 2):
        assert abs(U1[..., k].sum() - U[..., k].sum()) <= 1e-13 * max(abs(U[..., 0]).sum(), 1.0), k


def test_periodic_step_conserves_mass():
    cfg, f, F0 = W.orszag_tang(n=8, nv=8, dtype=np.float64)
    nx, ny = cfg["nx"], cfg["ny"]
    F = _yee(F0, nx, ny)
    moms, Us = [], []
    for k, sp in enumerate(cfg["species"]):
        v, dv = OS._grids(cfg, sp)
        mm = OM.raw_moments_3v(f[k], v, dv, sp["m"])
        moms.append(mm)
        Us.append(mm[..., :10].copy())
    st = dict(f=f, U=Us, mom_post=moms, F=F)
    m0 = [x.sum() for x in f]
    for _ in range(2):
        st = OS.step_2x3v(st, cfg, cfg["dt"])
    for a, b in zip(st["f"], m0):
        assert abs(a.sum() - b) <= 1e-12 * b
