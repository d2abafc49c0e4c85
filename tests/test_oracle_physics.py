"""Physics pins of the oracle's full steps.

* Linear Landau damping (Sec. 3.1): damping rate and frequency match the root
  of the kinetic dispersion relation 1 + k^-2 (1 + zeta Z(zeta)) = 0 (computed
  here with the Faddeeva function) and the values the paper prints
  (tests/golden/landau_linear.json), for standard PFC and for moment fitting.
* Standard PFC and moment fitting give the same linear Landau result
  (Sec. 3.1: "no correction of the moments is to be expected").
* Two-stream growth (two beams +-2.4, v_t 0.5, k 0.2) matches the kinetic root.
* V(tau) with a uniform B along z turns the mean velocity of a drifting
  Maxwellian at the cyclotron frequency (Eq. 1's Lorentz term).
* 2X3V GEM-like run: mass conserved to round-off, f >= 0, and moment fitting
  conserves total energy far better than standard PFC at coarse velocity
  resolution (Sec. 3.3's central claim).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import wofz

from oracle import fields, moments, step, vlasov
from paper_2109_06743_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _Z(z):
    return 1j * math.sqrt(math.pi) * wofz(z)


def _root(eps, w0):
    w = w0
    for _ in range(60):
        h = 1e-7
        d = (eps(w + h) - eps(w - h)) / (2 * h)
        w = w - eps(w) / d
    return w


def landau_root(k=0.5):
    return _root(lambda w: 1 + (1 + (w / (math.sqrt(2) * k)) * _Z(w / (math.sqrt(2) * k))) / k ** 2,
                 1.4 - 0.15j)


def twostream_root(k=0.2, vd=2.4, vt=0.5):
    def eps(w):
        s = 0
        for vb in (vd, -vd):
            z = (w - k * vb) / (math.sqrt(2) * k * vt)
            s += 0.5 / (k * k * vt * vt) * (1 + z * _Z(z))
        return 1 + s
    return _root(eps, 0.3j)


def _run_1x1v(cfg, f, steps, dt):
    v, dv = vlasov.centres(cfg["v_lo"], cfg["v_hi"], cfg["nv"])
    dx = (cfg["x_hi"] - cfg["x_lo"]) / cfg["nx"]
    mom = moments.raw_moments_1v(f, v, dv, cfg["m"])
    st = {"f": f, "mom_post": mom, "U": mom[:, :3].copy()}
    WE, E1 = [], []
    for _ in range(steps):
        st = step.step_1x1v(st, cfg, dt)
        E = fields.efield_1x1v(st["mom_post"][:, 0], dx, cfg["q"])
        WE.append(0.5 * (E * E).sum() * dx)
        E1.append(abs(np.fft.rfft(E)[1]))
    return st, np.array(WE), np.array(E1)


def _peaks(t, y):
    out_t, out_y = [], []
    for i in range(1, len(y) - 1):
        if y[i] > y[i - 1] and y[i] > y[i + 1]:
            a, b, c = y[i - 1], y[i], y[i + 1]
            d = 0.5 * (a - c) / (a - 2 * b + c)
            out_t.append(t[i] + d * (t[1] - t[0]))
            out_y.append(b - 0.25 * (a - c) * d)
    return np.array(out_t), np.array(out_y)


def test_landau_root_matches_printed_analytic():
    g = json.load(open(os.path.join(GOLDEN, "landau_linear.json")))
    w = landau_root(0.5)
    assert w.real == pytest.approx(g["omega_analytic_printed"], abs=1e-3)
    assert -w.imag == pytest.approx(g["gamma_analytic_printed"], abs=1e-4)


@pytest.fixture(scope="module")
def landau_runs():
    out = {}
    for fit in (False, True):
        cfg, f = W.landau(fit=fit)
        out[fit] = _run_1x1v(cfg, f, cfg["steps"], cfg["dt"])
    return out


@pytest.mark.parametrize("fit", [False, True])
def test_linear_landau_damping(landau_runs, fit):
    g = json.load(open(os.path.join(GOLDEN, "landau_linear.json")))
    st, WE, _ = landau_runs[fit]
    t = 0.1 * np.arange(1, len(WE) + 1)
    tp, yp = _peaks(t, np.log(WE))
    sel = tp >= 1.0
    gamma = -np.polyfit(tp[sel], yp[sel], 1)[0] / 2
    omega = math.pi / np.mean(np.diff(tp[sel]))
    w = landau_root(0.5)
    assert gamma == pytest.approx(-w.imag, rel=0.03)
    assert omega == pytest.approx(w.real, rel=0.01)
    assert gamma == pytest.approx(g["gamma_printed"], rel=0.03)
    assert omega == pytest.approx(g["omega_printed"], rel=0.01)


def test_fit_and_standard_pfc_agree_on_landau(landau_runs):
    f0 = landau_runs[False][0]["f"]
    f1 = landau_runs[True][0]["f"]
    assert np.linalg.norm(f1 - f0) / np.linalg.norm(f0) < 1e-4
    WE0, WE1 = landau_runs[False][1], landau_runs[True][1]
    t = 0.1 * np.arange(1, len(WE0) + 1)
    tp0, yp0 = _peaks(t, np.log(WE0))
    tp1, yp1 = _peaks(t, np.log(WE1))
    np.testing.assert_allclose(tp1, tp0, atol=2e-2)       # same oscillation (0.2 %)
    np.testing.assert_allclose(yp1, yp0, atol=2e-2)       # same damping envelope


def test_twostream_growth_rate():
    cfg, f = W.twostream(nx=32, nv=128)
    _, _, E1 = _run_1x1v(cfg, f, 180, 0.1)
    t = 0.1 * np.arange(1, 181)
    sel = (t >= 8) & (t <= 18)
    gamma = np.polyfit(t[sel], np.log(E1[sel]), 1)[0]
    assert twostream_root().imag == pytest.approx(0.3132, abs=1e-4)
    assert gamma == pytest.approx(twostream_root().imag, rel=0.05)


def test_v_rotation_in_uniform_Bz():
    n = 20
    vmax = 5.0
    v, h = vlasov.centres(-vmax, vmax, n)
    vv, dv = [v, v, v], [h, h, h]
    m, q, B = 1.0, 1.0, 1.0
    u0 = np.array([1.0, 0.0, 0.0])
    f = moments.maxwellian_3v(1.0, u0, np.eye(3) * 0.6, m, vv, dv)[None, None]
    E = np.zeros((1, 1, 3))
    Bv = np.zeros((1, 1, 3))
    Bv[..., 2] = B
    tau, steps = 0.05, 20
    for _ in range(steps):
        f = vlasov.v_advect_3v(f, E, Bv, q, m, vv, dv, tau)
    u = moments.derived_3v(moments.raw_moments_3v(f[0, 0], vv, dv, m), m)["u"]
    angle = math.atan2(u[1], u[0])
    assert angle == pytest.approx(-q * B / m * tau * steps, abs=2e-3)
    assert abs(u[2]) < 1e-12
    assert f.sum() * h ** 3 == pytest.approx(1.0, rel=1e-13)


def _gem_small(fit, steps=12):
    cfg, f, F0 = W.gem(nx=8, ny=4, nv=16, dt=0.003, fit=fit, dtype=np.float64)
    F = fields.Yee(cfg["nx"], cfg["ny"])
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
    mom, U = [], []
    for k, sp in enumerate(cfg["species"]):
        v, dv = step._grids(cfg, sp)
        mm = moments.raw_moments_3v(f[k], v, dv, sp["m"])
        mom.append(mm)
        U.append(mm[..., :10].copy())
    st = dict(f=f, U=U, mom_post=mom, F=F)
    e0 = sum(step.energy_2x3v(st, cfg))
    mass0 = [x.sum() for x in f]
    for _ in range(steps):
        st = step.step_2x3v(st, cfg, cfg["dt"])
    e1 = sum(step.energy_2x3v(st, cfg))
    return st, (e1 - e0) / e0, mass0


@pytest.mark.slow
def test_gem_small_conservation_and_energy():
    st_fit, drift_fit, mass0 = _gem_small(True)
    st_pfc, drift_pfc, _ = _gem_small(False)
    for st in (st_fit, st_pfc):
        for f, m0 in zip(st["f"], mass0):
            assert f.sum() == pytest.approx(m0, rel=1e-13)
            assert (f >= 0).all()
    assert abs(drift_pfc) > 5e-3            # standard PFC heats at 16^3
    assert abs(drift_fit) < 2e-4            # moment fitting holds energy


def test_energy_1x1v_closed_forms():
    """Kinetic energy of f = (1 + e cos kx) M(v), M a Maxwellian of
    temperature T sampled at the velocity cell centres, is (1/2) T L (the cos
    term integrates to zero over whole periods, the midpoint rule on a
    Gaussian is exact to far below 1e-12 here); with q = -1 the spectral
    Gauss law gives E = -e sin(kx)/k exactly for one mode, so the field energy
    is (1/2)(e/k)^2 L/2."""
    L, nx, nv, T, e = 4 * math.pi, 32, 256, 1.3, 0.07
    k = 2 * math.pi / L
    cfg = dict(kind="1x1v", nx=nx, x_lo=0.0, x_hi=L, nv=nv, v_lo=-10.0, v_hi=10.0, q=-1.0, m=1.0)
    v = -10.0 + (np.arange(nv) + 0.5) * 20.0 / nv
    x = (np.arange(nx) + 0.5) * L / nx
    M = np.exp(-v * v / (2 * T)) / math.sqrt(2 * math.pi * T)
    f = (1 + e * np.cos(k * x))[:, None] * M[None, :]
    kin, fld = step.energy_1x1v(f, cfg)
    assert kin == pytest.approx(0.5 * T * L, rel=1e-12)
    assert fld == pytest.approx(0.5 * (e / k) ** 2 * L / 2, rel=1e-10)
