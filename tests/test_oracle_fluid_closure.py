"""Pins of the oracle's ten-moment fluid model run with a heat-flux closure
(Sec. 2.3, Eq. 5), the fluid-only step.

* Eq. 5 on temperature modes between the y walls: the mirrored second
  difference has the cosine (even components) and sine (odd components,
  T_xy) modes of the cell-centred grid as eigenvectors with eigenvalue
  (2 cos(k dy) - 2)/dy^2, so div Q = -chi d_s n v_t lambda T' exactly;
* a uniform, isotropic plasma at rest in a uniform B_z is steady under the
  fluid-only step with the gradient closure, fields included;
* the step conserves the total density (flux form; the closure acts on P);
* the closure's contribution to one step, the difference of the steps with
  and without the Eq. 5 source, is dt times the source to first order in
  dt on a temperature mode: its relative error falls linearly with dt.
"""
import math

import numpy as np
import pytest

from oracle import fields, fluid
from oracle import mlp as OM
from oracle import step as OS
from paper_2109_06743_amd import workloads as W


def _iso_state(ny, nx, m, n, T6):
    """U of a plasma at rest: n[ny, nx], T6[ny, nx, 6] (PAIRS order)."""
    U = np.zeros((ny, nx, 10))
    U[..., 0] = n
    U[..., 4:10] = n[..., None] * T6
    return U


@pytest.mark.parametrize("comp,odd", [(3, False), (1, True)])
def test_gradient_closure_y_modes_between_walls(comp, odd):
    m, q = 0.04, -1.0
    ny, nx, dx, dy = 12, 4, 0.3, 0.25
    T0, e = 0.5, 0.05
    mode = 2 if not odd else 1
    k = math.pi * mode / (ny * dy)
    yc = (np.arange(ny) + 0.5) * dy
    shape = np.cos(k * yc) if not odd else np.sin(k * yc)
    T6 = np.zeros((ny, nx, 6))
    T6[..., 0] = T6[..., 3] = T6[..., 5] = T0
    T6[..., comp] += T0 * e * shape[:, None]
    n = np.ones((ny, nx))
    U = _iso_state(ny, nx, m, n, T6)
    d = OM.gradient_closure_divergence(U, m, q, dx, dy)
    lam = (2 * math.cos(k * dy) - 2) / dy ** 2
    vt = np.sqrt((T6[..., 0] + T6[..., 3] + T6[..., 5]) / (3 * m))
    want = -OM.CHI * math.sqrt(m) * vt * lam * (T0 * e * shape[:, None])
    np.testing.assert_allclose(d[..., comp], want, rtol=1e-10, atol=1e-13)
    others = [c for c in range(6) if c != comp]
    np.testing.assert_allclose(d[..., others], 0.0, atol=1e-13)


def _gem_small(nx=16, ny=8):
    cfg, U, F0 = W.gem_fluid(nx=nx, ny=ny)
    F = fields.Yee(nx, ny)
    for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        setattr(F, k, getattr(F0, k).copy())
    return cfg, U, F


def test_uniform_magnetised_plasma_is_steady():
    cfg, _, F = _gem_small()
    nx, ny = cfg["nx"], cfg["ny"]
    U = [_iso_state(ny, nx, sp["m"], np.ones((ny, nx)), np.tile([0.1, 0, 0, 0.1, 0, 0.1], (ny, nx, 1)))
         for sp in cfg["species"]]
    F = fields.Yee(nx, ny)
    F.Bz = np.full_like(F.Bz, 0.3)
    out = OS.fluid_step_2x3v({"U": U, "F": F}, cfg, 0.01, "gradient")
    for a, b in zip(out["U"], U):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    for c in ("Ex", "Ey", "Ez", "Bx", "By"):
        np.testing.assert_allclose(getattr(out["F"], c), 0.0, atol=1e-15)
    np.testing.assert_allclose(out["F"].Bz, 0.3, rtol=0, atol=1e-15)


def test_fluid_step_conserves_density():
    cfg, U, F = _gem_small()
    st = {"U": U, "F": F}
    for _ in range(3):
        st = OS.fluid_step_2x3v(st, cfg, cfg["dt"], "gradient")
    for a, b in zip(st["U"], U):
        assert abs(a[..., 0].sum() - b[..., 0].sum()) <= 1e-13 * b[..., 0].sum()


def test_closure_contribution_is_dt_times_eq5_source():
    m, q = 1.0, 1.0
    ny, nx, dx, dy = 3, 32, 0.25, 0.25
    k = 2 * math.pi / (nx * dx)
    xc = (np.arange(nx) + 0.5) * dx
    T6 = np.zeros((ny, nx, 6))
    T6[..., 0] = 0.5 * (1 + 0.1 * np.cos(k * xc))[None, :]
    T6[..., 3] = T6[..., 5] = 0.5
    U = _iso_state(ny, nx, m, np.ones((ny, nx)), T6)
    zero = (np.zeros((ny, nx, 3)), np.zeros((ny, nx, 3)))

    def qcal0(V, Bs):
        return OM.qcal_from_closure(V, np.zeros(V.shape[:-1] + (10,)), 0.0, m)

    def src(V):
        S = np.zeros(V.shape)
        S[..., 4:10] = -OM.gradient_closure_divergence(V, m, q, dx, dy)
        return S
    errs = []
    for dt in (2e-3, 1e-3):
        with_c = fluid.rk3_3v_closure(U, qcal0, src, zero, zero, zero, q, m, dx, dy, dt)
        without = fluid.rk3_3v_closure(U, qcal0, None, zero, zero, zero, q, m, dx, dy, dt)
        got = (with_c - without)[..., 4]
        want = dt * src(U)[..., 4]
        errs.append(np.abs(got - want).max() / np.abs(want).max())
    assert errs[0] < 0.05
    assert 1.6 < errs[0] / errs[1] < 2.4, errs
