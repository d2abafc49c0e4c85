"""Pins of the oracle's backsubstitution velocity split (Sec. 2.1 names the
method; the oracle factors the implicit-midpoint Lorentz map into three
one-dimensional affine maps, oracle.vlasov.v_advect_3v_backsub), against
facts fixed outside the oracle:

* the map v -> R v + c is Boris' rotation: v- = v + (q tau/2m) E,
  v+ = v- + (v- + v- x t) x s with t = (q tau/2m) B, s = 2t/(1 + t^2),
  v' = v+ + (q tau/2m) E (Boris 1970, as restated in every PIC text); R is
  orthogonal and turns about B by 2 atan(Omega tau / 2);
* the three factor maps, applied x, y, z, compose to that map;
* the affine sweep with per-face feet integrates the limited parabola
  exactly, so cell averages of a quadratic map to the cell averages of the
  transformed density q((xi - s)/alpha)/alpha; with alpha = 1 it is the
  uniform sweep; it conserves mass and keeps f >= 0;
* the mean velocity of a drifting Maxwellian follows the Boris map step by
  step (angle 2 atan(Omega tau/2), not Omega tau: at Omega tau = 0.5 the
  two differ by 0.0100 per step); with B = 0 and whole-cell shifts f moves
  exactly.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import moments, vlasov
from oracle.pfc import pfc_sweep, pfc_sweep_affine


def _boris(v, E, B, q, m, tau):
    h = 0.5 * tau * q / m
    vm = v + h * E
    t = h * B
    s = 2.0 * t / (1.0 + t @ t)
    vp = vm + np.cross(vm + np.cross(vm, t), s)
    return vp + h * E


@pytest.mark.parametrize("seed", range(4))
def test_lorentz_map_is_boris_rotation(seed):
    rng = np.random.default_rng(seed)
    E, B = rng.normal(size=3), rng.normal(size=3)
    q, m, tau = (1.0, 1.0, 0.3) if seed % 2 else (-1.0, 0.04, 0.05)
    R, c = vlasov.lorentz_map(E, B, q, m, tau)
    for v in rng.normal(size=(5, 3)):
        np.testing.assert_allclose(R @ v + c, _boris(v, E, B, q, m, tau), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
    ang = math.acos(max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0)))
    Om = abs(q) * np.linalg.norm(B) / m
    assert ang == pytest.approx(2.0 * math.atan(Om * tau / 2.0), rel=1e-12)
    np.testing.assert_allclose(R @ B, B, rtol=1e-13, atol=1e-13)    # the axis is B


@pytest.mark.parametrize("seed", range(4))
def test_factors_compose_to_the_map(seed):
    rng = np.random.default_rng(10 + seed)
    E, B = rng.normal(size=3), rng.normal(size=3) * 2
    R, c = vlasov.lorentz_map(E, B, -1.0, 1.0, 0.4)
    a, b, e, cx, d, g, h, cy, k, l, n, cz = vlasov.backsub_factors(R, c)
    for v in rng.normal(size=(6, 3)):
        x = a * v[0] + b * v[1] + e * v[2] + cx
        y = d * x + g * v[1] + h * v[2] + cy
        z = k * x + l * y + n * v[2] + cz
        np.testing.assert_allclose([x, y, z], R @ v + c, rtol=1e-13, atol=1e-13)
    assert a * g * n == pytest.approx(1.0, abs=1e-13)                 # volume preserving overall


def _avg_quad(cq, lo, hi):
    P = lambda x: cq[0] * x + cq[1] * x * x / 2 + cq[2] * x ** 3 / 3
    return (P(hi) - P(lo)) / (hi - lo)


@pytest.mark.parametrize("alpha,s", [(0.9, 0.4), (1.12, -1.3), (0.8, 2.6), (1.3, -0.45), (1.0, 1.7)])
def test_affine_sweep_quadratic_exact(alpha, s):
    """Content at xi moves to alpha xi + s: the density becomes
    q((xi - s)/alpha)/alpha, whose cell average over [i, i+1] is
    (Q((i+1-s)/alpha) - Q((i-s)/alpha)) with Q the primitive of q."""
    N = 40
    cq = np.array([50.0, 0.6, 0.01])              # positive and gentle: no limiter action
    e = np.arange(N + 1, dtype=float)
    f = _avg_quad(cq, e[:-1], e[1:])[None]
    out = pfc_sweep_affine(f, alpha, s, 1e30)[0]
    P = lambda x: cq[0] * x + cq[1] * x * x / 2 + cq[2] * x ** 3 / 3
    expect = P((e[1:] - s) / alpha) - P((e[:-1] - s) / alpha)
    # cells off the walls (a zero-flux wall keeps what would leave the box)
    # whose feet and stencils stay inside the box
    ok = [i for i in range(1, N - 1) if 2 <= (i - s) / alpha <= N - 3 and 2 <= (i + 1 - s) / alpha <= N - 3]
    assert len(ok) > 20
    np.testing.assert_allclose(out[ok], expect[ok], rtol=1e-12)


def test_affine_sweep_unit_stretch_is_uniform_sweep():
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, size=(9, 15))
    s = rng.uniform(-4, 4, size=9)
    # the same arithmetic up to the order of the whole-cell sums (cumulative here)
    np.testing.assert_allclose(pfc_sweep_affine(f, 1.0, s, f.max()), pfc_sweep(f, s, "zeroflux", f.max()),
                               rtol=0, atol=1e-14)


@settings(max_examples=50, deadline=None)
@given(seed=st.integers(0, 2 ** 31 - 1), alpha=st.floats(0.7, 1.4), s=st.floats(-5.0, 5.0),
       kind=st.sampled_from(["rough", "step", "spiky"]))
def test_affine_sweep_mass_and_positivity(seed, alpha, s, kind):
    rng = np.random.default_rng(seed)
    n = 18
    if kind == "rough":
        f = rng.uniform(0, 1, size=(3, n))
    elif kind == "step":
        f = (rng.uniform(size=(3, n)) > 0.5) * 1.0
    else:
        f = rng.uniform(0, 1, size=(3, n)) ** 8
    out = pfc_sweep_affine(f, alpha, s, f.max())
    assert (out >= 0).all()
    np.testing.assert_allclose(out.sum(1), f.sum(1), rtol=1e-13, atol=1e-15)


def _mean_u(f, vv, dv, m):
    return moments.derived_3v(moments.raw_moments_3v(f, vv, dv, m), m)["u"]


@pytest.mark.parametrize("Bv,E", [([0.0, 0.0, 1.0], [0.0, 0.0, 0.0]),
                                  ([1.0, 0.0, 0.0], [0.0, 0.0, 0.0]),
                                  ([0.5, -0.6, 0.62], [0.05, -0.1, 0.08])])
def test_mean_velocity_follows_boris_map(Bv, E):
    n, vmax, T, m, q, tau, steps = 28, 6.0, 0.9, 1.0, 1.0, 0.5, 8
    v, h = vlasov.centres(-vmax, vmax, n)
    vv, dv = [v, v, v], [h, h, h]
    u0 = np.array([1.2, -0.4, 0.6])
    f = moments.maxwellian_3v(1.0, u0, np.eye(3) * T, m, vv, dv)[None, None]
    Ef, Bf = np.asarray(E, float).reshape(1, 1, 3), np.asarray(Bv, float).reshape(1, 1, 3)
    u_b = _mean_u(f[0, 0], vv, dv, m)
    for _ in range(steps):
        f = vlasov.v_advect_3v_backsub(f, Ef, Bf, q, m, vv, dv, tau)
        u_b = _boris(u_b, np.asarray(E, float), np.asarray(Bv, float), q, m, tau)
    u = _mean_u(f[0, 0], vv, dv, m)
    np.testing.assert_allclose(u, u_b, atol=3e-3)
    assert f.sum() * h ** 3 == pytest.approx(1.0, rel=1e-13)
    assert (f >= 0).all()
    if np.allclose(E, 0):
        # the exact rotation (angle Omega tau per step) is a different point
        b = np.asarray(Bv) / np.linalg.norm(Bv)
        w = u0 - b * (b @ u0)
        ang = -q * np.linalg.norm(Bv) / m * tau * steps
        u_ex = b * (b @ u0) + w * math.cos(ang) + np.cross(b, w) * math.sin(ang)
        assert np.linalg.norm(u_ex - u_b) > 0.05


def test_whole_cell_shifts_with_b_zero_are_exact():
    n, vmax, m, q = 12, 3.0, 1.0, -1.0
    v, h = vlasov.centres(-vmax, vmax, n)
    vv, dv = [v, v, v], [h, h, h]
    rng = np.random.default_rng(5)
    f = rng.uniform(0.1, 1.0, size=(1, 1, n, n, n))
    tau = 1.0
    E = np.array([2.0, -1.0, 3.0]) * h / (q / m * tau)            # shifts of 2, -1 and 3 cells
    g = vlasov.v_advect_3v_backsub(f, E.reshape(1, 1, 3), np.zeros((1, 1, 3)), q, m, vv, dv, tau)
    ref = f[0, 0]
    for axis, K in ((0, 2), (1, -1), (2, 3)):
        ref = np.moveaxis(pfc_sweep(np.moveaxis(ref, axis, -1).reshape(-1, n), np.full(n * n, float(K)),
                                    "zeroflux", f.max()).reshape(np.moveaxis(ref, axis, -1).shape), -1, axis)
    np.testing.assert_allclose(g[0, 0], ref, rtol=0, atol=1e-14)
    # whole-cell moves are exact: away from the wall cells (which keep what
    # would leave the box) the values are the input's, moved (+2, -1, +3),
    # up to the rounding of the solved shift (2 + 4e-16 cells)
    np.testing.assert_allclose(g[0, 0, 2:n - 1, 1:n - 1, 3:n - 1], f[0, 0, 0:n - 3, 2:n, 0:n - 4], rtol=0, atol=1e-14)


def test_backsub_and_strang_agree_at_small_omega_tau():
    """The two splittings of the same Lorentz term differ by the Strang split's
    O((Omega tau)^3) error and the Boris angle's: small at Omega tau = 0.05."""
    n, vmax, T, m, q = 20, 5.0, 0.6, 1.0, 1.0
    v, h = vlasov.centres(-vmax, vmax, n)
    vv, dv = [v, v, v], [h, h, h]
    f = moments.maxwellian_3v(1.0, np.array([0.8, 0.3, -0.2]), np.eye(3) * T, m, vv, dv)[None, None]
    E = np.array([[[0.1, -0.05, 0.02]]])
    B = np.array([[[0.3, 0.5, 0.8]]])
    a = vlasov.v_advect_3v(f, E, B, q, m, vv, dv, 0.05)
    b = vlasov.v_advect_3v_backsub(f, E, B, q, m, vv, dv, 0.05)
    assert np.linalg.norm(a - b) / np.linalg.norm(f) < 2e-3
