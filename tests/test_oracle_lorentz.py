"""Pins of the oracle's 3V velocity operator V(tau) (the (q/m)(E + v x B)
term of Eq. 1) against the exact motion under a uniform field, which the
mean velocity u of a drifting Maxwellian follows:

    du/dt = (q/m) (E + u x B)
    u(t) = u_par(0) + (q/m) E_par t  +  v_d  +  R_b(-Omega t) (u_perp(0) - v_d),

with b = B/|B|, Omega = q|B|/m, v_d = E x B / |B|^2 and R_b the rotation
about b (Rodrigues' formula).  The split operator reproduces it up to the
splitting error, O((Omega tau)^3) per step; a sign or index mistake in any of
the Lorentz terms (v_y B_z, v_z B_y, v_z B_x, v_x B_z, v_x B_y, v_y B_x, or
an E component) is an O(Omega tau) error per step.  With B = 0 the mean
velocity grows by exactly (q/m) E tau per step: the flux form moves the first
moment of a pencil by exactly its shift wherever the limiter does not act.
That check lifts the limiter's upper bound and resolves the Maxwellian
finely enough (v_t = 3 cells) that the positivity side of the limiter acts
only on the far tails, which leaves a residual below 2e-5 of the gain.
"""
import math

import numpy as np
import pytest

from oracle import moments, vlasov


def _grid(n=20, vmax=5.0):
    v, h = vlasov.centres(-vmax, vmax, n)
    return [v, v, v], [h, h, h]


def _exact_u(u0, E, B, q, m, t):
    B = np.asarray(B, float)
    E = np.asarray(E, float)
    Bm = np.linalg.norm(B)
    if Bm == 0.0:
        return u0 + q / m * E * t
    b = B / Bm
    Om = q * Bm / m
    vd = np.cross(E, B) / Bm ** 2
    upar0 = b * (b @ u0)
    w = u0 - upar0 - vd                          # perpendicular part relative to the drift
    ang = -Om * t                                # dw/dt = Omega w x b
    w_t = w * math.cos(ang) + np.cross(b, w) * math.sin(ang)
    return upar0 + q / m * b * (b @ E) * t + vd + w_t


def _run(u0, E, B, q, m, tau, steps, T=0.6, f_inf=None, n=20, vmax=5.0):
    vv, dv = _grid(n, vmax)
    f = moments.maxwellian_3v(1.0, np.asarray(u0), np.eye(3) * T, m, vv, dv)[None, None]
    Ef = np.asarray(E, float).reshape(1, 1, 3)
    Bf = np.asarray(B, float).reshape(1, 1, 3)
    for _ in range(steps):
        f = vlasov.v_advect_3v(f, Ef, Bf, q, m, vv, dv, tau, f_inf=f_inf)
    d = moments.derived_3v(moments.raw_moments_3v(f[0, 0], vv, dv, m), m)
    return d["u"], f.sum() * dv[0] * dv[1] * dv[2]


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("q", [1.0, -1.0])
def test_gyration_about_each_axis(axis, q):
    m, Bm, tau, steps = 1.0, 1.0, 0.02, 50
    B = np.zeros(3)
    B[axis] = Bm
    u0 = np.array([0.9, -0.5, 0.7])
    u, mass = _run(u0, [0, 0, 0], B, q, m, tau, steps)
    ex = _exact_u(u0, [0, 0, 0], B, q, m, tau * steps)
    np.testing.assert_allclose(u, ex, atol=2e-3)
    # the component along B is untouched (the two shears that see it cancel exactly)
    assert u[axis] == pytest.approx(u0[axis], abs=1e-3)
    assert mass == pytest.approx(1.0, rel=1e-13)


@pytest.mark.parametrize("q", [1.0, -1.0])
def test_gyration_about_oblique_field(q):
    m, tau, steps = 0.5, 0.01, 100
    B = np.array([0.6, -0.5, 0.45])
    u0 = np.array([0.4, 0.8, -0.6])
    u, _ = _run(u0, [0, 0, 0], B, q, m, tau, steps)
    np.testing.assert_allclose(u, _exact_u(u0, [0, 0, 0], B, q, m, tau * steps), atol=2e-3)


@pytest.mark.parametrize("E,B", [([0.0, 0.4, 0.0], [0.0, 0.0, 1.0]),     # drift along x
                                 ([0.0, 0.3, 0.0], [1.0, 0.0, 0.0]),     # drift along -z
                                 ([0.25, 0.0, 0.2], [0.0, 1.0, 0.0])])   # drift in x-z
def test_e_cross_b_drift(E, B):
    """Started at the drift velocity a Maxwellian stays there; started at rest
    its centre circles about the drift (closed form above)."""
    q, m, tau, steps = 1.0, 1.0, 0.02, 60
    vd = np.cross(E, B) / np.dot(B, B)
    u, _ = _run(vd, E, B, q, m, tau, steps)
    np.testing.assert_allclose(u, vd, atol=1e-3)
    u0 = np.zeros(3)
    u, _ = _run(u0, E, B, q, m, tau, steps)
    np.testing.assert_allclose(u, _exact_u(u0, E, B, q, m, tau * steps), atol=2e-3)


def test_oblique_fields_with_parallel_e():
    q, m, tau, steps = -1.0, 0.8, 0.01, 80
    E = np.array([0.1, -0.2, 0.15])
    B = np.array([0.3, 0.7, -0.4])
    u0 = np.array([0.2, -0.3, 0.5])
    u, _ = _run(u0, E, B, q, m, tau, steps)
    np.testing.assert_allclose(u, _exact_u(u0, E, B, q, m, tau * steps), atol=3e-3)


@pytest.mark.parametrize("E", [[0.5, 0.0, 0.0], [0.0, -0.7, 0.0], [0.0, 0.0, 0.3], [0.2, -0.3, 0.4]])
@pytest.mark.parametrize("q", [1.0, -1.0])
def test_uniform_e_acceleration_is_exact(E, q):
    """B = 0: each sweep shifts every pencil of axis d by (q/m) E_d sigma / dv;
    with the limiter bound lifted the first moment moves by exactly that."""
    m, tau, steps = 1.0, 0.1, 5
    u0 = np.array([0.3, -0.2, 0.1])
    u, mass = _run(u0, E, [0, 0, 0], q, m, tau, steps, T=1.0, f_inf=1e30, n=48, vmax=8.0)
    gain = q / m * np.asarray(E) * tau * steps
    np.testing.assert_allclose(u, u0 + gain, rtol=0, atol=2e-5 * np.abs(gain).max())
    assert mass == pytest.approx(1.0, rel=1e-13)
