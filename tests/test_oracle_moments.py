"""Pins of the oracle's moments, discrete Maxwellian and moment fitting.

* raw moments of a single occupied velocity cell have a closed form;
* the heat-flux identity of Sec. 2.1, Q = Qcal - sym(u(x)P) + 2mnuuu, equals the
  central third moment m int (v-u)(v-u)(v-u) f computed by brute force;
* T from P (Sec. 2.1) equals (m/n) int (v-u)(v-u) f (Sec. 2.2's definition);
* the discrete Maxwellian's density is n exactly and its u, T match the
  parameters within the midpoint rule's aliasing bound for a Gaussian;
* fitting f to its own moments leaves f unchanged (self-fit identity);
* fitting a Maxwellian to new (u, T) yields the new Maxwellian;
* after fitting the density is n_V, f >= 0, clipped cells are counted.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import moments as M
from oracle.vlasov import centres


def _grid(n=12, vmax=5.0):
    v, h = centres(-vmax, vmax, n)
    return [v, v, v], [h, h, h]


def test_single_cell_closed_form():
    v, dv = _grid(6, 3.0)
    f = np.zeros((6, 6, 6))
    f[1, 4, 2] = 2.5
    mom = M.raw_moments_3v(f, v, dv, m=0.7)
    dV = dv[0] ** 3
    w = np.array([v[0][1], v[1][4], v[2][2]])
    assert mom[0] == pytest.approx(2.5 * dV, rel=1e-15)
    np.testing.assert_allclose(mom[1:4], 2.5 * dV * w, rtol=1e-15)
    for k, (a, b) in enumerate(M.PAIRS):
        assert mom[4 + k] == pytest.approx(0.7 * 2.5 * dV * w[a] * w[b], rel=1e-14)
    for k, (a, b, c) in enumerate(M.TRIPLES):
        assert mom[10 + k] == pytest.approx(0.7 * 2.5 * dV * w[a] * w[b] * w[c], rel=1e-14, abs=1e-15)


def test_heat_flux_identity_vs_central_moment():
    rng = np.random.default_rng(5)
    v, dv = _grid(8, 4.0)
    f = rng.uniform(0, 1, size=(8, 8, 8))
    m = 0.3
    mom = M.raw_moments_3v(f, v, dv, m)
    d = M.derived_3v(mom, m)
    dV = dv[0] ** 3
    VX, VY, VZ = np.meshgrid(*v, indexing="ij")
    W = [VX - d["u"][0], VY - d["u"][1], VZ - d["u"][2]]
    for i, j, k in itertools.product(range(3), repeat=3):
        central = m * (f * W[i] * W[j] * W[k]).sum() * dV
        assert d["Q"][i, j, k] == pytest.approx(central, abs=1e-12)
    for i, j in itertools.product(range(3), repeat=2):
        Tc = m / d["n"] * (f * W[i] * W[j]).sum() * dV
        assert d["T"][i, j] == pytest.approx(Tc, rel=1e-12)


def test_1v_identities():
    rng = np.random.default_rng(6)
    v, dv = centres(-5, 5, 40)
    f = rng.uniform(0, 1, size=(3, 40))
    m = 1.7
    d = M.derived_1v(M.raw_moments_1v(f, v, dv, m), m)
    for r in range(3):
        w = v - d["u"][r]
        assert d["T"][r] == pytest.approx(m * (f[r] * w * w).sum() * dv / d["n"][r], rel=1e-12)
        assert d["Q"][r] == pytest.approx(m * (f[r] * w ** 3).sum() * dv, abs=1e-12)


def _aliasing_bound(sigma, h):
    """Relative error bound of midpoint moments of a Gaussian (Poisson summation)."""
    a = 2 * math.pi * sigma / h
    return 4 * (1 + a * a) * math.exp(-2 * math.pi ** 2 * sigma ** 2 / h ** 2)


def test_discrete_maxwellian_moments():
    v, dv = _grid(32, 9.0)                      # box edge > 7 sigma from the centre
    m = 0.5
    n, u = 1.3, np.array([0.4, -0.2, 0.1])
    T = np.array([[0.6, 0.1, 0.0], [0.1, 0.5, 0.05], [0.0, 0.05, 0.7]])
    f = M.maxwellian_3v(n, u, T, m, v, dv)
    d = M.derived_3v(M.raw_moments_3v(f, v, dv, m), m)
    assert d["n"] == pytest.approx(n, rel=1e-14)
    sig = math.sqrt(min(np.linalg.eigvalsh(T)) / m)
    tol = _aliasing_bound(sig, dv[0]) + 1e-9        # + truncation at the box edge (> 6 sigma)
    np.testing.assert_allclose(d["u"], u, atol=tol * 10)
    np.testing.assert_allclose(d["T"], T, atol=tol * 10)
    assert np.abs(d["q"]).max() < 1e-6


def test_self_fit_identity():
    rng = np.random.default_rng(7)
    v, dv = _grid(10, 5.0)
    m = 1.0
    base = M.maxwellian_3v(1.0, np.zeros(3), np.eye(3), m, v, dv)
    f = base * (1 + 0.4 * rng.uniform(-1, 1, size=base.shape))
    mom = M.raw_moments_3v(f, v, dv, m)
    U = mom[:10].copy()
    g, U2, clipped, skipped = M.fit_cell_3v(f, mom, U, m, v, dv)
    assert not skipped and clipped == 0
    np.testing.assert_allclose(g, f, rtol=1e-12, atol=1e-14 * f.max())
    np.testing.assert_allclose(U2, U, rtol=1e-14)


def test_fit_maxwellian_to_new_moments():
    v, dv = _grid(20, 6.0)
    m = 1.0
    T0 = np.eye(3) * 0.8
    f = M.maxwellian_3v(2.0, np.zeros(3), T0, m, v, dv)
    mom = M.raw_moments_3v(f, v, dv, m)
    u1 = np.array([0.3, 0.0, -0.2])
    T1 = np.array([[0.9, 0.1, 0.0], [0.1, 0.7, 0.0], [0.0, 0.0, 0.8]])
    nF = 1.9                                    # fluid density differs: rescaled to n_V
    U = np.concatenate([[nF], nF * u1, [0] * 6])
    P1 = T1 * nF + m * nF * np.outer(u1, u1)
    for k, (a, b) in enumerate(M.PAIRS):
        U[4 + k] = P1[a, b]
    g, U2, clipped, skipped = M.fit_cell_3v(f, mom, U, m, v, dv)
    expect = M.maxwellian_3v(2.0, u1, T1, m, v, dv)
    assert clipped == 0 and not skipped
    np.testing.assert_allclose(g, expect, atol=1e-7 * expect.max())
    assert U2[0] == pytest.approx(mom[0], rel=1e-14)
    np.testing.assert_allclose(U2[1:4] / U2[0], u1, rtol=1e-14)


def test_fit_density_positivity_and_clipping():
    rng = np.random.default_rng(8)
    v, dv = _grid(8, 4.0)
    m = 1.0
    f = rng.uniform(0, 1, size=(8, 8, 8)) ** 4
    mom = M.raw_moments_3v(f, v, dv, m)
    U = mom[:10].copy()
    U[1] += 0.8 * U[0]                          # push the fluid velocity far away
    U[4] += 0.8 * U[0] * 2                      # keep T_F positive definite
    g, _, clipped, skipped = M.fit_cell_3v(f, mom, U, m, v, dv)
    assert not skipped and clipped > 0
    assert (g >= 0).all()
    assert g.sum() * dv[0] ** 3 == pytest.approx(mom[0], rel=1e-14)


def test_fit_skips_non_spd():
    v, dv = _grid(6, 3.0)
    f = np.zeros((6, 6, 6))
    f[2, 2, 2] = 1.0                            # one cell: T_V = 0, not positive definite
    mom = M.raw_moments_3v(f, v, dv, 1.0)
    U = np.array([1.0, 0, 0, 0, 1, 0, 0, 1, 0, 1.0])
    g, U2, clipped, skipped = M.fit_cell_3v(f, mom, U, 1.0, v, dv)
    assert skipped and clipped == 0
    np.testing.assert_array_equal(g, f)
    np.testing.assert_array_equal(U2, U)


def test_fit_1v_self_identity_and_new_maxwellian():
    v, dv = centres(-6, 6, 48)
    m = 1.0
    f = M.maxwellian_1v(1.0, 0.2, 1.1, m, v, dv) * (1 + 0.1 * np.sin(3 * v))
    mom = M.raw_moments_1v(f, v, dv, m)
    g, U2, c, s = M.fit_cell_1v(f, mom, mom[:3].copy(), m, v, dv)
    np.testing.assert_allclose(g, f, rtol=1e-12, atol=1e-15)
    h = M.maxwellian_1v(1.0, 0.0, 1.0, m, v, dv)
    mh = M.raw_moments_1v(h, v, dv, m)
    U = np.array([1.0, 0.5, 1.2 + 0.25])        # u = 0.5, T = 1.2
    g, U2, c, s = M.fit_cell_1v(h, mh, U, m, v, dv)
    # tolerance: the v-box truncates both Maxwellians at 6 v_t (e^-18 ~ 1.5e-8)
    np.testing.assert_allclose(g, M.maxwellian_1v(mh[0], 0.5, 1.2, m, v, dv), atol=3e-8)
