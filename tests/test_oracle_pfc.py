"""Pins of the oracle's 1-D PFC sweep against facts fixed by the scheme and by
mathematics (not by re-typing its formula):

* integer shifts are cyclic shifts (the foot lands on a face), up to the
  round-off of the flux sums;
* shift 0 is the identity;
* mass is conserved to round-off (flux form telescopes), for every boundary;
* 0 <= f' <= f_inf on random non-negative and step data (the PFC
  limiter's positivity and maximum principle);
* with the limiter inactive the sweep integrates the parabola through three
  cell averages exactly, so cell averages of any quadratic are advected
  exactly (checked against analytic cell averages of the shifted quadratic);
* third-order convergence on smooth periodic data;
* a v-symmetric, y-uniform state is steady between reflecting walls.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle.pfc import pfc_sweep, pfc_sweep_reflect_pair


def test_integer_shift_is_exact_roll():
    rng = np.random.default_rng(1)
    f = rng.uniform(0, 1, size=(7, 24))
    s = np.array([0, 1, 2, 5, -1, -3, 23], dtype=float)
    out = pfc_sweep(f, s, "periodic", f.max())
    for p in range(7):
        # the flux form sums K cells then differences neighbouring faces:
        # exact up to the round-off of those sums
        np.testing.assert_allclose(out[p], np.roll(f[p], int(s[p])), rtol=0, atol=1e-15 * (1 + abs(s[p])))


def test_zero_shift_identity_zeroflux():
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 1, size=(5, 16))
    np.testing.assert_array_equal(pfc_sweep(f, np.zeros(5), "zeroflux", f.max()), f)


def test_integer_shift_zeroflux_piles_at_wall():
    f = np.arange(1.0, 9.0)[None, :]
    out = pfc_sweep(f, np.array([3.0]), "zeroflux", f.max())[0]
    # cells shift up by 3; the three cells that reach the top wall stay in the last cell
    np.testing.assert_array_equal(out, [0, 0, 0, 1, 2, 3, 4, 5 + 6 + 7 + 8])


@pytest.mark.parametrize("bc", ["periodic", "zeroflux"])
def test_mass_conservation(bc):
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, size=(64, 32))
    s = rng.uniform(-7.5, 7.5, size=64)
    out = pfc_sweep(f, s, bc, f.max())
    np.testing.assert_allclose(out.sum(1), f.sum(1), rtol=1e-14, atol=0)


def test_reflect_pair_mass_and_steady_state():
    rng = np.random.default_rng(4)
    up, dn = rng.uniform(0, 1, size=(2, 10, 12))
    s = rng.uniform(-3, 3, size=10)
    nu, nd = pfc_sweep_reflect_pair(up, dn, s, max(up.max(), dn.max()))
    np.testing.assert_allclose(nu.sum(1) + nd.sum(1), up.sum(1) + dn.sum(1), rtol=1e-14)
    # uniform in y and equal at +v and -v: reflection keeps it steady
    c = rng.uniform(0.5, 1, size=(10, 1)) * np.ones((10, 12))
    nu, nd = pfc_sweep_reflect_pair(c, c, s, c.max())
    np.testing.assert_allclose(nu, c, rtol=1e-14)
    np.testing.assert_allclose(nd, c, rtol=1e-14)


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 2 ** 31 - 1), s=st.floats(-9.9, 9.9), kind=st.sampled_from(["rough", "step", "spiky"]),
       bc=st.sampled_from(["periodic", "zeroflux"]))
def test_positivity_and_max_principle(seed, s, kind, bc):
    rng = np.random.default_rng(seed)
    n = 20
    if kind == "rough":
        f = rng.uniform(0, 1, size=(3, n))
    elif kind == "step":
        f = (rng.uniform(size=(3, n)) > 0.5) * 1.0
    else:
        f = rng.uniform(0, 1, size=(3, n)) ** 8
    f_inf = f.max()
    out = pfc_sweep(f, np.full(3, s), bc, f_inf)
    assert (out >= 0).all()
    if bc == "periodic":
        assert (out <= f_inf * (1 + 1e-14)).all()


def _avg_quadratic(c, lo, hi):
    """Exact cell average of c0 + c1 x + c2 x^2 over [lo, hi]."""
    P = lambda x: c[0] * x + c[1] * x * x / 2 + c[2] * x ** 3 / 3
    return (P(hi) - P(lo)) / (hi - lo)


@pytest.mark.parametrize("s", [0.3, 0.77, 1.5, 2.25, -0.4, -1.9])
def test_quadratic_advected_exactly(s):
    n = 24
    edges = np.arange(n + 1, dtype=float)
    c = np.array([40.0, 1.3, 0.05])                 # positive, gentle: limiter inactive
    f = _avg_quadratic(c, edges[:-1], edges[1:])[None, :]
    out = pfc_sweep(f, np.array([s]), "zeroflux", 1e30)[0]
    expect = _avg_quadratic(c, edges[:-1] - s, edges[1:] - s)
    inner = slice(int(np.ceil(abs(s))) + 3, n - int(np.ceil(abs(s))) - 3)
    np.testing.assert_allclose(out[inner], expect[inner], rtol=1e-13)


def test_limiter_clips_parabola_overshoot():
    # a lone spike: the unlimited parabola would go negative next to it
    f = np.zeros((1, 12))
    f[0, 5] = 1.0
    out = pfc_sweep(f, np.array([0.5]), "periodic", 1.0)
    assert (out >= 0).all() and out.max() <= 1.0
    np.testing.assert_allclose(out.sum(), 1.0, rtol=1e-15)


def _sine_avgs(n, shift):
    h = 1.0 / n
    lo = np.arange(n) * h - shift
    hi = lo + h
    # average of 1 + 0.5 sin(2 pi x)
    return 1.0 + 0.5 * (np.cos(2 * np.pi * lo) - np.cos(2 * np.pi * hi)) / (2 * np.pi * h)


@pytest.mark.parametrize("f_inf_mode", ["unbounded", "max"])
def test_third_order_convergence(f_inf_mode):
    """Unbounded: third order in the max norm.  With f_inf = running maximum
    the max-principle limiter flattens the crest each step, which costs order
    at the extremum only: L1 error still falls by > 4 per halving."""
    errs, errs1 = [], []
    for n in (32, 64, 128):
        f = _sine_avgs(n, 0.0)[None, :]
        s = 0.37
        steps = int(round(0.5 / (s / n)))          # move ~half a period
        for _ in range(steps):
            bound = 1e30 if f_inf_mode == "unbounded" else f.max()
            f = pfc_sweep(f, np.array([s]), "periodic", bound)
        exact = _sine_avgs(n, steps * s / n)
        errs.append(np.abs(f[0] - exact).max())
        errs1.append(np.abs(f[0] - exact).mean())
    if f_inf_mode == "unbounded":
        r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
        assert r1 > 6.5 and r2 > 7.0, errs
    else:
        r1, r2 = errs1[0] / errs1[1], errs1[1] / errs1[2]
        assert r1 > 4.0 and r2 > 4.0, errs1
