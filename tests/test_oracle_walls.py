"""Pins of the oracle's reflecting y walls (Sec. 3.3 boundary: particles are
reflected at the conducting walls), against facts fixed by the geometry of
reflection rather than by the sweep's own formula:

* a particle at cell centre r moving K whole cells reaches r + K, or, past the
  wall at N, the mirrored cell 2N - 1 - r - K of the velocity -v (and likewise
  at the wall at 0): integer shifts move single spikes exactly there;
* a wall is a mirror: where f is the cell average of one smooth function of
  the unfolded coordinate (the -v pencil read backwards past the wall), the
  limiter-free sweep integrates the parabola through three cell averages
  exactly, so cell averages of a quadratic in the unfolded coordinate are
  carried exactly across either wall, also at fractional shifts;
* the 2X3V y-sweep commutes with the reflection y -> -y, v_y -> -v_y;
* composition of unit shifts equals one shift by their sum.

A missing reversal of the mirror pencil or a wrong v_y pairing moves a
spike to the wrong cell and breaks the exact quadratic transport and the
reflection symmetry.
"""
import numpy as np
import pytest

from oracle.pfc import pfc_sweep, pfc_sweep_reflect_pair
from oracle.vlasov import centres, y_sweep_2x3v


def _spike(N, r):
    f = np.full((1, N), 1e-3)
    f[0, r] = 1.0
    return f


@pytest.mark.parametrize("r,K", [(2, 3), (7, 3), (9, 4), (11, 1), (0, 12), (5, 17)])
def test_integer_shift_spike_reflects_at_top_wall(r, K):
    """+v pencil: a spike at r moving K cells lands at r + K or, reflected at
    the wall y = N, at 2N - 1 - (r + K) of the -v pencil (again reflected at
    y = 0 beyond that)."""
    N = 12
    up = _spike(N, r)
    dn = np.full((1, N), 1e-3)
    nu, nd = pfc_sweep_reflect_pair(up, dn, np.array([float(K)]), 1.0)
    p = (r + K) % (2 * N)                       # position on the unfolded (doubled) line
    if p < N:
        assert np.argmax(nu[0]) == p and nu[0, p] == pytest.approx(1.0, abs=1e-14)
        assert nd[0].max() == pytest.approx(1e-3, abs=1e-14)
    else:
        row = 2 * N - 1 - p
        assert np.argmax(nd[0]) == row and nd[0, row] == pytest.approx(1.0, abs=1e-14)
        assert nu[0].max() == pytest.approx(1e-3, abs=1e-14)


@pytest.mark.parametrize("r,K", [(3, 1), (3, 4), (0, 1), (10, 5)])
def test_integer_shift_spike_reflects_at_bottom_wall(r, K):
    """-v pencil (moving down by K): a spike at r lands at r - K or, reflected
    at y = 0, at K - r - 1 of the +v pencil."""
    N = 12
    up = np.full((1, N), 1e-3)
    dn = _spike(N, r)
    nu, nd = pfc_sweep_reflect_pair(up, dn, np.array([float(K)]), 1.0)
    if r - K >= 0:
        assert np.argmax(nd[0]) == r - K
    else:
        assert np.argmax(nu[0]) == K - r - 1 and nu[0, K - r - 1] == pytest.approx(1.0, abs=1e-14)


def _avg_quad(c, lo, hi):
    P = lambda x: c[0] * x + c[1] * x * x / 2 + c[2] * x ** 3 / 3
    return (P(hi) - P(lo)) / (hi - lo)


@pytest.mark.parametrize("wall", ["top", "bottom"])
@pytest.mark.parametrize("s", [0.35, 0.8, 1.6, 2.45])
def test_quadratic_crosses_wall_exactly(wall, s):
    """f_up(r) = avg of q over [r, r+1] and f_dn(r) = avg of q over the mirror
    image of cell r: [2N-1-r, 2N-r] beyond the top wall (unfolded), or
    [-r-1, -r] beyond the bottom wall.  Moving every point by s (up for +v,
    i.e. down for -v), each output cell near the chosen wall is the average of
    q over its source interval."""
    N = 16
    c = np.array([60.0, 0.9, 0.03]) if wall == "top" else np.array([60.0, -0.4, 0.03])
    r = np.arange(N, dtype=float)
    up_lo = r
    dn_lo = (2 * N - 1 - r) if wall == "top" else (-r - 1)
    up = _avg_quad(c, up_lo, up_lo + 1)[None]
    dn = _avg_quad(c, dn_lo, dn_lo + 1)[None]
    nu, nd = pfc_sweep_reflect_pair(up, dn, np.array([s]), 1e30)
    # on the unfolded line the +v cell r is at r, the -v cell r at dn_lo; content moves by +s
    e_up = _avg_quad(c, up_lo - s, up_lo + 1 - s)
    e_dn = _avg_quad(c, dn_lo - s, dn_lo + 1 - s)
    if wall == "top":
        sel = slice(N - 6, N)                   # near the top wall, both pencils
        np.testing.assert_allclose(nu[0, sel], e_up[sel], rtol=1e-13)
        np.testing.assert_allclose(nd[0, sel], e_dn[sel], rtol=1e-13)
    else:
        # the bottom wall sits at unfolded 0: content reaching +v cells 0..5 comes from -v cells
        sel = slice(0, 6)
        np.testing.assert_allclose(nu[0, sel], e_up[sel], rtol=1e-13)
        np.testing.assert_allclose(nd[0, sel], e_dn[sel], rtol=1e-13)


def _vy_grid(nvy, vmax=2.0):
    v, h = centres(-vmax, vmax, nvy)
    return v, h


def _reflect_y(f):
    """y -> -y and v_y -> -v_y on f[ny, nx, nvx, nvy, nvz]."""
    return f[::-1, :, :, ::-1, :]


@pytest.mark.parametrize("nvy", [4, 5])
@pytest.mark.parametrize("bc", ["reflect", "periodic"])
def test_y_sweep_commutes_with_reflection(nvy, bc):
    rng = np.random.default_rng(31)
    f = rng.uniform(0.1, 1.0, size=(9, 3, 2, nvy, 2))
    vy, _ = _vy_grid(nvy)
    for tau in (0.3, 1.7):
        a = y_sweep_2x3v(_reflect_y(f), vy, 1.0, tau, f.max(), bc)
        b = _reflect_y(y_sweep_2x3v(f, vy, 1.0, tau, f.max(), bc))
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-15)


def test_y_sweep_integer_shifts_pair_mirror_velocities():
    """v_y centres -1.5 .. 1.5 and tau/dy = 2: shifts -3, -1, 1, 3 cells.  A
    spike at row r and v_y index j lands at row r + s_j, or past a wall at the
    mirrored row of v_y index nvy - 1 - j."""
    ny = 8
    vy = np.array([-1.5, -0.5, 0.5, 1.5])
    for j in range(4):
        for r in (0, 3, 6, 7):
            f = np.full((ny, 2, 1, 4, 1), 1e-3)
            f[r, :, 0, j, 0] = 1.0
            g = y_sweep_2x3v(f, vy, 1.0, 2.0, 1.0)
            s = int(round(vy[j] * 2.0))
            t = r + s
            if 0 <= t < ny:
                row, jj = t, j
            elif t >= ny:
                row, jj = 2 * ny - 1 - t, 3 - j
            else:
                row, jj = -t - 1, 3 - j
            assert g[row, 0, 0, jj, 0] == pytest.approx(1.0, abs=1e-14), (j, r)
            assert np.isclose(g, 1.0, atol=1e-12).sum() == 2     # the spike, in both columns


@pytest.mark.parametrize("K", [2, 3, 5, 13])
def test_unit_shift_composition(K):
    rng = np.random.default_rng(32)
    N = 10
    f = rng.uniform(0, 1, size=(3, N))
    one = f.copy()
    for _ in range(K):
        one = pfc_sweep(one, np.ones(3), "periodic", f.max())
    np.testing.assert_allclose(pfc_sweep(f, np.full(3, float(K)), "periodic", f.max()), one, rtol=0, atol=1e-14)
    up, dn = rng.uniform(0, 1, size=(2, 3, N))
    a, b = up.copy(), dn.copy()
    for _ in range(K):
        a, b = pfc_sweep_reflect_pair(a, b, np.ones(3), 1.0)
    c, d = pfc_sweep_reflect_pair(up, dn, np.full(3, float(K)), 1.0)
    np.testing.assert_allclose(a, c, rtol=0, atol=1e-14)
    np.testing.assert_allclose(b, d, rtol=0, atol=1e-14)
