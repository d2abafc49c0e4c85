"""Pins of the learned-closure oracle (oracle/mlp.py) against closed forms,
finite differences and reductions to library routines."""
import math
import sys
import os

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import mlp as OM  # noqa: E402
from oracle import moments as OMo  # noqa: E402
from paper_2109_06743_amd import workloads as W  # noqa: E402


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=scale, size=OM.N_PARAM)
    d = OM.unpack(p)
    d["W4"][10:] = 0.0
    d["b4"][10:] = 0.0
    return OM.pack(d)


def test_layout_and_size():
    assert OM.N_PARAM == 3 * (64 * 64 + 64) + 16 * 64 + 16 == 13520
    p = np.arange(OM.N_PARAM, dtype=np.float64)
    assert np.array_equal(OM.pack(OM.unpack(p)), p)
    assert OM.unpack(p)["W2"][1, 0] == 4096 + 64 + 64     # row-major [out][in]


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _rand_params(2)
    x = rng.normal(size=(7, 64))
    t = np.zeros((7, 16))
    t[:, :10] = rng.normal(size=(7, 10))
    L0, g = OM.gradient(p, x, t, exact_weights=True)
    idx = []
    for name, off, shape in OM._LAYOUT:
        size = int(np.prod(shape))
        idx += list(off + rng.choice(size, size=min(size, 12), replace=False))
    h = 1e-5
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (OM.loss(OM.forward(pp, x, True)[0], t) - OM.loss(OM.forward(pm, x, True)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_padding_outputs_get_no_gradient():
    rng = np.random.default_rng(3)
    p = _rand_params(4)
    x = rng.normal(size=(5, 64))
    t = np.zeros((5, 16))
    t[:, :10] = 1.0
    t[:, 10:] = 123.0                                     # ignored
    _, g = OM.gradient(p, x, t, exact_weights=True)
    d = OM.unpack(g)
    assert np.all(d["W4"][10:] == 0) and np.all(d["b4"][10:] == 0)


def test_small_weights_reduce_to_matrix_product():
    """tanh(a) = a + O(a^3): with weights of size eps the network is the
    product of its affine maps up to O(eps^3)."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=(4, 64))
    for eps in (1e-2, 5e-3):
        p = _rand_params(6, scale=eps)
        d = OM.unpack(p)
        lin = (((x @ d["W1"].T + d["b1"]) @ d["W2"].T + d["b2"]) @ d["W3"].T + d["b3"]) @ d["W4"].T + d["b4"]
        y, _ = OM.forward(p, x, exact_weights=True)
        err = np.abs(y - lin).max()
        assert err < 50 * eps ** 3, (eps, err)
        assert np.abs(lin).max() > 10 * err


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e-3], dtype=np.float32)
    r = OM.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                                    # tie at 1 + 2^-8 rounds to even (1.0)
    assert r[2] == 1.0 + 2 ** -6                          # tie rounds to even mantissa
    assert r[3] == 1.0
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    bits = OM.bf16_bits(np.array([1.0, -2.0], dtype=np.float32))
    assert bits[0] == 0x3F80 and bits[1] == 0xC000


def test_adam_closed_forms():
    """Constant gradient: every bias-corrected step moves by lr g/(|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    p = np.zeros(3)
    m1 = np.zeros(3)
    m2 = np.zeros(3)
    lr = 0.01
    for k in range(1, 6):
        p_new, m1, m2 = OM.adam_step(p, g, m1, m2, k, lr)
        np.testing.assert_allclose(p_new - p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
        p = p_new
    # a zero gradient after one step: m1 = 0.1 g * 0.9, m2 = 0.001 g^2 * 0.999
    p0 = np.zeros(3)
    _, m1, m2 = OM.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, lr)
    p2, _, _ = OM.adam_step(p0, np.zeros(3), m1, m2, 2, lr)
    mh = 0.9 * 0.1 * g / (1 - 0.81)
    vh = 0.999 * 0.001 * g * g / (1 - 0.999 ** 2)
    np.testing.assert_allclose(p2, -lr * mh / (np.sqrt(vh) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(256, 64)) * 0.5
    A = rng.normal(size=(10, 64)) * 0.1
    t = np.zeros((256, 16))
    t[:, :10] = np.tanh(x @ A.T)
    p = W.mlp_init(0).astype(np.float64)
    m1 = np.zeros_like(p)
    m2 = np.zeros_like(p)
    L0 = OM.gradient(p, x, t, exact_weights=True)[0]
    for k in range(1, 151):
        L, g = OM.gradient(p, x, t, exact_weights=True)
        p, m1, m2 = OM.adam_step(p, g, m1, m2, k, 3e-3)
    assert L < 0.1 * L0, (L0, L)


# ---------------------------------------------------------------- features --
def _state(ny, nx, m, fn):
    """U (n, nu, P) of a cold-free state n(x,y), u(x,y), T(x,y) given by fn."""
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    n, u, T = fn(x, y)
    U = np.empty((ny, nx, 10))
    U[..., 0] = n
    U[..., 1:4] = n[..., None] * u
    for k, (a, b) in enumerate(OMo.PAIRS):
        U[..., 4 + k] = n * T[..., a, b] + m * n * u[..., a] * u[..., b]
    return U


def _iso(T0, shape):
    T = np.zeros(shape + (3, 3))
    for a in range(3):
        T[..., a, a] = T0
    return T


def test_features_of_uniform_state():
    m = 0.04
    u0 = np.array([0.3, -0.1, 0.2])
    Tm = np.array([[1.0, 0.1, 0.0], [0.1, 0.8, 0.05], [0.0, 0.05, 1.2]])

    def fn(x, y):
        return np.full(x.shape, 2.0), np.broadcast_to(u0, x.shape + (3,)), np.broadcast_to(Tm, x.shape + (3, 3))
    U = _state(4, 5, m, fn)
    # u_y != 0 and T_xy, T_yz != 0 are odd under the wall mirror, so only
    # rows away from the walls see a uniform stencil
    x, scale = OM.features(U, m, species=1)
    x = x.reshape(4, 5, 64)
    Tref = np.trace(Tm) / 3
    vt = math.sqrt(Tref / m)
    np.testing.assert_allclose(x[..., 0:3], np.broadcast_to(u0 / vt, (4, 5, 3)), rtol=1e-13)
    np.testing.assert_allclose(x[..., 3:9], np.broadcast_to([Tm[a, b] / Tref for a, b in OMo.PAIRS], (4, 5, 6)),
                               rtol=1e-13)
    np.testing.assert_allclose(x[1:-1, :, 9:59], 0.0, atol=1e-13)
    assert np.all(x[..., 60] == 1.0) and np.all(x[..., 59] == 0.0) and np.all(x[..., 61:] == 0.0)
    np.testing.assert_allclose(scale, 2.0 * m * vt ** 3, rtol=1e-13)


def test_features_finite_differences_closed_form():
    """n = 1 + e cos(k x) (grid units): d_x = -e sin(kx) sin(k), d_xx =
    2 e cos(kx)(cos k - 1), divided by the centre density."""
    m, e, nx = 1.0, 0.1, 16
    k = 2 * math.pi / nx

    def fn(x, y):
        return 1.0 + e * np.cos(k * x), np.zeros(x.shape + (3,)), _iso(0.5, x.shape)
    U = _state(3, nx, m, fn)
    x, _ = OM.features(U, m, 0)
    x = x.reshape(3, nx, 64)
    xi = np.arange(nx)
    nc = 1.0 + e * np.cos(k * xi)
    np.testing.assert_allclose(x[1, :, 9], -e * np.sin(k * xi) * math.sin(k) / nc, atol=1e-14)
    np.testing.assert_allclose(x[1, :, 11], 2 * e * np.cos(k * xi) * (math.cos(k) - 1) / nc, atol=1e-14)
    np.testing.assert_allclose(x[..., 10], 0.0, atol=1e-14)    # d_y
    np.testing.assert_allclose(x[..., 13], 0.0, atol=1e-14)    # d_xy
    # T field: phi_4 = T_xx / T_ref_c is constant -> all its differences vanish
    np.testing.assert_allclose(x[..., 9 + 5 * 4: 9 + 5 * 5], 0.0, atol=1e-14)


def test_features_cross_difference_closed_form():
    """n = 1 + e sin(kx i) sin(ky j): d_xy = e cos(kx i) sin(kx) cos(ky j) sin(ky)
    and d_yy = 2 e sin(kx i) sin(ky j)(cos ky - 1), over the centre density
    (rows away from the walls)."""
    m, e, nx, ny = 1.0, 0.1, 12, 10
    kx, ky = 2 * math.pi / nx, 0.37

    def fn(x, y):
        return 1.0 + e * np.sin(kx * x) * np.sin(ky * y), np.zeros(x.shape + (3,)), _iso(0.5, x.shape)
    U = _state(ny, nx, m, fn)
    x, _ = OM.features(U, m, 0)
    x = x.reshape(ny, nx, 64)
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    nc = 1.0 + e * np.sin(kx * I) * np.sin(ky * J)
    dxy = e * np.cos(kx * I) * math.sin(kx) * np.cos(ky * J) * math.sin(ky) / nc
    dyy = 2 * e * np.sin(kx * I) * np.sin(ky * J) * (math.cos(ky) - 1) / nc
    np.testing.assert_allclose(x[1:-1, :, 13], dxy[1:-1], atol=1e-14)
    np.testing.assert_allclose(x[1:-1, :, 12], dyy[1:-1], atol=1e-14)


def test_features_mirror_parity():
    """A state symmetric under y -> -y (n, T_xx even; u_y, T_xy odd) gives
    features at row j equal to those at the mirrored row up to the sign of
    every y-odd quantity: d_y and d_xy flip for even fields, and the other
    three flip for odd fields."""
    m, ny, nx = 0.5, 6, 7
    yc = lambda y: (y + 0.5) - ny / 2.0

    def fn(x, y):
        Y = yc(y)
        n = 1.0 + 0.2 * np.cos(0.5 * Y) * (1 + 0.1 * np.sin(0.9 * x))
        u = np.stack([0.1 * np.cos(0.3 * Y + 0 * x), 0.2 * np.sin(0.4 * Y) * (1 + 0.1 * np.cos(0.9 * x)),
                      0.05 + 0 * x], axis=-1)
        T = _iso(0.7 + 0.1 * np.cos(0.6 * Y), x.shape)
        T[..., 0, 1] = T[..., 1, 0] = 0.05 * np.sin(0.7 * Y)
        T[..., 1, 2] = T[..., 2, 1] = 0.03 * np.sin(0.2 * Y) * np.cos(0.9 * x)
        return n, u, T
    U = _state(ny, nx, m, fn)
    x, _ = OM.features(U, m, 0)
    x = x.reshape(ny, nx, 64)
    odd_field = np.array([False, False, True, False, False, True, False, False, True, False])   # n, u(3), T6
    sign = np.ones(64)
    sign[1] = -1                                   # u_y
    sign[3 + 1] = sign[3 + 4] = -1                 # T_xy, T_yz
    for k in range(10):
        for d in range(5):
            y_odd_deriv = d in (1, 4)
            sign[9 + 5 * k + d] = -1 if (y_odd_deriv != odd_field[k]) else 1
    for j in range(ny):
        np.testing.assert_allclose(x[j], sign * x[ny - 1 - j], atol=1e-13)


def test_targets_of_two_cells():
    """All mass in two velocity cells: Q_xxx = m sum n_k (v_k - u)^3 (closed
    form); components with a y or z index vanish."""
    m = 2.0
    nv = 6
    v = [np.linspace(-2.5, 2.5, nv)] * 3
    dv = [1.0] * 3
    f = np.zeros((1, 1, nv, nv, nv))
    f[0, 0, 1, 3, 2] = 0.7
    f[0, 0, 4, 3, 2] = 0.2
    mom = OMo.raw_moments_3v(f, v, dv, m)
    n = 0.9
    u = (0.7 * v[0][1] + 0.2 * v[0][4]) / n
    Qxxx = m * (0.7 * (v[0][1] - u) ** 3 + 0.2 * (v[0][4] - u) ** 3)
    Q = OM.heat_flux(mom, m)[0, 0]
    assert abs(Q[0] - Qxxx) < 1e-13
    np.testing.assert_allclose(Q[1:], 0.0, atol=1e-13)
    T = m * (0.7 * (v[0][1] - u) ** 2 + 0.2 * (v[0][4] - u) ** 2) / n / 3.0   # tr(T)/3: only T_xx
    vt = math.sqrt(T / m)
    y = OM.targets(mom, m)
    assert abs(y[0, 0] - Qxxx / (n * m * vt ** 3)) < 1e-12


def test_targets_of_maxwellian_vanish():
    m = 0.04
    nv = 32
    vmax = 12.5
    h = 2 * vmax / nv
    v = [np.linspace(-vmax + h / 2, vmax - h / 2, nv)] * 3
    dv = [h] * 3
    T = np.diag([0.09, 0.07, 0.08])
    f = OMo.maxwellian_3v(1.3, np.array([0.3, -0.2, 0.1]), T, m, v, dv)
    mom = OMo.raw_moments_3v(f[None, None], v, dv, m)
    y = OM.targets(mom, m)
    assert np.abs(y[0, :10]).max() < 1e-6


def test_qcal_round_trip():
    rng = np.random.default_rng(9)
    m = 0.3
    f = rng.uniform(0.1, 1.0, size=(2, 3, 6, 6, 6))
    v = [np.linspace(-2, 2, 6)] * 3
    dv = [0.8] * 3
    mom = OMo.raw_moments_3v(f, v, dv, m)
    Q = OM.heat_flux(mom, m)
    scale = np.full(mom.shape[:-1], 1.7)
    Qc = OM.qcal_from_closure(mom[..., :10], Q / 1.7, scale, m)
    np.testing.assert_allclose(Qc, mom[..., 10:], rtol=1e-12, atol=1e-12)


def test_divergence_of_heat_flux_closed_form():
    nx, ny = 16, 4
    dx, dy = 0.3, 0.5
    k = 2 * math.pi / (nx * dx)
    xs = (np.arange(nx) + 0.5) * dx
    Q = np.zeros((ny, nx, 10))
    Q[..., 0] = np.sin(k * xs)                          # Q_xxx
    Q[..., 3] = 2.0 * np.sin(k * xs)                    # Q_xyy
    d = OM.divergence_heat_flux(Q, dx, dy)
    fac = math.sin(k * dx) / dx
    np.testing.assert_allclose(d[..., 0], fac * np.cos(k * xs) * np.ones((ny, 1)), atol=1e-13)   # xx
    np.testing.assert_allclose(d[..., 3], 2 * fac * np.cos(k * xs) * np.ones((ny, 1)), atol=1e-13)  # yy
    np.testing.assert_allclose(d[..., [1, 2, 4, 5]], 0.0, atol=1e-13)


def test_gradient_closure_closed_form():
    """Eq. 5 on T = T0 (1 + e cos kx), n = 1: div Q_ii = -chi d_s v_t lap T with
    the discrete Laplacian T0 e (2 cos(k dx) - 2)/dx^2 cos(kx)."""
    m, q = 0.04, -1.0
    nx, ny, dx, dy = 32, 3, 0.2, 0.4
    k = 2 * math.pi / (nx * dx)
    T0, e = 0.5, 0.05

    def fn(x, y):
        return np.ones(x.shape), np.zeros(x.shape + (3,)), _iso(T0 * (1 + e * np.cos(k * (x + 0.5) * dx)), x.shape)
    U = _state(ny, nx, m, fn)
    d = OM.gradient_closure_divergence(U, m, q, dx, dy)
    xs = (np.arange(nx) + 0.5) * dx
    T = T0 * (1 + e * np.cos(k * xs))
    vt = np.sqrt(T / m)
    lap = T0 * e * (2 * math.cos(k * dx) - 2) / dx ** 2 * np.cos(k * xs)
    d_s = math.sqrt(m)
    for c in (0, 3, 5):
        np.testing.assert_allclose(d[1, :, c], -OM.CHI * d_s * vt * lap, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(d[..., [1, 2, 4]], 0.0, atol=1e-14)


def test_field_direction_features():
    m = 1.0

    def fn(x, y):
        return np.full(x.shape, 1.5), np.zeros(x.shape + (3,)), _iso(0.3, x.shape)
    U = _state(3, 4, m, fn)
    B = np.zeros((3, 4, 3))
    B[..., 0] = 3.0
    B[..., 2] = -4.0
    B[1, 2] = 0.0                                   # no field in one cell
    x0, _ = OM.features(U, m, 1)
    x1, _ = OM.features(U, m, 1, B)
    x0, x1 = x0.reshape(3, 4, 64), x1.reshape(3, 4, 64)
    np.testing.assert_array_equal(x0[..., :61], x1[..., :61])
    np.testing.assert_allclose(x1[0, 0, 61:], [0.6, 0.0, -0.8], rtol=1e-15)
    np.testing.assert_array_equal(x1[1, 2, 61:], 0.0)
    np.testing.assert_array_equal(x0[..., 61:], 0.0)


def test_judge_error_contracts_the_full_tensor(monkeypatch):
    """The judge compares heat-flux vectors q_i = sum_j Q_ijj of the network's
    and the kinetic third moments.  Both tensors are drawn as full symmetric
    3x3x3 arrays, packed in the documented order (xxx, xxy, xxz, xyy, xyz,
    xzz, yyy, yyz, yzz, zzz) and handed to the judge in place of the network
    and the kinetic heat flux; its value must be the relative L2 norm of the
    difference of the two contractions taken with einsum on the full tensors."""
    import itertools
    rng = np.random.default_rng(17)
    ny, nx = 3, 4

    def sym(shape):
        t = rng.normal(size=shape + (3, 3, 3))
        return sum(np.transpose(t, (0, 1) + tuple(2 + p for p in perm))
                   for perm in itertools.permutations(range(3))) / 6.0

    order = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
             (2, 2, 2)]
    pack = lambda T: np.stack([T[..., a, b, c] for a, b, c in order], axis=-1)
    Tn, Tk = sym((ny, nx)), sym((ny, nx))
    scale = rng.uniform(0.5, 2.0, size=(ny, nx))
    y = np.zeros((ny, nx, OM.N_OUT_PAD))
    y[..., :OM.N_OUT] = pack(Tn) / scale[..., None]
    monkeypatch.setattr(OM, "network_heat_flux", lambda U, m, s, p, B=None: (y, scale))
    monkeypatch.setattr(OM, "heat_flux", lambda mom, m: pack(Tk))
    got = OM.judge_error(np.zeros((ny, nx, 20)), 1.0, 0, None)
    qn, qk = np.einsum("...ijj->...i", Tn), np.einsum("...ijj->...i", Tk)
    assert got == pytest.approx(np.linalg.norm(qn - qk) / np.linalg.norm(qk), rel=1e-12)
    # and zero for the same tensor
    monkeypatch.setattr(OM, "heat_flux", lambda mom, m: pack(Tn))
    assert OM.judge_error(np.zeros((ny, nx, 20)), 1.0, 0, None) < 1e-14
