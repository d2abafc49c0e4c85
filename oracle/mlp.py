"""Learned heat-flux closure for the ten-moment fluid update, FP64 CPU oracle.
Test infrastructure only.

The paper closes the fluid equations either with the kinetic third moment (the
moment-fitting method, Sec. 2.2) or, for fluid-only runs, with the
temperature-gradient closure of Eq. 5 (Sec. 2.3):
    div Q_s = -(chi / k_{s,0}) n_s v_{t,s} lap T_s,  chi = 2 sqrt(2/pi),
    k_{s,0} = 1/d_s,  v_{t,s} = sqrt(tr(T_s)/(3 m_s)).
Here a small network predicts the heat-flux tensor Q (Sec. 2.1 definition)
from local moments and their 3x3-stencil differences; the kinetic Q computed
from f is both its training target and the judge of its error.  Nothing of
the network is in the paper; every choice below is a reading:

* Sample: one spatial cell of one species, described by its ten moments
  (n, nu, P), i.e. the first ten raw moments.
* Features (64, in this order), computed in FP64 then rounded to FP32 and
  then to BF16 (round to nearest even at each step):
    0-2    u / v_t                 (v_t = sqrt(T_ref/m), T_ref = tr(T)/3)
    3-8    T / T_ref               (xx, xy, xz, yy, yz, zz)
    9-58   for each of ten stencil fields phi_k (k = 0..9):
           [d_x, d_y, d_xx, d_yy, d_xy] in grid units (central differences on
           the 3x3 stencil), with phi_0 = n / n_c, phi_1..3 = u / v_t,c and
           phi_4..9 = T / T_ref,c (the centre cell's scales for every
           neighbour); x periodic, y mirrored at the walls with the sign of
           u_y, T_xy, T_yz flipped (reflection symmetry of the particles).
    59-60  species one-hot (0: first species, 1: second)
    61-63  direction B/|B| of the cell-centred magnetic field (0 where |B| <=
           1e-12 or no field is given): the paper observes that the heat
           flux follows B, which the temperature-gradient closure cannot see
           (Sec. 4.1 discussion).
  A cell with n <= 1e-12 or tr(T) <= 0 gets all-zero features and scale 0.
* Target: the heat-flux tensor normalised by n m v_t^3, ten components in
  the order of oracle.moments.TRIPLES, padded to 16 outputs with zeros.
* Network: y = W4 h3 + b4, h_l = tanh(W_l h_{l-1} + b_l) for l = 1..3,
  h_0 = features; widths 64-64-64-64-16.  Parameters are one FP32 vector
  W1[64][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[16][64] b4[16]
  (13520 values, row-major [out][in]); the network evaluates the BF16-rounded
  weights (biases stay FP32).  This oracle evaluates that network exactly in
  FP64 on the BF16-rounded weights and features.
* Loss: mean over samples and the ten valid outputs of the squared error.
* Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master
  parameters with bias correction.
"""
import math

import numpy as np

from .moments import PAIRS, TRIPLES, derived_3v

N_IN = 64
WIDTH = 64
N_OUT = 10
N_OUT_PAD = 16
CHI = 2.0 * math.sqrt(2.0 / math.pi)

# parameter vector layout: (name, offset, shape)
_LAYOUT = []
_off = 0
for _name, _shape in (("W1", (WIDTH, N_IN)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
                      ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (N_OUT_PAD, WIDTH)), ("b4", (N_OUT_PAD,))):
    _LAYOUT.append((_name, _off, _shape))
    _off += int(np.prod(_shape))
N_PARAM = _off


def unpack(params):
    """FP32/FP64 parameter vector -> dict of arrays (views)."""
    p = np.asarray(params)
    return {name: p[off:off + int(np.prod(shape))].reshape(shape) for name, off, shape in _LAYOUT}


def pack(d):
    out = np.zeros(N_PARAM)
    for name, off, shape in _LAYOUT:
        out[off:off + int(np.prod(shape))] = np.asarray(d[name], dtype=np.float64).ravel()
    return out


# ---------------------------------------------------------------- rounding --
def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_round(x):
    """FP32 -> BF16 (round to nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """FP32 -> BF16 bit patterns (uint16), same rounding as bf16_round."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


# ---------------------------------------------------------------- features --
def _local(U, m):
    """U[..., >=10] = (n, nu, P) -> n, u[...,3], T6[...,6] (xx,xy,xz,yy,yz,zz)."""
    n = U[..., 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = U[..., 1:4] / n[..., None]
        T6 = np.stack([(U[..., 4 + k] - m * n * u[..., a] * u[..., b]) / n for k, (a, b) in enumerate(PAIRS)],
                      axis=-1)
    return n, u, T6


def _y_parity_uT():
    """Sign of (u_x, u_y, u_z) and T6 under y -> -y."""
    pu = np.array([1.0, -1.0, 1.0])
    pT = np.array([(-1.0) ** ((a == 1) + (b == 1)) for a, b in PAIRS])
    return pu, pT


def features(U, m, species, B=None):
    """U[ny, nx, >=10], B[ny, nx, 3] or None -> (x[ny*nx, 64] FP64 before
    rounding, scale[ny*nx])."""
    U = np.asarray(U, dtype=np.float64)
    ny, nx = U.shape[:2]
    n, u, T6 = _local(U, m)
    Tref = (T6[..., 0] + T6[..., 3] + T6[..., 5]) / 3.0
    ok = (n > 1e-12) & (Tref > 0)
    vt = np.sqrt(np.where(ok, Tref, 1.0) / m)
    pu, pT = _y_parity_uT()

    def nb(dj, di):
        """Neighbour (j+dj, i+di) values of n, u, T6 with the wall mirror."""
        j = np.arange(ny)[:, None] + dj
        i = (np.arange(nx)[None, :] + di) % nx
        mir = (j < 0) | (j >= ny)
        jj = np.where(j < 0, -1 - j, np.where(j >= ny, 2 * ny - 1 - j, j))
        jj = np.broadcast_to(jj, (ny, nx))
        ii = np.broadcast_to(i, (ny, nx))
        mir = np.broadcast_to(mir, (ny, nx))
        nn = n[jj, ii]
        uu = np.where(mir[..., None], u[jj, ii] * pu, u[jj, ii])
        TT = np.where(mir[..., None], T6[jj, ii] * pT, T6[jj, ii])
        return nn, uu, TT

    def fields_at(dj, di):
        nn, uu, TT = nb(dj, di)
        phi = np.empty((ny, nx, 10))
        with np.errstate(divide="ignore", invalid="ignore"):
            phi[..., 0] = nn / n
            phi[..., 1:4] = uu / vt[..., None]
            phi[..., 4:10] = TT / np.where(ok, Tref, 1.0)[..., None]
        return phi

    P = {(dj, di): fields_at(dj, di) for dj in (-1, 0, 1) for di in (-1, 0, 1)}
    d_x = (P[(0, 1)] - P[(0, -1)]) / 2.0
    d_y = (P[(1, 0)] - P[(-1, 0)]) / 2.0
    d_xx = P[(0, 1)] - 2.0 * P[(0, 0)] + P[(0, -1)]
    d_yy = P[(1, 0)] - 2.0 * P[(0, 0)] + P[(-1, 0)]
    d_xy = (P[(1, 1)] - P[(-1, 1)] - P[(1, -1)] + P[(-1, -1)]) / 4.0
    x = np.zeros((ny, nx, N_IN))
    with np.errstate(divide="ignore", invalid="ignore"):
        x[..., 0:3] = u / vt[..., None]
        x[..., 3:9] = T6 / np.where(ok, Tref, 1.0)[..., None]
    for k in range(10):
        for d, arr in enumerate((d_x, d_y, d_xx, d_yy, d_xy)):
            x[..., 9 + 5 * k + d] = arr[..., k]
    x[..., 59 + species] = 1.0
    if B is not None:
        B = np.asarray(B, dtype=np.float64).reshape(ny, nx, 3)
        bn = np.sqrt((B * B).sum(-1))
        with np.errstate(divide="ignore", invalid="ignore"):
            x[..., 61:64] = np.where((bn > 1e-12)[..., None], B / bn[..., None], 0.0)
    x = np.where(ok[..., None], x, 0.0)
    scale = np.where(ok, n * m * vt ** 3, 0.0)
    return x.reshape(ny * nx, N_IN), scale.reshape(ny * nx)


def features_bf16(U, m, species, B=None):
    """Features as the network sees them: FP64 -> FP32 -> BF16."""
    x, scale = features(U, m, species, B)
    return bf16_round(to_f32(x)), scale


def heat_flux(mom, m):
    """Raw moments [..., 20] -> heat-flux tensor Q [..., 10] (TRIPLES order)."""
    Q = derived_3v(mom, m)["Q"]
    return np.stack([Q[..., a, b, c] for a, b, c in TRIPLES], axis=-1)


def targets(mom, m):
    """Normalised kinetic heat flux Q / (n m v_t^3), [cells, 16] (10 valid)."""
    mom = np.asarray(mom, dtype=np.float64)
    n, u, T6 = _local(mom, m)
    Tref = (T6[..., 0] + T6[..., 3] + T6[..., 5]) / 3.0
    ok = (n > 1e-12) & (Tref > 0)
    vt = np.sqrt(np.where(ok, Tref, 1.0) / m)
    Q = heat_flux(mom, m)
    y = np.zeros(mom.shape[:-1] + (N_OUT_PAD,))
    with np.errstate(divide="ignore", invalid="ignore"):
        y[..., :N_OUT] = np.where(ok[..., None], Q / (n * m * vt ** 3)[..., None], 0.0)
    return y.reshape(-1, N_OUT_PAD)


def qcal_from_closure(U, Qn, scale, m):
    """Third moment Q-calligraphic = Q + sym(u (x) P) - 2 m n uuu (the
    definition of Q in Sec. 2.1 solved for Q-calligraphic), with the heat flux
    Q = scale * Qn from the network; U[..., 10], Qn[..., >=10], scale[...]."""
    U = np.asarray(U, dtype=np.float64)
    n = U[..., 0]
    u = U[..., 1:4] / n[..., None]
    Pm = np.empty(U.shape[:-1] + (3, 3))
    for k, (a, b) in enumerate(PAIRS):
        Pm[..., a, b] = U[..., 4 + k]
        Pm[..., b, a] = U[..., 4 + k]
    out = np.empty(U.shape[:-1] + (10,))
    for k, (a, b, c) in enumerate(TRIPLES):
        symuP = u[..., a] * Pm[..., b, c] + u[..., b] * Pm[..., a, c] + u[..., c] * Pm[..., a, b]
        out[..., k] = scale * Qn[..., k] + symuP - 2.0 * m * n * u[..., a] * u[..., b] * u[..., c]
    return out


# ----------------------------------------------------------------- network --
def weights_as_used(params):
    """The network's weights: BF16-rounded W, FP32 b (as FP64 arrays)."""
    d = unpack(np.asarray(params, dtype=np.float32))
    return {k: (bf16_round(v) if k[0] == "W" else v.astype(np.float64)) for k, v in d.items()}


def forward(params, x, exact_weights=False):
    """x[N, 64] -> (y[N, 16], cache).  exact_weights: use params as given (FP64)
    instead of their BF16 rounding (for derivative checks)."""
    w = unpack(np.asarray(params, dtype=np.float64)) if exact_weights else weights_as_used(params)
    h0 = np.asarray(x, dtype=np.float64)
    a1 = h0 @ w["W1"].T + w["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.tanh(a2)
    a3 = h2 @ w["W3"].T + w["b3"]
    h3 = np.tanh(a3)
    y = h3 @ w["W4"].T + w["b4"]
    return y, dict(w=w, h0=h0, h1=h1, h2=h2, h3=h3)


def loss(y, t):
    """Mean over samples and the ten valid outputs of (y - t)^2."""
    d = np.asarray(y)[:, :N_OUT] - np.asarray(t)[:, :N_OUT]
    return float((d * d).sum() / (d.shape[0] * N_OUT))


def gradient(params, x, t, exact_weights=False):
    """(loss, dloss/dparams) by backpropagation through forward()."""
    y, c = forward(params, x, exact_weights)
    N = y.shape[0]
    w = c["w"]
    dy = np.zeros_like(y)
    dy[:, :N_OUT] = 2.0 * (y[:, :N_OUT] - t[:, :N_OUT]) / (N * N_OUT)
    g = {}
    g["W4"] = dy.T @ c["h3"]
    g["b4"] = dy.sum(0)
    da3 = (dy @ w["W4"]) * (1.0 - c["h3"] ** 2)
    g["W3"] = da3.T @ c["h2"]
    g["b3"] = da3.sum(0)
    da2 = (da3 @ w["W3"]) * (1.0 - c["h2"] ** 2)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(0)
    da1 = (da2 @ w["W2"]) * (1.0 - c["h1"] ** 2)
    g["W1"] = da1.T @ c["h0"]
    g["b1"] = da1.sum(0)
    return loss(y, t), pack(g)


def adam_step(params, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; step is
    1-based.  Returns (params, m1, m2) in FP64."""
    params, grad = np.asarray(params, dtype=np.float64), np.asarray(grad, dtype=np.float64)
    m1 = beta1 * np.asarray(m1, dtype=np.float64) + (1.0 - beta1) * grad
    m2 = beta2 * np.asarray(m2, dtype=np.float64) + (1.0 - beta2) * grad * grad
    mh = m1 / (1.0 - beta1 ** step)
    vh = m2 / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2


# ------------------------------------------------ comparators (Eq. 5) -------
def _pad_y(arr, parity):
    """One mirrored ghost row on each side in y (axis 0), periodic x handled by roll."""
    lo = arr[:1] * parity
    hi = arr[-1:] * parity
    return np.concatenate([lo, arr, hi], axis=0)


def divergence_heat_flux(Q10, dx, dy):
    """(div Q)_ij = d_x Q_xij + d_y Q_yij (2-D, z-invariant) by central
    differences; Q10[ny, nx, 10] -> [ny, nx, 6] (PAIRS order)."""
    Q10 = np.asarray(Q10, dtype=np.float64)
    par = np.array([(-1.0) ** sum(i == 1 for i in t) for t in TRIPLES])
    Qg = _pad_y(Q10, par)

    def comp(a, b, c):
        key = tuple(sorted((a, b, c)))
        return TRIPLES.index(key)

    out = np.empty(Q10.shape[:2] + (6,))
    for k, (i, j) in enumerate(PAIRS):
        qx = Q10[..., comp(0, i, j)]
        ddx = (np.roll(qx, -1, axis=1) - np.roll(qx, 1, axis=1)) / (2.0 * dx)
        qy = Qg[..., comp(1, i, j)]
        ddy = (qy[2:] - qy[:-2]) / (2.0 * dy)
        out[..., k] = ddx + ddy
    return out


def gradient_closure_divergence(U, m, q, dx, dy, bc_y="reflect"):
    """Eq. 5: div Q = -(chi/k0) n v_t lap T with k0 = 1/d_s, d_s = sqrt(m/(n0 q^2))
    for the reference density n0 = 1 (Sec. 2.1 normalisation, eps0 = 1/c^2),
    v_t = sqrt(tr(T)/(3m)); lap by central second differences (x periodic, y
    mirrored).  U[ny, nx, 10] -> [ny, nx, 6]."""
    n, u, T6 = _local(np.asarray(U, dtype=np.float64), m)
    vt = np.sqrt((T6[..., 0] + T6[..., 3] + T6[..., 5]) / (3.0 * m))
    d_s = math.sqrt(m / (q * q))
    _, pT = _y_parity_uT()
    Tg = _pad_y(T6, pT) if bc_y != "periodic" else np.concatenate([T6[-1:], T6, T6[:1]], axis=0)
    lap = ((np.roll(T6, -1, axis=1) - 2.0 * T6 + np.roll(T6, 1, axis=1)) / dx ** 2
           + (Tg[2:] - 2.0 * T6 + Tg[:-2]) / dy ** 2)
    return -(CHI * d_s) * (n * vt)[..., None] * lap


# ------------------------------------------------- the closure in a step ----
def network_heat_flux(U, m, species, params, B=None):
    """Normalised network output y[ny, nx, 16] and scale[ny, nx] for the cells
    of U[ny, nx, >=10] (B: cell-centred field for the direction features)."""
    ny, nx = U.shape[:2]
    x, scale = features_bf16(U, m, species, B)
    y, _ = forward(params, x)
    return y.reshape(ny, nx, N_OUT_PAD), scale.reshape(ny, nx)


def closure_qcal(U, m, species, params, B=None):
    """Q-calligraphic of every cell from the network applied to U."""
    y, scale = network_heat_flux(U, m, species, params, B)
    return qcal_from_closure(U, y, scale, m)


def judge_error(mom, m, species, params, B=None):
    """Relative L2 error over the cells of the network's heat-flux vector
    q_i = sum_j Q_ijj against the kinetic one, both from raw moments mom."""
    y, scale = network_heat_flux(mom[..., :10], m, species, params, B)
    Qn = scale[..., None] * y[..., :N_OUT]
    Qk = heat_flux(mom, m)

    def qvec(Q):
        return np.stack([Q[..., 0] + Q[..., 3] + Q[..., 5], Q[..., 1] + Q[..., 6] + Q[..., 8],
                         Q[..., 2] + Q[..., 7] + Q[..., 9]], axis=-1)
    qn, qk = qvec(Qn), qvec(Qk)
    return float(np.sqrt(((qn - qk) ** 2).sum()) / max(np.sqrt((qk ** 2).sum()), 1e-300))
