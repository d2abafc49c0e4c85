"""Ten-moment fluid solver with kinetic (or external) heat-flux input, FP64
CPU oracle.  Test infrastructure only.

Equations: Eqs. 2-4 of the paper (continuity, momentum, second-moment
equation with the symmetrised Lorentz terms) with the flux of the second
moment P given by the third moment Q-calligraphic.  In the moment-fitting
method that third moment comes from f (Sec. 2.1 after Eq. 4; Algorithm 1,
"calculate third moment"), at the Runge-Kutta stage times t, t+1 and t+1/2.

Scheme (Sec. 2.1 names it; the paper prints no formula):
* CWENO-3 reconstruction of Kurganov and Levy (2000), componentwise on the
  conserved variables and on Q-calligraphic ("incorporated into the CWENO
  reconstruction", Sec. 2.2): three polynomials P_L, P_C, P_R with linear
  weights (1/4, 1/2, 1/4), smoothness indicators
  IS_L = (u_j - u_{j-1})^2, IS_R = (u_{j+1} - u_j)^2,
  IS_C = 13/3 (u_{j+1} - 2u_j + u_{j-1})^2 + 1/4 (u_{j+1} - u_{j-1})^2,
  nonlinear weights C_k / (eps + IS_k)^2 with eps = 1e-6, normalised.
* Semi-discrete central (local Lax-Friedrichs) flux
  H = (F(U+) + F(U-))/2 - a/2 (U+ - U-), a = max over U+- of
  abs(u_d) + sqrt(3 p_dd / (m n)), p = P - m n u u.
* SSP-RK3 of Shu and Osher (1988); its stage times t, t+1, t+1/2 are the
  times at which Algorithm 1 supplies Q-calligraphic.

Component orders: U = (n, nu_x, nu_y, nu_z, P_xx, P_xy, P_xz, P_yy, P_yz,
P_zz); Q-calligraphic as in oracle.moments.TRIPLES.  1V: U = (n, nu, P).
Boundaries: x periodic; y reflecting (ghost cells mirror the interior, with
the sign flipped for components carrying an odd number of y indices) or
periodic.
"""
import numpy as np

from .moments import PAIRS, TRIPLES

EPS = 1e-6
LIN_W = (0.25, 0.5, 0.25)


# ------------------------------------------------------- reconstruction ---
def cweno_faces(um, u0, up):
    """CWENO-3 point values of cell j's reconstruction at its left and right
    faces, from the cell averages u_{j-1}, u_j, u_{j+1}.  Returns (left, right)."""
    d2 = up - 2.0 * u0 + um

    def P_L(xi):
        return u0 + (u0 - um) * xi

    def P_R(xi):
        return u0 + (up - u0) * xi

    def P_C(xi):
        return u0 - d2 / 12.0 + 0.5 * (up - um) * xi + d2 * xi * xi

    IS = ((u0 - um) ** 2,
          13.0 / 3.0 * d2 ** 2 + 0.25 * (up - um) ** 2,
          (up - u0) ** 2)
    alpha = [c / (EPS + s) ** 2 for c, s in zip(LIN_W, IS)]
    tot = alpha[0] + alpha[1] + alpha[2]
    w = [a / tot for a in alpha]
    left = w[0] * P_L(-0.5) + w[1] * P_C(-0.5) + w[2] * P_R(-0.5)
    right = w[0] * P_L(0.5) + w[1] * P_C(0.5) + w[2] * P_R(0.5)
    return left, right


def _pair_index(a, b):
    return PAIRS.index(tuple(sorted((a, b))))


def _triple_index(a, b, c):
    return TRIPLES.index(tuple(sorted((a, b, c))))


def y_parity_u():
    """+1/-1 per U component under y -> -y."""
    par = [1.0, 1.0, -1.0, 1.0]
    par += [(-1.0) ** ((a == 1) + (b == 1)) for a, b in PAIRS]
    return np.array(par)


def y_parity_q():
    return np.array([(-1.0) ** sum(i == 1 for i in t) for t in TRIPLES])


# ------------------------------------------------------- 3V (2X3V) --------
def _flux_3v(U, Qc, d, m):
    F = np.empty_like(U)
    F[..., 0] = U[..., 1 + d]
    for i in range(3):
        F[..., 1 + i] = U[..., 4 + _pair_index(i, d)] / m
    for k, (i, j) in enumerate(PAIRS):
        F[..., 4 + k] = Qc[..., _triple_index(i, j, d)]
    return F


def _speed_3v(U, d, m):
    n = U[..., 0]
    u = U[..., 1 + d] / n
    p = U[..., 4 + _pair_index(d, d)] - m * n * u * u
    return np.abs(u) + np.sqrt(np.maximum(3.0 * p / (m * n), 0.0))


def _source_3v(U, E, B, q, m):
    S = np.zeros_like(U)
    n = U[..., 0]
    nu = U[..., 1:4]
    P = np.zeros(U.shape[:-1] + (3, 3))
    for k, (a, b) in enumerate(PAIRS):
        P[..., a, b] = P[..., b, a] = U[..., 4 + k]
    # momentum: (q/m) (n E + nu x B)
    S[..., 1:4] = (q / m) * (n[..., None] * E + np.cross(nu, B))
    # second moment: q (nu_i E_j + nu_j E_i) + (q/m)(eps_jkl P_ik B_l + eps_ikl P_jk B_l)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    PxB = np.einsum("jkl,...ik,...l->...ij", eps, P, B)     # eps_jkl P_ik B_l
    for k, (a, b) in enumerate(PAIRS):
        S[..., 4 + k] = (q * (nu[..., a] * E[..., b] + nu[..., b] * E[..., a])
                         + (q / m) * (PxB[..., a, b] + PxB[..., b, a]))
    return S


def _pad(arr, axis, bc, parity):
    """Two ghost cells on each side of `axis` (0 = y, 1 = x).  Periodic
    ghosts are the cells of index mod n, also where the axis has fewer cells
    than ghosts (n = 1)."""
    if bc == "periodic":
        return np.concatenate([np.take(arr, [-2, -1], axis=axis, mode="wrap"), arr,
                               np.take(arr, [0, 1], axis=axis, mode="wrap")], axis=axis)
    lo = np.take(arr, [1, 0], axis=axis) * parity
    hi = np.take(arr, [-1, -2], axis=axis) * parity
    return np.concatenate([lo, arr, hi], axis=axis)


def rhs_3v(U, Qc, E, B, q, m, dx, dy, bc_y="reflect"):
    """L(U) = -div H + S on U[ny, nx, 10] with Q-calligraphic Qc[ny, nx, 10]."""
    L = _source_3v(U, E, B, q, m)
    pu, pq = y_parity_u(), y_parity_q()
    for axis, d, h, bc in ((1, 0, dx, "periodic"), (0, 1, dy, bc_y)):
        Ug = _pad(U, axis, bc, pu)
        Qg = _pad(Qc, axis, bc, pq)
        n = U.shape[axis]

        def sl(a, lo, hi):
            idx = [slice(None)] * a.ndim
            idx[axis] = slice(lo, hi)
            return a[tuple(idx)]

        # reconstructions of cells -1 .. n (indices 1 .. n+2 in padded arrays)
        UL, UR = cweno_faces(sl(Ug, 0, n + 2), sl(Ug, 1, n + 3), sl(Ug, 2, n + 4))
        QL, QR = cweno_faces(sl(Qg, 0, n + 2), sl(Qg, 1, n + 3), sl(Qg, 2, n + 4))
        # faces -1/2 .. n-1/2: left state = right face of cell f-1, right state = left face of cell f
        Um, Up = sl(UR, 0, n + 1), sl(UL, 1, n + 2)
        Qm, Qp = sl(QR, 0, n + 1), sl(QL, 1, n + 2)
        a = np.maximum(_speed_3v(Um, d, m), _speed_3v(Up, d, m))[..., None]
        H = 0.5 * (_flux_3v(Up, Qp, d, m) + _flux_3v(Um, Qm, d, m)) - 0.5 * a * (Up - Um)
        L -= (sl(H, 1, n + 1) - sl(H, 0, n)) / h
    return L


def rk3_3v(U, Q_t, Q_t1, fields_t, fields_t1, fields_th, q, m, dx, dy, dt, bc_y="reflect"):
    """One SSP-RK3 step; Q and (E, B) given at the stage times t, t+1, t+1/2."""
    Q_th = 0.5 * (Q_t + Q_t1)
    U1 = U + dt * rhs_3v(U, Q_t, *fields_t, q, m, dx, dy, bc_y)
    U2 = 0.75 * U + 0.25 * (U1 + dt * rhs_3v(U1, Q_t1, *fields_t1, q, m, dx, dy, bc_y))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * rhs_3v(U2, Q_th, *fields_th, q, m, dx, dy, bc_y))


def rk3_3v_stagewise(U, qcal_of, fields_t, fields_t1, fields_th, q, m, dx, dy, dt, bc_y="reflect"):
    """SSP-RK3 with the third moment of each stage computed from that stage's
    state and fields by qcal_of(U_stage, B_stage) (a closure instead of the
    kinetic moments)."""
    U1 = U + dt * rhs_3v(U, qcal_of(U, fields_t[1]), *fields_t, q, m, dx, dy, bc_y)
    U2 = 0.75 * U + 0.25 * (U1 + dt * rhs_3v(U1, qcal_of(U1, fields_t1[1]), *fields_t1, q, m, dx, dy, bc_y))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * rhs_3v(U2, qcal_of(U2, fields_th[1]), *fields_th, q, m, dx, dy, bc_y))


def rk3_3v_closure(U, qcal_of, source_of, fields_t, fields_t1, fields_th, q, m, dx, dy, dt, bc_y="reflect"):
    """SSP-RK3 in which every stage takes its third moment from
    qcal_of(U_stage, B_stage) and adds source_of(U_stage) ([ny, nx, 10], or
    None for no source) to L: the fluid model run with a heat-flux closure
    (Sec. 2.3) instead of the kinetic third moment."""
    def L(V, fl):
        r = rhs_3v(V, qcal_of(V, fl[1]), *fl, q, m, dx, dy, bc_y)
        return r if source_of is None else r + source_of(V)
    U1 = U + dt * L(U, fields_t)
    U2 = 0.75 * U + 0.25 * (U1 + dt * L(U1, fields_t1))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * L(U2, fields_th))


# ------------------------------------------------------- 1V (1X1V) --------
def rhs_1v(U, Qc, E, q, m, dx):
    """L(U) on U[nx, 3] = (n, nu, P) with Q-calligraphic Qc[nx], E[nx]; periodic."""
    n_, nu, P = U[:, 0], U[:, 1], U[:, 2]
    S = np.zeros_like(U)
    S[:, 1] = (q / m) * n_ * E
    S[:, 2] = 2.0 * q * nu * E
    N = U.shape[0]
    ring = np.arange(-2, N + 2)                  # two ghosts each side, cell index mod N
    Ug = np.take(U, ring, axis=0, mode="wrap")
    Qg = np.take(Qc, ring, mode="wrap")
    UL, UR = cweno_faces(Ug[0:N + 2], Ug[1:N + 3], Ug[2:N + 4])
    QL, QR = cweno_faces(Qg[0:N + 2], Qg[1:N + 3], Qg[2:N + 4])
    Um, Up = UR[0:N + 1], UL[1:N + 2]
    Qm, Qp = QR[0:N + 1], QL[1:N + 2]

    def flux(V, Qv):
        return np.stack([V[:, 1], V[:, 2] / m, Qv], axis=1)

    def speed(V):
        u = V[:, 1] / V[:, 0]
        p = V[:, 2] - m * V[:, 0] * u * u
        return np.abs(u) + np.sqrt(np.maximum(3.0 * p / (m * V[:, 0]), 0.0))

    a = np.maximum(speed(Um), speed(Up))[:, None]
    H = 0.5 * (flux(Up, Qp) + flux(Um, Qm)) - 0.5 * a * (Up - Um)
    return S - (H[1:] - H[:-1]) / dx


def rk3_1v(U, Q_t, Q_t1, E_t, E_t1, q, m, dx, dt):
    Q_th = 0.5 * (Q_t + Q_t1)
    E_th = 0.5 * (E_t + E_t1)
    U1 = U + dt * rhs_1v(U, Q_t, E_t, q, m, dx)
    U2 = 0.75 * U + 0.25 * (U1 + dt * rhs_1v(U1, Q_t1, E_t1, q, m, dx))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * rhs_1v(U2, Q_th, E_th, q, m, dx))
