"""Velocity moments, ten-moment Maxwellian and moment fitting, FP64 CPU
oracle.  Test infrastructure only.

Moments (Sec. 2.1, the definitions after Eq. 1): n = int f dv,
u = (1/n) int v f dv, P = m int v(x)v f dv, Q = m int v(x)v(x)v f dv,
heat flux Q_ijk = Q_ijk - sym(u(x)P)_ijk + 2 m n u_i u_j u_k,
T = (P - m n u u)/(n k_B), heat-flux vector q_i = sum_j Q_ijj.  k_B = 1.

Ten-moment Maxwellian (Sec. 2.2, the display after Algorithm 1):
f_M ~ exp(-(m/2)(v-u)^t T^-1 (v-u)).

Moment fitting (Algorithm 1, the "Moment Fitting" block, and Sec. 2.2):
f <- f - f_M[n_V,u_V,T_V] + f_M[n_V,u_F,T_F], then limit.

Readings where the paper is silent:
* Quadrature is the midpoint rule on cell centres, used for moments,
  Maxwellians and initial data alike.
* The Maxwellian's normalisation is the discrete one, n g_j / (sum_k g_k dV),
  so that its zeroth moment is n exactly.
* The fluid moments are rescaled by n_V/n_F (n, nu and P all scaled, so u_F
  and T_F are unchanged); the fluid state itself is overwritten with the
  rescaled values.
* The limiter sets negative values to 0 and then rescales f to n_V; the
  rescale is applied in every cell (it is 1 up to round-off where nothing
  was clipped).
* A cell is left unchanged (and counted as skipped) when n_V <= 1e-12 or when
  T_V or T_F is not positive definite.

Component orders: P as (xx, xy, xz, yy, yz, zz), Q as (xxx, xxy, xxz, xyy,
xyz, xzz, yyy, yyz, yzz, zzz).  Raw moment vector per cell (3V):
[M0, M1x, M1y, M1z, P(6), Q(10)] = 20 numbers; (1V): [M0, M1, P, Q].
"""
import itertools

import numpy as np

PAIRS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
TRIPLES = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2),
           (1, 1, 1), (1, 1, 2), (1, 2, 2), (2, 2, 2)]
N_MOM_3V = 20
N_MOM_1V = 4
N_FLUID_3V = 10   # n, nu(3), P(6)
N_FLUID_1V = 3    # n, nu, P


# ------------------------------------------------------------- raw moments --
def raw_moments_1v(f, v, dv, m):
    """f[nx, nv] -> [nx, 4] = (int f, int v f, m int v^2 f, m int v^3 f)."""
    f = np.asarray(f, dtype=np.float64)
    out = np.empty(f.shape[:-1] + (4,))
    out[..., 0] = (f * dv).sum(-1)
    out[..., 1] = (f * v * dv).sum(-1)
    out[..., 2] = m * (f * v * v * dv).sum(-1)
    out[..., 3] = m * (f * v * v * v * dv).sum(-1)
    return out


def raw_moments_3v(f, v, dv, m):
    """f[..., nvx, nvy, nvz] -> [..., 20] raw moments (order in module doc)."""
    f = np.asarray(f, dtype=np.float64)
    vx, vy, vz = np.meshgrid(v[0], v[1], v[2], indexing="ij")
    vv = (vx, vy, vz)
    dV = dv[0] * dv[1] * dv[2]
    out = np.empty(f.shape[:-3] + (N_MOM_3V,))
    axes = (-3, -2, -1)
    out[..., 0] = (f * dV).sum(axes)
    for a in range(3):
        out[..., 1 + a] = (f * vv[a] * dV).sum(axes)
    for k, (a, b) in enumerate(PAIRS):
        out[..., 4 + k] = m * (f * vv[a] * vv[b] * dV).sum(axes)
    for k, (a, b, c) in enumerate(TRIPLES):
        out[..., 10 + k] = m * (f * vv[a] * vv[b] * vv[c] * dV).sum(axes)
    return out


# ----------------------------------------------------------- derived ones --
def sym2(t6):
    """(.., 6) -> (.., 3, 3) symmetric matrix."""
    t6 = np.asarray(t6)
    out = np.empty(t6.shape[:-1] + (3, 3))
    for k, (a, b) in enumerate(PAIRS):
        out[..., a, b] = t6[..., k]
        out[..., b, a] = t6[..., k]
    return out


def sym3(t10):
    """(.., 10) -> (.., 3, 3, 3) fully symmetric tensor."""
    t10 = np.asarray(t10)
    out = np.empty(t10.shape[:-1] + (3, 3, 3))
    for k, idx in enumerate(TRIPLES):
        for perm in set(itertools.permutations(idx)):
            out[(...,) + perm] = t10[..., k]
    return out


def derived_3v(mom, m):
    """Raw moments [..., 20] -> dict of n, u, P (3x3), T (3x3), Q (full heat
    flux tensor 3x3x3), q (heat-flux vector), following the definitions of
    Sec. 2.1 literally."""
    n = mom[..., 0]
    u = mom[..., 1:4] / n[..., None]
    P = sym2(mom[..., 4:10])
    Qcal = sym3(mom[..., 10:20])
    T = (P - m * n[..., None, None] * u[..., :, None] * u[..., None, :]) / n[..., None, None]
    # sym(u (x) P)_ijk = u_i P_jk + u_j P_ik + u_k P_ij
    symuP = (u[..., :, None, None] * P[..., None, :, :]
             + u[..., None, :, None] * P[..., :, None, :]
             + u[..., None, None, :] * P[..., :, :, None])
    uuu = u[..., :, None, None] * u[..., None, :, None] * u[..., None, None, :]
    Q = Qcal - symuP + 2.0 * m * n[..., None, None, None] * uuu
    q = np.einsum("...ijj->...i", Q)
    return {"n": n, "u": u, "P": P, "T": T, "Q": Q, "q": q}


def derived_1v(mom, m):
    n = mom[..., 0]
    u = mom[..., 1] / n
    P = mom[..., 2]
    T = (P - m * n * u * u) / n
    Q = mom[..., 3] - 3.0 * u * P + 2.0 * m * n * u ** 3
    return {"n": n, "u": u, "P": P, "T": T, "Q": Q, "q": Q}


# ------------------------------------------------- discrete Maxwellian -----
def maxwellian_1v(n, u, T, m, v, dv):
    """n g_j / (sum g dv), g_j = exp(-(m/2) (v_j-u)^2 / T)."""
    g = np.exp(-0.5 * m * (v - u) ** 2 / T)
    return n * g / (g.sum() * dv)


def maxwellian_3v(n, u, T, m, v, dv):
    """Discrete ten-moment Maxwellian on the velocity grid of one cell.

    g_j = exp(-(m/2) (v_j-u)^t T^-1 (v_j-u)), normalised so sum f dV = n.
    """
    Tinv = np.linalg.inv(T)
    vx, vy, vz = np.meshgrid(v[0] - u[0], v[1] - u[1], v[2] - u[2], indexing="ij")
    w = np.stack([vx, vy, vz], axis=-1)
    quad = np.einsum("...i,ij,...j->...", w, Tinv, w)
    g = np.exp(-0.5 * m * quad)
    dV = dv[0] * dv[1] * dv[2]
    return n * g / (g.sum() * dV)


def _spd(T):
    try:
        np.linalg.cholesky(T)
        return True
    except np.linalg.LinAlgError:
        return False


# -------------------------------------------------------- moment fitting ---
def fit_cell_3v(f, mom, U, m, v, dv, n_floor=1e-12):
    """Moment fitting of one cell's velocity block f[nvx, nvy, nvz].

    mom: raw moments of f (20); U: fluid state (n, nu(3), P(6)).
    Returns (f_new, U_rescaled, clipped_count, skipped).
    """
    dV = dv[0] * dv[1] * dv[2]
    nV = mom[0]
    if not nV > n_floor:
        return f.copy(), U.copy(), 0, True
    uV = mom[1:4] / nV
    TV = (sym2(mom[4:10]) - m * nV * np.outer(uV, uV)) / nV
    nF = U[0]
    if not nF > n_floor:
        return f.copy(), U.copy(), 0, True
    UF = U * (nV / nF)                                   # rescale the fluid moments
    uF = UF[1:4] / UF[0]
    TF = (sym2(UF[4:10]) - m * UF[0] * np.outer(uF, uF)) / UF[0]
    if not (_spd(TV) and _spd(TF)):
        return f.copy(), U.copy(), 0, True
    fMV = maxwellian_3v(nV, uV, TV, m, v, dv)
    fMF = maxwellian_3v(nV, uF, TF, m, v, dv)
    g = f - fMV + fMF                                    # exchange the Maxwellians
    clipped = int((g < 0).sum())
    g = np.maximum(g, 0.0)                               # limit f
    g = g * (nV / (g.sum() * dV))                        # back to the pre-exchange density
    return g, UF, clipped, False


def fit_cell_1v(f, mom, U, m, v, dv, n_floor=1e-12):
    """1V moment fitting of one cell's f[nv]; mom = (M0, M1, P, Q); U = (n, nu, P)."""
    nV = mom[0]
    if not nV > n_floor:
        return f.copy(), U.copy(), 0, True
    uV = mom[1] / nV
    TV = (mom[2] - m * nV * uV * uV) / nV
    nF = U[0]
    if not nF > n_floor:
        return f.copy(), U.copy(), 0, True
    UF = U * (nV / nF)
    uF = UF[1] / UF[0]
    TF = (UF[2] - m * UF[0] * uF * uF) / UF[0]
    if not (TV > 0 and TF > 0):
        return f.copy(), U.copy(), 0, True
    g = f - maxwellian_1v(nV, uV, TV, m, v, dv) + maxwellian_1v(nV, uF, TF, m, v, dv)
    clipped = int((g < 0).sum())
    g = np.maximum(g, 0.0)
    g = g * (nV / (g.sum() * dv))
    return g, UF, clipped, False


def moment_fit_3v(f, mom, U, m, v, dv):
    """Fit every cell of f[ny, nx, nvx, nvy, nvz]; returns (f, U, clipped, skipped)."""
    out = np.empty_like(f, dtype=np.float64)
    Uo = np.empty_like(U, dtype=np.float64)
    clipped = skipped = 0
    for idx in np.ndindex(f.shape[:2]):
        out[idx], Uo[idx], c, sk = fit_cell_3v(f[idx], mom[idx], U[idx], m, v, dv)
        clipped += c
        skipped += int(sk)
    return out, Uo, clipped, skipped


def moment_fit_1v(f, mom, U, m, v, dv):
    out = np.empty_like(f, dtype=np.float64)
    Uo = np.empty_like(U, dtype=np.float64)
    clipped = skipped = 0
    for i in range(f.shape[0]):
        out[i], Uo[i], c, sk = fit_cell_1v(f[i], mom[i], U[i], m, v, dv)
        clipped += c
        skipped += int(sk)
    return out, Uo, clipped, skipped
