"""Split Vlasov operators X(tau) and V(tau), FP64 CPU oracle.  Test
infrastructure only.

Eq. 1 of the paper is advanced by dimensional splitting (Sec. 2.1): free
streaming X(tau) along each spatial axis and acceleration V(tau) along each
velocity axis, each a sequence of uniform 1-D PFC sweeps (oracle.pfc).

Layouts (cell-centred, C order):
  1X1V  f[nx, nv]
  2X3V  f[ny, nx, nvx, nvy, nvz]   (vz fastest)
Velocity cell centres are v_j = v_lo + (j + 1/2) dv.

Readings where the paper is silent:
* X(tau) = x-sweep then y-sweep; both use f_inf = max of X's input.  The two
  commute exactly since every shift depends only on v.
* y is bounded by reflecting walls for particles (GEM setup, Sec. 3.3):
  the pencil at +v_y and the pencil at -v_y are swept as one periodic pencil
  of twice the length (oracle.pfc.pfc_sweep_reflect_pair).  This needs a
  velocity grid that is symmetric in v_y.
* V(tau) in 3V realises the velocity splitting named in Sec. 2.1 as the
  Strang-symmetric sequence vx(tau/2) vy(tau/2) vz(tau) vy(tau/2) vx(tau/2).
  Each sweep along v_d uses the acceleration (q/m)(E_d + (v x B)_d) evaluated
  at the pencil's transverse cell-centre velocities; (v x B)_d does not
  depend on v_d, so each sweep is a uniform shift.  All five sweeps use
  f_inf = max of V's input.  Velocity boundaries are zero-flux.
"""
import numpy as np

from .pfc import pfc_sweep, pfc_sweep_affine, pfc_sweep_reflect_pair


def centres(lo, hi, n):
    """Cell-centre coordinates of a uniform grid on [lo, hi] with n cells."""
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h, h


def _sweep_axis(f, axis, s_of_pencil, bc, f_inf):
    """Sweep f along `axis`; s_of_pencil has f's shape with `axis` removed."""
    moved = np.moveaxis(f, axis, -1)
    shape = moved.shape
    pencils = moved.reshape(-1, shape[-1])
    s = np.broadcast_to(s_of_pencil, shape[:-1]).reshape(-1)
    out = pfc_sweep(pencils, s, bc, f_inf).reshape(shape)
    return np.moveaxis(out, -1, axis)


# ----------------------------------------------------------------- 1X1V ----
def x_advect_1x1v(f, v, dx, tau, f_inf=None):
    """Free streaming along periodic x: each f[:, j] moves by v_j tau / dx cells."""
    f_inf = f.max() if f_inf is None else f_inf
    s = v * tau / dx                       # per velocity cell
    return _sweep_axis(f, 0, s, "periodic", f_inf)


def v_advect_1x1v(f, E, q, m, dv, tau, f_inf=None):
    """Acceleration along v with zero-flux walls: f[i, :] moves by (q/m) E_i tau / dv."""
    f_inf = f.max() if f_inf is None else f_inf
    s = (q / m) * E * tau / dv             # per spatial cell
    return _sweep_axis(f, 1, s, "zeroflux", f_inf)


# ----------------------------------------------------------------- 2X3V ----
def x_sweep_2x3v(f, vx, dx, tau, f_inf):
    """Sweep along periodic x (axis 1) of f[ny, nx, nvx, nvy, nvz]."""
    ny, nx, nvx, nvy, nvz = f.shape
    s = np.broadcast_to((vx * tau / dx)[None, :, None, None], (ny, nvx, nvy, nvz))
    return _sweep_axis(f, 1, s, "periodic", f_inf)


def y_sweep_2x3v(f, vy, dy, tau, f_inf, bc="reflect"):
    """Sweep along y (axis 0): between reflecting walls, pairing v_y with -v_y,
    or periodic (every v_y cell its own cyclic pencil)."""
    ny, nx, nvx, nvy, nvz = f.shape
    if bc == "periodic":
        s = np.broadcast_to((vy * tau / dy)[None, None, :, None], (nx, nvx, nvy, nvz))
        return _sweep_axis(f, 0, s, "periodic", f_inf)
    assert np.allclose(vy, -vy[::-1]), "reflecting walls need a v_y grid symmetric about 0"
    out = np.empty_like(f)
    for jy in range(nvy - 1, (nvy - 1) // 2, -1):      # the v_y > 0 half (with its mirror)
        jm = nvy - 1 - jy
        up = np.moveaxis(f[:, :, :, jy, :], 0, -1).reshape(-1, ny)
        dn = np.moveaxis(f[:, :, :, jm, :], 0, -1).reshape(-1, ny)
        s = np.full(up.shape[0], vy[jy] * tau / dy)
        new_up, new_dn = pfc_sweep_reflect_pair(up, dn, s, f_inf)
        out[:, :, :, jy, :] = np.moveaxis(new_up.reshape(nx, nvx, nvz, ny), -1, 0)
        out[:, :, :, jm, :] = np.moveaxis(new_dn.reshape(nx, nvx, nvz, ny), -1, 0)
    if nvy % 2 == 1:                                     # v_y = 0 cell: no motion
        out[:, :, :, nvy // 2, :] = f[:, :, :, nvy // 2, :]
    return out


def x_advect_2x3v(f, vx, vy, dx, dy, tau, f_inf=None, bc_y="reflect"):
    """X(tau) in 2X3V: x-sweep then y-sweep, one f_inf for both."""
    f_inf = f.max() if f_inf is None else f_inf
    g = x_sweep_2x3v(f, vx, dx, tau, f_inf)
    return y_sweep_2x3v(g, vy, dy, tau, f_inf, bc_y)


def v_advect_3v(f, E, B, q, m, v, dv, tau, f_inf=None):
    """V(tau) in 3V: five uniform sweeps vx, vy, vz, vy, vx with zero-flux walls.

    f: [ny, nx, nvx, nvy, nvz]; E, B: cell-centred fields [ny, nx, 3];
    v = (vx, vy, vz) cell-centre arrays; dv = (dvx, dvy, dvz).
    """
    f_inf = f.max() if f_inf is None else f_inf
    qm = q / m
    vx, vy, vz = v
    Ex, Ey, Ez = (E[..., k][:, :, None, None] for k in range(3))
    Bx, By, Bz = (B[..., k][:, :, None, None] for k in range(3))
    g = np.asarray(f, dtype=np.float64)
    for d, frac in ((0, 0.5), (1, 0.5), (2, 1.0), (1, 0.5), (0, 0.5)):
        sig = frac * tau
        if d == 0:     # a_x = (q/m)(Ex + vy Bz - vz By), pencils (iy, ix, jy, jz)
            a = qm * (Ex + vy[None, None, :, None] * Bz - vz[None, None, None, :] * By)
        elif d == 1:   # a_y = (q/m)(Ey + vz Bx - vx Bz), pencils (iy, ix, jx, jz)
            a = qm * (Ey + vz[None, None, None, :] * Bx - vx[None, None, :, None] * Bz)
        else:          # a_z = (q/m)(Ez + vx By - vy Bx), pencils (iy, ix, jx, jy)
            a = qm * (Ez + vx[None, None, :, None] * By - vy[None, None, None, :] * Bx)
        g = _sweep_axis(g, 2 + d, a * sig / dv[d], "zeroflux", f_inf)
    return g


# ------------------------------------------------ 3V, backsubstitution split --
def lorentz_map(E, B, q, m, tau):
    """The implicit-midpoint (Boris) velocity map of one step under uniform E,
    B: v' - v = tau (q/m) (E + (v + v')/2 x B), i.e. v' = R v + c with
    R = (I - A)^-1 (I + A), A v = (tau/2)(q/m) v x B, c = (I - A)^-1 tau (q/m) E.
    R turns about B by 2 atan(Omega tau / 2).  E, B: [..., 3]."""
    E = np.asarray(E, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    t = 0.5 * tau * (q / m) * B
    # A v = v x t: rows of the matrix of v -> v x t
    A = np.zeros(B.shape[:-1] + (3, 3))
    A[..., 0, 1], A[..., 0, 2] = t[..., 2], -t[..., 1]
    A[..., 1, 0], A[..., 1, 2] = -t[..., 2], t[..., 0]
    A[..., 2, 0], A[..., 2, 1] = t[..., 1], -t[..., 0]
    I = np.broadcast_to(np.eye(3), A.shape)
    R = np.linalg.solve(I - A, I + A)
    c = np.linalg.solve(I - A, (tau * q / m * E)[..., None])[..., 0]
    return R, c


def backsub_factors(R, c):
    """Factor v -> R v + c into three maps that each change one component,
    applied x, then y, then z, each taking the components already updated:
        x' = a x + b y + e z + cx
        y' = d x' + g y + h z + cy
        z' = k x' + l y' + n z + cz
    Row by row this is back-substitution: x' is R's first row, y' gives R's
    second row through x', and (k, l) solve the 2x2 system that gives R's
    third row through x' and y'.  Returns the 12 coefficients in that order
    (a, b, e, cx, d, g, h, cy, k, l, n, cz), each [...]."""
    R = np.asarray(R)
    a, b, e = R[..., 0, 0], R[..., 0, 1], R[..., 0, 2]
    cx = c[..., 0]
    d = R[..., 1, 0] / a
    g = R[..., 1, 1] - d * b
    h = R[..., 1, 2] - d * e
    cy = c[..., 1] - d * cx
    # k R0j + l R1j = R2j for j = 0, 1
    det = R[..., 0, 0] * R[..., 1, 1] - R[..., 0, 1] * R[..., 1, 0]
    k = (R[..., 2, 0] * R[..., 1, 1] - R[..., 2, 1] * R[..., 1, 0]) / det
    l = (R[..., 0, 0] * R[..., 2, 1] - R[..., 0, 1] * R[..., 2, 0]) / det
    n = R[..., 2, 2] - k * R[..., 0, 2] - l * R[..., 1, 2]
    cz = c[..., 2] - k * c[..., 0] - l * c[..., 1]
    return a, b, e, cx, d, g, h, cy, k, l, n, cz


def v_advect_3v_backsub(f, E, B, q, m, v, dv, tau, f_inf=None):
    """V(tau) in 3V by the backsubstitution split (the velocity splitting the
    paper names in Sec. 2.1): the Boris map of each cell (lorentz_map),
    factored by backsub_factors into an x-, a y- and a z-sweep, each an
    affine map of its pencils (a stretch that is the same for every pencil
    of the cell and a shift linear in the pencil's transverse cell-centre
    velocities), swept with per-face feet (oracle.pfc.pfc_sweep_affine) and
    zero-flux walls.  The composition moves every characteristic exactly as
    the Boris map; f_inf = max of V's input for all three sweeps."""
    f = np.asarray(f, dtype=np.float64)
    f_inf = f.max() if f_inf is None else f_inf
    R, c = lorentz_map(E, B, q, m, tau)
    a, b, e, cx, d, g, h, cy, k, l, n, cz = backsub_factors(R, c)
    vx, vy, vz = v
    lo = [v[i][0] - 0.5 * dv[i] for i in range(3)]
    ex = lambda x: x[:, :, None, None]
    # stretch and velocity shift of each sweep, per cell and pencil
    sweeps = (
        (0, a, ex(b) * vy[None, None, :, None] + ex(e) * vz[None, None, None, :] + ex(cx)),
        (1, g, ex(d) * vx[None, None, :, None] + ex(h) * vz[None, None, None, :] + ex(cy)),
        (2, n, ex(k) * vx[None, None, :, None] + ex(l) * vy[None, None, None, :] + ex(cz)),
    )
    for axis, alpha, shift in sweeps:
        moved = np.moveaxis(f, 2 + axis, -1)
        shape = moved.shape
        al = np.broadcast_to(alpha[:, :, None, None], shape[:-1])
        # v -> alpha v + s in cell units xi = (v - lo)/dv: xi -> alpha xi + ((alpha - 1) lo + s) / dv
        sig = ((al - 1.0) * lo[axis] + np.broadcast_to(shift, shape[:-1])) / dv[axis]
        out = pfc_sweep_affine(moved.reshape(-1, shape[-1]), al.reshape(-1), sig.reshape(-1), f_inf)
        f = np.moveaxis(out.reshape(shape), -1, 2 + axis)
    return f
