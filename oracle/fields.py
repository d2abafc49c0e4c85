"""Field solvers, FP64 CPU oracle.  Test infrastructure only.

Electrostatic 1X1V (Sec. 3.1): Gauss's law dE/dx = rho/eps0 with eps0 = 1 and a
static uniform neutralising ion background, solved spectrally on the
periodic grid.  The uniform background only sets the k = 0 mode, which is
fixed to E_0 = 0, so E depends on the electron density's fluctuation only.
The Nyquist mode of E is set to zero.

Electromagnetic 2X3V (Sec. 2.1, Maxwell's equations; FDTD): Yee grid with
mu0 = 1, eps0 = 1/c^2 (Sec. 2.1 normalisation), so dB/dt = -curl E and
dE/dt = c^2 (curl B - j).  2-D in (x, y), translation-invariant in z.

Yee placement on cell indices (i, j) = cell centres, x periodic, y between
conducting walls at the faces j = -1/2 and j = ny - 1/2:
  Ex (i+1/2, j)   [ny,   nx]      By (i+1/2, j)    [ny,   nx]
  Ey (i, j-1/2)   [ny+1, nx]      Bx (i, j-1/2)    [ny+1, nx]
  Ez (i, j)       [ny,   nx]      Bz (i+1/2, j-1/2)[ny+1, nx]
(rows jh = 0 and jh = ny of the [ny+1] arrays lie on the walls).
Conducting walls: tangential E (Ex, Ez) and normal B (By) are odd about the
wall (ghost = -mirror), Ey, Bx, Bz are even and are updated on the wall.

Reading of "half step of Maxwell solver" (Algorithm 1; the paper gives no
form): one half step of length h = dt/2 is B -= (h/2) curl E;
E += h c^2 (curl B - j); B -= (h/2) curl E, with j fixed during it.
The current j = sum_s q_s int v f_s dv at cell centres is averaged to the E
positions (j_y on a wall face is 0 by the particles' reflection symmetry).
"""
import numpy as np


# ------------------------------------------------------------- Poisson ----
def poisson_1d(rho, dx):
    """E at cell centres from dE/dx = rho on a periodic grid (E_0 = 0)."""
    rho = np.asarray(rho, dtype=np.float64)
    N = rho.size
    rh = np.fft.rfft(rho)
    k = 2.0 * np.pi * np.fft.rfftfreq(N, d=dx)
    Eh = np.zeros_like(rh)
    Eh[1:] = rh[1:] / (1j * k[1:])
    if N % 2 == 0:
        Eh[-1] = 0.0
    return np.fft.irfft(Eh, n=N)


def efield_1x1v(n_e, dx, q_e=-1.0):
    """Electron density -> E (the uniform ion background drops out)."""
    return poisson_1d(q_e * np.asarray(n_e, dtype=np.float64), dx)


# --------------------------------------------------------------- Yee ------
class Yee:
    """Field state on the Yee grid described in the module docstring."""

    def __init__(self, nx, ny):
        self.nx, self.ny = nx, ny
        self.Ex = np.zeros((ny, nx))
        self.Ey = np.zeros((ny + 1, nx))
        self.Ez = np.zeros((ny, nx))
        self.Bx = np.zeros((ny + 1, nx))
        self.By = np.zeros((ny, nx))
        self.Bz = np.zeros((ny + 1, nx))

    def copy(self):
        o = Yee(self.nx, self.ny)
        for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            setattr(o, k, getattr(self, k).copy())
        return o


def _odd_pad_y(a):
    """Integer-row array [ny, nx] -> [ny+2, nx] with odd ghosts at both walls."""
    return np.concatenate([-a[:1], a, -a[-1:]], axis=0)


def _pad_y(a, bc_y):
    """Ghost rows -1 and ny: odd at conducting walls, wrapped when periodic."""
    if bc_y == "periodic":
        return np.concatenate([a[-1:], a, a[:1]], axis=0)
    return _odd_pad_y(a)


def _curl_e(F, dx, dy, bc_y="reflect"):
    """(curl E)_x at Bx, (curl E)_y at By, (curl E)_z at Bz positions.  With
    periodic y the [ny+1] arrays' rows 0 and ny are the same points."""
    Ez_p = _pad_y(F.Ez, bc_y)                        # rows -1 .. ny
    Ex_p = _pad_y(F.Ex, bc_y)
    cx = (Ez_p[1:] - Ez_p[:-1]) / dy                 # dEz/dy at jh = 0..ny
    cy = -(np.roll(F.Ez, -1, axis=1) - F.Ez) / dx    # -dEz/dx at (i+1/2, j)
    dEy_dx = (np.roll(F.Ey, -1, axis=1) - F.Ey) / dx  # at (i+1/2, jh)
    dEx_dy = (Ex_p[1:] - Ex_p[:-1]) / dy              # at (i+1/2, jh)
    cz = dEy_dx - dEx_dy
    return cx, cy, cz


def _curl_b(F, dx, dy):
    """(curl B)_x at Ex, (curl B)_y at Ey, (curl B)_z at Ez positions."""
    cx = (F.Bz[1:] - F.Bz[:-1]) / dy                  # dBz/dy at (i+1/2, j)
    cy = -(F.Bz - np.roll(F.Bz, 1, axis=1)) / dx      # -dBz/dx at (i, jh)
    cz = (F.By - np.roll(F.By, 1, axis=1)) / dx - (F.Bx[1:] - F.Bx[:-1]) / dy
    return cx, cy, cz


def current_on_yee(jc, bc_y="reflect"):
    """Cell-centred current jc[ny, nx, 3] -> (jx at Ex, jy at Ey, jz at Ez);
    j_y on the wall rows is 0 (reflecting), the mean across the seam
    (periodic)."""
    jx = 0.5 * (jc[..., 0] + np.roll(jc[..., 0], -1, axis=1))
    ny, nx = jc.shape[:2]
    jy = np.zeros((ny + 1, nx))
    jy[1:ny] = 0.5 * (jc[:-1, :, 1] + jc[1:, :, 1])
    if bc_y == "periodic":
        jy[0] = jy[ny] = 0.5 * (jc[-1, :, 1] + jc[0, :, 1])
    jz = jc[..., 2].copy()
    return jx, jy, jz


def maxwell_half_step(F, jc, dt, c, dx, dy, bc_y="reflect"):
    """One half step (length dt/2) of the FDTD solver with fixed current jc."""
    F = F.copy()
    h = 0.5 * dt
    jx, jy, jz = current_on_yee(jc, bc_y)
    cx, cy, cz = _curl_e(F, dx, dy, bc_y)
    F.Bx -= 0.5 * h * cx
    F.By -= 0.5 * h * cy
    F.Bz -= 0.5 * h * cz
    bx, by, bz = _curl_b(F, dx, dy)
    F.Ex += h * c * c * (bx - jx)
    F.Ey += h * c * c * (by - jy)
    F.Ez += h * c * c * (bz - jz)
    cx, cy, cz = _curl_e(F, dx, dy, bc_y)
    F.Bx -= 0.5 * h * cx
    F.By -= 0.5 * h * cy
    F.Bz -= 0.5 * h * cz
    return F


def cell_centred(F):
    """Average the Yee components to cell centres -> (E[ny,nx,3], B[ny,nx,3])."""
    E = np.empty((F.ny, F.nx, 3))
    B = np.empty((F.ny, F.nx, 3))
    E[..., 0] = 0.5 * (np.roll(F.Ex, 1, axis=1) + F.Ex)
    E[..., 1] = 0.5 * (F.Ey[:-1] + F.Ey[1:])
    E[..., 2] = F.Ez
    B[..., 0] = 0.5 * (F.Bx[:-1] + F.Bx[1:])
    B[..., 1] = 0.5 * (np.roll(F.By, 1, axis=1) + F.By)
    bz = 0.5 * (np.roll(F.Bz, 1, axis=1) + F.Bz)
    B[..., 2] = 0.5 * (bz[:-1] + bz[1:])
    return E, B


def field_energy(F, c, dx, dy):
    """sum over Yee points of B^2/2 + E^2/(2 c^2) times the cell area; points on
    the walls (rows 0 and ny of the [ny+1] arrays) carry half weight."""
    w = np.ones((F.ny + 1, 1))
    w[0] = w[-1] = 0.5
    eb = 0.5 * ((F.Bx ** 2 * w).sum() + (F.By ** 2).sum() + (F.Bz ** 2 * w).sum())
    ee = 0.5 / (c * c) * ((F.Ex ** 2).sum() + (F.Ey ** 2 * w).sum() + (F.Ez ** 2).sum())
    return (eb + ee) * dx * dy
