"""One-dimensional PFC sweep (positive and flux conservative semi-Lagrangian
advection), FP64 CPU oracle.  Test infrastructure only.

The paper advances f with the third-order PFC scheme of Filbet, Sonnendruecker
and Bertrand (2001) (Sec. 2.1, "The Vlasov-Maxwell System and its Numerical
Representation"; Introduction), with zero-flux boundaries in velocity space.
The paper does not print the scheme; what follows is that scheme restated:

* f_i are cell averages on a uniform 1-D grid; over one sub-step every point
  moves by s cells (s uniform along the pencil: true for each split direction
  of Eq. 1, since the x-speed does not depend on x and each velocity-space
  acceleration component does not depend on its own velocity coordinate).
* The cell update is in flux form, f_i' = f_i + Phi_{i-1/2} - Phi_{i+1/2},
  with Phi_{i+1/2} the mass that crosses face i+1/2 during the sub-step.
* For s >= 0 write s = K + a, K = floor(s), 0 <= a < 1.  The foot of face i+1/2
  lies in cell j = i - K, a distance a*dx left of that cell's right face, and
  Phi_{i+1/2} = sum_{m=j+1}^{i} f_m + phi(j, a) with
      phi(j, a) = a [f_j + (1-a)(2-a)/6 * eps+_j (f_{j+1}-f_j)
                         + (1-a)(1+a)/6 * eps-_j (f_j - f_{j-1})]
  the integral over [x_{j+1/2} - a dx, x_{j+1/2}] of the parabola that has the
  cell averages f_{j-1}, f_j, f_{j+1}.
* The slope limiters eps+-, in ratio form (bound f_inf):
      eps+ = min(1, 2 f_j / (f_{j+1}-f_j))            if f_{j+1} > f_j
             min(1, 2 (f_inf-f_j) / (f_j-f_{j+1}))    if f_{j+1} < f_j,  else 1
      eps- = min(1, 2 (f_inf-f_j) / (f_j-f_{j-1}))    if f_j > f_{j-1}
             min(1, 2 f_j / (f_{j-1}-f_j))            if f_j < f_{j-1},  else 1
  They make 0 <= f' <= f_inf whenever 0 <= f <= f_inf.
* For s < 0 the pencil is mirrored, swept with -s, and mirrored back.

Readings where the paper is silent (all listed in the design notes):
* f_inf is the maximum of the whole species array at the start of the split
  operator the sweep belongs to (X(tau) or V(tau)).  Where a zero-flux wall
  has piled mass above that bound inside V(tau), the cell's own value is the
  bound (M_j = max(f_inf, f_j)), so the limiter never inverts.
* Each result is clamped at 0 (only round-off negatives can occur).
* Zero-flux boundary: cells outside the box hold 0 and both wall faces carry
  zero flux.
* Reflecting boundary: a pencil at +v and its mirror pencil at -v form one
  periodic pencil of twice the length (the mirror copy reversed), which moves
  uniformly; this is exact reflection of the characteristics at the wall.
"""
import numpy as np


def limited_slopes(fm, f0, fp, f_inf):
    """Return (eps+ (f_{j+1}-f_j), eps- (f_j-f_{j-1})) in the ratio form above."""
    fm, f0, fp = (np.asarray(a, dtype=np.float64) for a in (fm, f0, fp))
    bound = np.maximum(f_inf, f0)
    dp = fp - f0
    dm = f0 - fm
    eps_p = np.ones_like(f0)
    eps_m = np.ones_like(f0)
    with np.errstate(divide="ignore", invalid="ignore"):
        up = dp > 0
        dn = dp < 0
        eps_p = np.where(up, np.minimum(1.0, 2.0 * f0 / dp), eps_p)
        eps_p = np.where(dn, np.minimum(1.0, 2.0 * (bound - f0) / (f0 - fp)), eps_p)
        up = dm > 0
        dn = dm < 0
        eps_m = np.where(up, np.minimum(1.0, 2.0 * (bound - f0) / dm), eps_m)
        eps_m = np.where(dn, np.minimum(1.0, 2.0 * f0 / (fm - f0)), eps_m)
    return eps_p * dp, eps_m * dm


def partial_flux(fm, f0, fp, a, f_inf):
    """phi(j, a): mass of the reconstructed cell j within a*dx of its right face."""
    lp, lm = limited_slopes(fm, f0, fp, f_inf)
    return a * (f0 + (1.0 - a) * (2.0 - a) / 6.0 * lp + (1.0 - a) * (1.0 + a) / 6.0 * lm)


def _split_shift(s):
    s = np.asarray(s, dtype=np.float64)
    K = np.floor(s).astype(np.int64)
    a = s - K
    return K, a


def _sweep_periodic_pos(f, s, f_inf):
    """f: [P, N] pencils, s: [P] shifts >= 0.  Periodic flux-form update."""
    P, N = f.shape
    K, a = _split_shift(s)
    rows = np.arange(P)
    phi_face = np.empty((P, N))  # Phi_{i+1/2}, i = 0..N-1
    for i in range(N):
        j = (i - K) % N
        total = np.zeros(P)
        for k in range(int(K.max()) if P else 0):
            take = k < K
            total += np.where(take, f[rows, (i - k) % N], 0.0)
        total += partial_flux(f[rows, (j - 1) % N], f[rows, j], f[rows, (j + 1) % N], a, f_inf)
        phi_face[:, i] = total
    out = f + np.roll(phi_face, 1, axis=1) - phi_face
    return np.maximum(out, 0.0)


def _sweep_zeroflux_pos(f, s, f_inf):
    """f: [P, N] pencils, s: [P] shifts >= 0.  Zero-flux walls at both ends."""
    P, N = f.shape
    K, a = _split_shift(s)
    def val(idx):                     # f at pencil index idx (ghosts are 0)
        idx = np.asarray(idx)
        inside = (idx >= 0) & (idx < N)
        return np.where(inside, f[np.arange(P), np.clip(idx, 0, N - 1)], 0.0)

    phi_face = np.zeros((P, N + 1))   # Phi at faces -1/2 .. N-1/2; walls stay 0
    for i in range(N - 1):            # interior faces i+1/2
        j = i - K
        total = np.zeros(P)
        for k in range(int(K.max()) if P else 0):
            total += np.where(k < K, val(i - k), 0.0)
        total += partial_flux(val(j - 1), val(j), val(j + 1), a, f_inf)
        phi_face[:, i + 1] = total
    out = f + phi_face[:, :N] - phi_face[:, 1:]
    return np.maximum(out, 0.0)


def pfc_sweep(f, s, bc, f_inf):
    """Sweep every pencil f[p, :] by s[p] cells.

    bc: "periodic" or "zeroflux".  f_inf: scalar limiter bound.
    Negative shifts are handled by mirroring the pencil.
    """
    f = np.asarray(f, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), f.shape[:1]).copy()
    kernel = {"periodic": _sweep_periodic_pos, "zeroflux": _sweep_zeroflux_pos}[bc]
    out = np.empty_like(f)
    pos = s >= 0
    if pos.any():
        out[pos] = kernel(f[pos], s[pos], f_inf)
    if (~pos).any():
        out[~pos] = kernel(f[~pos][:, ::-1], -s[~pos], f_inf)[:, ::-1]
    return out


def pfc_sweep_reflect_pair(f_up, f_dn, s, f_inf):
    """Reflecting walls at both ends for a pencil pair.

    f_up: [P, N] pencils at velocity +w (shift s >= 0 or any sign),
    f_dn: [P, N] the mirror pencils at -w.  The two form one periodic pencil
    of length 2N, [f_up, reverse(f_dn)], moving by s.  Returns (f_up', f_dn').
    """
    N = f_up.shape[1]
    doubled = np.concatenate([f_up, f_dn[:, ::-1]], axis=1)
    new = pfc_sweep(doubled, s, "periodic", f_inf)
    return new[:, :N], new[:, N:][:, ::-1]


def pfc_sweep_affine(f, alpha, s, f_inf):
    """Zero-flux sweep of pencils f[P, N] for the affine map xi -> alpha xi + s
    (alpha > 0, in cell units: cell j is [j, j+1], so the content at xi moves
    to alpha xi + s; alpha and s per pencil or scalars).

    Flux form with a foot per face: the mass that crosses the interior face at
    xi_F = i + 1 is the integral of the limited reconstruction from the foot
    xi* = (xi_F - s) / alpha to xi_F (negative when the foot lies above the
    face).  Inside cell j the reconstruction's mass from a point at distance
    a below its right face up to that face is phi(j, a), so any partial cell
    is a difference of two phi's.  Cells outside the box hold 0; both wall
    faces carry no flux.  With alpha = 1 this is the uniform sweep."""
    f = np.asarray(f, dtype=np.float64)
    P, N = f.shape
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (P,))
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), (P,))
    rows = np.arange(P)

    def val(idx):
        idx = np.asarray(idx)
        inside = (idx >= 0) & (idx < N)
        return np.where(inside, f[rows, np.clip(idx, 0, N - 1)], 0.0)

    def phi(j, a):
        """Mass of cell j within a (0..1) of its right face (0 outside the box)."""
        inside = (j >= 0) & (j < N)
        return np.where(inside, partial_flux(val(j - 1), val(j), val(j + 1), a, f_inf), 0.0)

    # cumulative masses C[k] = sum_{m<k} f_m with the zero ghosts, k = 0..N
    C = np.concatenate([np.zeros((P, 1)), np.cumsum(f, axis=1)], axis=1)

    def cum(k):                        # sum of f_m over m < k, for any integer k
        return C[rows, np.clip(k, 0, N)]

    flux = np.zeros((P, N + 1))
    for i in range(N - 1):
        xf = float(i + 1)
        foot = (xf - s) / alpha
        below = foot <= xf
        # foot below the face: cells j+1 .. i whole, plus the top part of cell j
        jb = np.ceil(foot).astype(np.int64) - 1
        ab = jb + 1 - foot                              # in (0, 1]
        fb = cum(i + 1) - cum(jb + 1) + phi(jb, ab)
        # foot above the face: cells i+1 .. j-1 whole, plus the bottom part of cell j
        ja = np.floor(foot).astype(np.int64)
        aa = ja + 1 - foot                              # in (0, 1]
        fa = -(cum(ja) - cum(i + 1) + (val(ja) - phi(ja, aa)))
        flux[:, i + 1] = np.where(below, fb, fa)
    out = f + flux[:, :N] - flux[:, 1:]
    return np.maximum(out, 0.0)
