"""Oracle: point sets of the DPM and projection of the discrete boundary onto Gamma.

Point sets follow the paper's definition "point sets" (Sec. 2): M0 = interior nodes of the
auxiliary cube, M+ = M0 inside Omega, M- = M0 \\ M+, N+/N-/N0 = union of the 7-point stencils
centred at M+/M-/M0, gamma = N+ intersect N-, gamma_in = M+ intersect gamma,
gamma_ex = M- intersect gamma.  They are computed literally, as unions of stencils on the array
padded with the ghost layer.

Readings where the paper is silent:
  * a node exactly on Gamma belongs to M- (M+ is the interior of Omega);
  * if N+ reaches the ghost layer (an M+ node on the outermost interior layer) the auxiliary
    cube has no margin and the geometry is rejected: the AP would pin N+ values to zero;
  * gamma is listed in ascending linear index of the [z][y][x] interior array;
  * the projection x' is the closest point of Gamma (sphere: radial; ellipsoid: foot point of
    the normal), d is the signed distance, positive outside (extension operator, Sec. 2),
    and the angles are the polar/azimuthal angles of x' (ellipsoid: the parametric angles of
    x' = (a sin t cos p, b sin t sin p, c cos t)).

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def inside_sphere(z, y, x, center=(0.0, 0.0, 0.0), radius=1.0):
    cx, cy, cz = center
    return (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 < radius**2


def inside_ellipsoid(z, y, x, center=(0.0, 0.0, 0.0), axes=(1.0, 0.8, 0.6)):
    cx, cy, cz = center
    a, b, c = axes
    return ((x - cx) / a) ** 2 + ((y - cy) / b) ** 2 + ((z - cz) / c) ** 2 < 1.0


def _dilate(s: np.ndarray) -> np.ndarray:
    """Union of the 7-point stencils centred at the points of s (no wrap-around)."""
    d = s.copy()
    d[1:, :, :] |= s[:-1, :, :]
    d[:-1, :, :] |= s[1:, :, :]
    d[:, 1:, :] |= s[:, :-1, :]
    d[:, :-1, :] |= s[:, 1:, :]
    d[:, :, 1:] |= s[:, :, :-1]
    d[:, :, :-1] |= s[:, :, 1:]
    return d


class PointSets:
    """gamma, gamma_in, gamma_ex of an M+ mask over the n^3 interior nodes."""

    def __init__(self, m_plus: np.ndarray):
        m_plus = np.asarray(m_plus, dtype=bool)
        n = m_plus.shape[0]
        self.n = n
        padded = np.zeros((n + 2,) * 3, dtype=bool)
        m0 = padded.copy()
        m0[1:-1, 1:-1, 1:-1] = True
        mp = padded.copy()
        mp[1:-1, 1:-1, 1:-1] = m_plus
        mm = m0 & ~mp
        n_plus = _dilate(mp)
        n_minus = _dilate(mm)
        gamma = n_plus & n_minus
        # the AP forces zero on the ghost layer, so N+ must stay inside M0
        self.margin_ok = not bool((n_plus & ~m0).any())
        inner = (slice(1, -1),) * 3
        self.m_plus = m_plus
        self.m_minus = ~m_plus
        self.n_plus = n_plus[inner]
        self.gamma = gamma[inner]
        self.gamma_in = self.gamma & m_plus
        self.gamma_ex = self.gamma & ~m_plus
        self.idx = np.flatnonzero(self.gamma.ravel())          # ascending linear index
        self.is_in = self.gamma_in.ravel()[self.idx]
        self.idx_in = self.idx[self.is_in]

    @property
    def n_gamma(self) -> int:
        return int(self.idx.size)

    @property
    def n_gamma_in(self) -> int:
        return int(self.idx_in.size)


def project_sphere(z, y, x, center=(0.0, 0.0, 0.0), radius=1.0):
    """Closest point on the sphere: returns (d, theta, phi) with d = |x-c| - r (+ outside)."""
    cx, cy, cz = center
    px, py, pz = x - cx, y - cy, z - cz
    rho = np.sqrt(px * px + py * py + pz * pz)
    d = rho - radius
    # polar angle as atan2(sin, cos): well conditioned at the poles (arccos loses sqrt(eps))
    theta = np.arctan2(np.sqrt(px * px + py * py), pz)
    phi = np.arctan2(py, px)
    return d, theta, phi


def project_ellipsoid(z, y, x, center=(0.0, 0.0, 0.0), axes=(1.0, 0.8, 0.6)):
    """Foot point of the normal through each point onto the ellipsoid.

    The closest point q satisfies q_i = a_i^2 p_i / (a_i^2 + t) with the scalar t a root of
    sum_i a_i^2 p_i^2 / (a_i^2 + t)^2 = 1 on (-min a_i^2, inf); found by bracketing + Brent.
    Returns (d, theta, phi): signed distance (+ outside) and the parametric angles of q.
    """
    a = np.asarray(axes, dtype=np.float64)
    p_all = np.stack([np.ravel(x) - center[0], np.ravel(y) - center[1], np.ravel(z) - center[2]], 1)
    d = np.empty(len(p_all))
    th = np.empty(len(p_all))
    ph = np.empty(len(p_all))
    a2 = a * a
    lo = -a2.min()
    for i, p in enumerate(p_all):
        def F(t):
            return float(np.sum(a2 * p * p / (a2 + t) ** 2) - 1.0)
        t_lo = lo * (1.0 - 1e-14)
        t_hi = max(1.0, 4.0 * np.linalg.norm(p) * a.max())
        while F(t_hi) > 0:
            t_hi *= 2.0
        if F(t_lo) < 0:
            raise ValueError("projection onto the ellipsoid is not unique for this point")
        t = brentq(F, t_lo, t_hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
        q = a2 * p / (a2 + t)
        outside = float(np.sum(p * p / a2)) > 1.0
        dist = float(np.linalg.norm(p - q))
        d[i] = dist if outside else -dist
        u, v, w = q / a
        th[i] = np.arctan2(np.hypot(u, v), w)
        ph[i] = np.arctan2(v, u)
    shp = np.shape(x)
    return d.reshape(shp), th.reshape(shp), ph.reshape(shp)


def gamma_coords(ps: PointSets, x0: float, h: float):
    """Coordinates (z, y, x) of the gamma nodes, in gamma order."""
    n = ps.n
    iz, iy, ix = np.unravel_index(ps.idx, (n, n, n))
    return x0 + h * iz, x0 + h * iy, x0 + h * ix
