"""Oracle: spectral basis densities on the discrete boundary gamma.

Paper, Sec. 2 "Spectral Approach" (eqs extension_operator1, spectral_approximation_sd,
extension_operator_recast): with zero Neumann data the extension operator is
u|Gamma + beta (d^2/2) d2u/dn2|Gamma, and both terms are expanded in spherical harmonics of the
angles of the projection of each gamma node.  Column nu of the BEP system is therefore the
density phi_nu (theta, phi) for the first family and beta (d^2/2) phi_nu for the second.

Reading: the basis is the real, orthonormal spherical harmonics Y_lm, l = 0..L, m = -l..l in
ascending order, without the Condon-Shortley phase; the density matrix is [Y_lm ; (d^2/2) Y_lm]
(beta = 1) or [Y_lm] (beta = 0).  The paper itself uses zonal P_l(cos theta) for its symmetric
tests; the fitted solution does not depend on the scaling of the columns.

Evaluated here through scipy.special.sph_harm_y (complex, with the Condon-Shortley phase),
converted to the real form.

Zonal basis (the paper's choice for initial data symmetric about the z axis, "Basis functions,
extension operators and BEPs" and remark (i) of the spectral approach): phi_nu = P_nu(cos theta),
the Legendre polynomial of degree nu (unnormalised, as in the paper), nu = 0..M, evaluated here
through scipy.special.eval_legendre.

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, sph_harm_y


def real_sph_harm(l: int, m: int, theta, phi):
    """Real orthonormal Y_lm without the Condon-Shortley phase."""
    phi = np.mod(phi, 2.0 * np.pi)
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    sgn = (-1.0) ** abs(m)          # removes the Condon-Shortley phase
    if m > 0:
        return np.sqrt(2.0) * sgn * np.real(y)
    return np.sqrt(2.0) * sgn * np.imag(y)


def lm_list(lmax: int):
    return [(l, m) for l in range(lmax + 1) for m in range(-l, l + 1)]


def basis_matrix(d, theta, phi, lmax: int, beta: int = 1) -> np.ndarray:
    """Densities on gamma, shape (n_basis, n_gamma): rows Y_lm, then (if beta) (d^2/2) Y_lm."""
    rows = [real_sph_harm(l, m, theta, phi) for (l, m) in lm_list(lmax)]
    Y = np.array(rows, dtype=np.float64)
    if beta:
        return np.concatenate([Y, 0.5 * np.asarray(d)[None, :] ** 2 * Y], axis=0)
    return Y


def zonal_basis_matrix(d, theta, mmax: int, beta: int = 0) -> np.ndarray:
    """Zonal densities on gamma, shape ((beta + 1)(mmax + 1), n_gamma): rows P_nu(cos theta),
    nu = 0..mmax, then (if beta) (d^2/2) P_nu(cos theta)."""
    x = np.cos(np.asarray(theta, dtype=np.float64))
    P = np.array([eval_legendre(nu, x) for nu in range(mmax + 1)], dtype=np.float64)
    if beta:
        return np.concatenate([P, 0.5 * np.asarray(d)[None, :] ** 2 * P], axis=0)
    return P
