"""Oracle: the domain-decomposition approach, Case 1 (the interface Z inside Omega, Z cap Gamma
empty), one IMEX time step.

Paper, Sec. 3 ("Case 1" and "BEPs for Case 1", eqs interface_condition, DD1_BEP1, DD1_BEP2,
reduced_DD1_BEP1, reduced_DD1_BEP2): Omega_1 = {|x| < r_Z} and Omega_2 = {r_Z < |x| < 1}, each
embedded in its own cube with its own mesh (N_l, h_l).  The discrete grid interface zeta_1 is
gamma of Omega_1; gamma of Omega_2 is the union of the discrete grid boundary near Gamma and the
discrete grid interface zeta_2 near Z.  Each subdomain gets the reduced BEP of the
single-domain approach; the densities are spectral extensions,
  near Gamma: sum_nu C0_nu P_nu + beta (d_G^2/2) sum_nu C2_nu P_nu   (zero Neumann data),
  near Z:     sum_nu A0_nu P_nu + d_Z sum_nu A1_nu P_nu + (d_Z^2/2) sum_nu A2_nu P_nu,
with d_G = |x| - 1 and d_Z = |x| - r_Z measured along the same (radial) normal from both sides of
Z, so that one coefficient set A for both subdomains imposes continuity of u and of its first two
normal derivatives across Z.  The coupled reduced BEPs are solved together by least squares for
[C, A]; each subdomain's solution then follows from its own Green's formula.

Readings: zonal harmonics P_nu(cos theta) on both surfaces (the paper's choice for data symmetric
about the z axis); a gamma node of Omega_2 belongs to the Gamma part when |x| > (r_Z + 1)/2,
else to zeta_2; nodes exactly on Z belong to Omega_2's M- (strict interiors, as in the single
domain).  Columns are ordered [C (Gamma part) ; A (Z part)].

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np

import dpm_inputs as inp

from .basis import zonal_basis_matrix
from .dpm import bep_matrix, difference_potential, least_squares, particular_solution, trace
from .geometry import PointSets, gamma_coords
from .pks import pks_rhs


class DDCase:
    """Grids, point sets and spectral densities of the two subdomains."""

    def __init__(self, n1: int, half1: float, n2: int, r_z: float, m_gamma: int, m_z: int,
                 beta: int = 1):
        self.r_z = r_z
        self.n1, self.n2 = n1, n2
        self.h1, self.x01 = inp.grid(n1, half1)
        self.h2, self.x02 = inp.grid(n2)
        z1, y1, x1 = inp.mesh(n1, half1)
        z2, y2, x2 = inp.mesh(n2)
        self.mesh1, self.mesh2 = (z1, y1, x1), (z2, y2, x2)
        r1 = x1 * x1 + y1 * y1 + z1 * z1
        r2 = x2 * x2 + y2 * y2 + z2 * z2
        self.ps1 = PointSets(r1 < r_z * r_z)
        self.ps2 = PointSets((r2 < 1.0) & (r2 > r_z * r_z))
        nz = m_z + 1
        self.n_gamma_cols = (beta + 1) * (m_gamma + 1)
        self.n_z_cols = 3 * nz
        # Omega_1: the Z densities on zeta_1
        self.B1 = self._z_rows(*gamma_coords(self.ps1, self.x01, self.h1), m_z)
        # Omega_2: Gamma densities on the Gamma part, Z densities on zeta_2
        gz, gy, gx = gamma_coords(self.ps2, self.x02, self.h2)
        rr = np.sqrt(gx * gx + gy * gy + gz * gz)
        on_g = rr > 0.5 * (r_z + 1.0)
        th = np.arctan2(np.sqrt(gx * gx + gy * gy), gz)
        bg = zonal_basis_matrix(rr - 1.0, th, m_gamma, beta) * on_g[None, :]
        bz = self._z_rows(gz, gy, gx, m_z) * (~on_g)[None, :]
        self.B2 = np.concatenate([bg, bz], axis=0)
        self.on_gamma2 = on_g

    def _z_rows(self, gz, gy, gx, m_z):
        rr = np.sqrt(gx * gx + gy * gy + gz * gz)
        d = rr - self.r_z
        th = np.arctan2(np.sqrt(gx * gx + gy * gy), gz)
        p = zonal_basis_matrix(d, th, m_z, 0)
        return np.concatenate([p, d[None, :] * p, 0.5 * d[None, :] ** 2 * p], axis=0)

    @property
    def n_cols(self) -> int:
        return self.n_gamma_cols + self.n_z_cols


def dd_matrix(case: DDCase, sigma: float) -> np.ndarray:
    """The coupled reduced BEP matrix, rows zeta_1,in then gamma_in of Omega_2, columns [C ; A]."""
    a1 = bep_matrix(case.B1, case.ps1, sigma, case.h1)           # |zeta_1,in| x n_z_cols
    a2 = bep_matrix(case.B2, case.ps2, sigma, case.h2)           # |gamma_2,in| x n_cols
    top = np.concatenate([np.zeros((a1.shape[0], case.n_gamma_cols)), a1], axis=1)
    return np.concatenate([top, a2], axis=0)


def dd_step(rho1, c1, rho2, c2, case: DDCase, A: np.ndarray, dt: float, chi: float):
    """One step on both subdomains (sigma = 1/dt for both species); returns the four new states
    (each on its N+, zero elsewhere) and the coefficients of both species."""
    sigma = 1.0 / dt
    f1r, f1c = pks_rhs(rho1, c1, case.ps1.m_plus, case.h1, dt, chi)
    f2r, f2c = pks_rhs(rho2, c2, case.ps2.m_plus, case.h2, dt, chi)
    out, coefs = [], []
    for f1, f2 in ((f1r, f2r), (f1c, f2c)):
        G1 = particular_solution(f1, case.ps1, sigma, case.h1)             # Step 4a
        G2 = particular_solution(f2, case.ps2, sigma, case.h2)
        g = np.concatenate([trace(G1, case.ps1.idx_in), trace(G2, case.ps2.idx_in)])
        C = least_squares(A, g)                                            # Step 5, coupled
        u1g = case.B1.T @ C[case.n_gamma_cols:]
        u2g = case.B2.T @ C
        u1 = np.where(case.ps1.n_plus, difference_potential(u1g, case.ps1, sigma, case.h1) + G1, 0.0)
        u2 = np.where(case.ps2.n_plus, difference_potential(u2g, case.ps2, sigma, case.h2) + G2, 0.0)
        out.append((u1, u2))                                               # Steps 6-7
        coefs.append(C)
    (r1, r2), (cc1, cc2) = out
    return r1, cc1, r2, cc2, coefs
