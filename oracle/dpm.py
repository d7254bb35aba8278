"""Oracle: Difference Potentials machinery on top of the AP solve.

Paper, Sec. 2, in sigma-form (sigma = 1/dt; the paper's AP(q) equals aux_solve with b = sigma*q):
  * Particular solution G f (eq rhs:particular_solution): AP with q = f on M+, 0 on M-,
    i.e. aux_solve(sigma * 1_{M+} f), restricted to N+.
  * Difference potential P_{N+ gamma} v (Def. "DP", eq rhs:difference_potentials): AP with
    q = 0 on M+ and L[v extended by zero] on M-, i.e. aux_solve(1_{M-} (sigma - Lap_h)[v]).
  * Trace Tr_gamma / Tr_gamma_in: restriction; P_gamma = Tr_gamma P_{N+ gamma}.
  * Reduced BEP with the spectral extension (eq BEP_recast): columns
    Tr_gamma_in (I - P_gamma) phi_nu, right-hand side Tr_gamma_in G f, solved by least squares.
  * Density u_gamma = sum_nu C_nu phi_nu (eq extension_operator_recast).
  * Discrete generalized Green's formula (Prop. "discrete_gene_green_formula"):
    u = P_{N+ gamma} u_gamma + G f on N+.

Each quantity is computed as the paper states it (separate AP solves, no merging).

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np

from .aux import apply_operator, aux_solve
from .geometry import PointSets


def extend_by_zero(v_gamma: np.ndarray, ps: PointSets) -> np.ndarray:
    """Grid function on M0 equal to v on gamma and 0 elsewhere (densities of V_gamma)."""
    n = ps.n
    vol = np.zeros(n**3)
    vol[ps.idx] = v_gamma
    return vol.reshape(n, n, n)


def trace(vol: np.ndarray, idx: np.ndarray) -> np.ndarray:
    return np.asarray(vol).reshape(-1)[idx]


def particular_solution(f: np.ndarray, ps: PointSets, sigma: float, h: float) -> np.ndarray:
    """G f on M0 (use its restriction to N+)."""
    return aux_solve(sigma * np.where(ps.m_plus, f, 0.0), sigma, h)


def potential_rhs(v_gamma: np.ndarray, ps: PointSets, sigma: float, h: float) -> np.ndarray:
    """1_{M-} (sigma - Lap_h)[v extended by zero]."""
    w = extend_by_zero(v_gamma, ps)
    return np.where(ps.m_minus, apply_operator(w, sigma, h), 0.0)


def difference_potential(v_gamma: np.ndarray, ps: PointSets, sigma: float, h: float) -> np.ndarray:
    """P_{N+ gamma} v on M0 (use its restriction to N+)."""
    return aux_solve(potential_rhs(v_gamma, ps, sigma, h), sigma, h)


def projection_matrix(ps: PointSets, sigma: float, h: float) -> np.ndarray:
    """Dense P_gamma (|gamma| x |gamma|), column j = P_gamma e_j.  Small grids only."""
    ng = ps.n_gamma
    P = np.empty((ng, ng))
    for j in range(ng):
        e = np.zeros(ng)
        e[j] = 1.0
        P[:, j] = trace(difference_potential(e, ps, sigma, h), ps.idx)
    return P


def bep_matrix(basis: np.ndarray, ps: PointSets, sigma: float, h: float) -> np.ndarray:
    """Reduced-BEP matrix A (|gamma_in| x n_basis): A[:, nu] = Tr_gin (phi_nu - P_gamma phi_nu)."""
    n_basis = basis.shape[0]
    A = np.empty((ps.n_gamma_in, n_basis))
    for nu in range(n_basis):
        v = basis[nu]
        pv = trace(difference_potential(v, ps, sigma, h), ps.idx_in)
        A[:, nu] = v[ps.is_in] - pv
    return A


def least_squares(A: np.ndarray, g: np.ndarray, rcond: float | None = None) -> np.ndarray:
    """argmin_C ||A C - g||_2 (Sec. 2, the reduced BEP solved by least squares; LAPACK via
    numpy).  rcond None: the plain least-squares solution (full column rank).  rcond > 0: the
    minimum-norm least-squares solution with every singular value s <= rcond * s_max of A taken
    as zero (the truncated pseudo-inverse, the reading used where the coupled matrix of the
    decomposed domain is numerically rank deficient)."""
    return np.linalg.lstsq(A, g, rcond=rcond)[0]


def green_formula(u_gamma: np.ndarray, f: np.ndarray, ps: PointSets, sigma: float,
                  h: float) -> np.ndarray:
    """u = P_{N+ gamma} u_gamma + G f, as two separate AP solves; returned on M0."""
    return difference_potential(u_gamma, ps, sigma, h) + particular_solution(f, ps, sigma, h)
