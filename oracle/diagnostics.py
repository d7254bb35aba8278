"""Oracle: the quantities the paper tracks along a run (Sec. 4, "Error metrics and quantities
of interest": max density, second moment, free energy), for the single domain and summed over
the two subdomains of the domain decomposition.

  ||rho||_inf = max over M+ of |rho|                                       (eqs sd/dd-norm:max)
  M_h = sum over M+ of h^3 |x|^2 rho                                       (eqs sd/dd-norm:second-moment)
  E_h = sum over M+ of h^3 { rho ln rho - rho c + c^2/2
                             + (1/(8 h^2)) sum over axes (c_{+1} - c_{-1})^2 }   (eqs sd/dd-norm:free-energy)

with x the node coordinates (the paper's domain is centred at the origin).  Readings: rho ln rho
is taken as 0 for rho <= 0 (its limit at 0; the scheme keeps rho >= 0 in exact arithmetic, so
negative values are rounding, of the order of 1e-16 times the data); a NaN rho makes it NaN; the
central differences use the neighbours in N+
(inside the cube, as every M+ node's are).  For the decomposed domain the maximum is taken over
both subdomains and the sums add, each with its own h and node coordinates.

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np

from .pks import _shift


def max_density(rho: np.ndarray, m_plus: np.ndarray) -> float:
    return float(np.max(np.where(m_plus, np.abs(rho), 0.0)))


def second_moment(rho: np.ndarray, m_plus: np.ndarray, h: float, mesh) -> float:
    z, y, x = mesh
    return float(np.sum(np.where(m_plus, h**3 * (x * x + y * y + z * z) * rho, 0.0)))


def free_energy(rho: np.ndarray, c: np.ndarray, m_plus: np.ndarray, h: float) -> float:
    with np.errstate(divide="ignore", invalid="ignore"):
        rlr = np.where(rho > 0, rho * np.log(np.where(rho > 0, rho, 1.0)),
                       np.where(np.isnan(rho), np.nan, 0.0))
    grad = np.zeros_like(c)
    for ax in range(3):
        d = _shift(c, ax, 1) - _shift(c, ax, -1)
        grad += d * d
    dens = rlr - rho * c + 0.5 * c * c + grad / (8.0 * h * h)
    return float(np.sum(np.where(m_plus, h**3 * dens, 0.0)))


def diagnostics(rho, c, m_plus, h, mesh) -> tuple[float, float, float]:
    """(max density, second moment, free energy) of one domain."""
    return (max_density(rho, m_plus), second_moment(rho, m_plus, h, mesh),
            free_energy(rho, c, m_plus, h))


def dd_diagnostics(parts) -> tuple[float, float, float]:
    """The same over the subdomains: parts = [(rho_l, c_l, m_plus_l, h_l, mesh_l), ...]."""
    vals = [diagnostics(*p) for p in parts]
    return (max(v[0] for v in vals), sum(v[1] for v in vals), sum(v[2] for v in vals))
