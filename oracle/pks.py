"""Oracle: the IMEX right-hand sides of the chemotaxis scheme and one DPM time step.

Paper, Sec. 2 (eqs discrete_chemotaxis, discrete_convective_term, c-central-difference,
upwind_approximation, truncated_taylor_expansion, slope_limiter) with chi, alpha = gamma_rho =
gamma_c = 1 apart from chi:
  f_rho = rho - dt g,  f_c = (1 - dt) c + dt rho   on M+,
  g = sum over the 3 axes of (F_{+1/2} - F_{-1/2}) / h,  F = chi rho_face (c_{+1} - c)/h,
  rho_face = upwind value of the minmod-limited piecewise-linear reconstruction:
     left state  rho_j + (h/2) s_j        if the face gradient of c is > 0,
     right state rho_{j+1} - (h/2) s_{j+1} otherwise,
  s_j = minmod(2(rho_{j+1}-rho_j)/h, (rho_{j+1}-rho_{j-1})/(2h), 2(rho_j-rho_{j-1})/h).
Readings: the slope is taken as zero at gamma_ex nodes (the paper leaves the values two layers
out of N+ open); a face gradient exactly 0 takes the right state, as written.

One DPM step (Algorithm "Main Steps", Steps 4a, 5, 6, 7; sigma = 1/dt for both species):
particular solutions, Tr_gamma_in G f, least squares against the precomputed BEP matrix,
density, difference potential, Green's formula, restricted to N+.

The adaptive loop (Steps 3-8): each step takes dt = min(CFL-type bound of the positivity
theorem, previous dt), rebuilds the BEP matrix at sigma = 1/dt when dt shrank (Step 4b), and
stops at the final time, after a step budget, or when max |rho| over M+ passes a threshold
(Step 8).  Reading: dt never grows once reduced, so the matrix always belongs to the step's dt
(the algorithm rebuilds only on a decrease and is silent on increases).

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np

from .dpm import bep_matrix, difference_potential, least_squares, particular_solution, trace
from .geometry import PointSets


def minmod3(a, b, c):
    pos = (a > 0) & (b > 0) & (c > 0)
    neg = (a < 0) & (b < 0) & (c < 0)
    return np.where(pos, np.minimum(np.minimum(a, b), c),
                    np.where(neg, np.maximum(np.maximum(a, b), c), 0.0))


def _shift(a: np.ndarray, axis: int, k: int) -> np.ndarray:
    """out[i] = a[i + k] along axis, zero where i + k is outside."""
    out = np.zeros_like(a)
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if k > 0:
        src[axis] = slice(k, None)
        dst[axis] = slice(None, -k)
    else:
        src[axis] = slice(None, k)
        dst[axis] = slice(-k, None)
    out[tuple(dst)] = a[tuple(src)]
    return out


def limited_slopes(rho: np.ndarray, m_plus: np.ndarray, h: float):
    """Minmod slopes along z, y, x at the nodes of M+ (zero elsewhere)."""
    out = []
    for ax in range(3):
        rp, rm = _shift(rho, ax, 1), _shift(rho, ax, -1)
        s = minmod3(2.0 * (rp - rho) / h, (rp - rm) / (2.0 * h), 2.0 * (rho - rm) / h)
        out.append(np.where(m_plus, s, 0.0))
    return out


def convective_term(rho: np.ndarray, c: np.ndarray, m_plus: np.ndarray, h: float,
                    chi: float) -> np.ndarray:
    """g on M+ (zero elsewhere); rho and c hold values on N+."""
    slopes = limited_slopes(rho, m_plus, h)
    g = np.zeros_like(rho)
    for ax in range(3):
        s = slopes[ax]
        rp, sp, cp = _shift(rho, ax, 1), _shift(s, ax, 1), _shift(c, ax, 1)
        grad_c = (cp - c) / h                               # at the face i + 1/2
        face = np.where(grad_c > 0, rho + 0.5 * h * s, rp - 0.5 * h * sp)
        flux = chi * face * grad_c                          # F_{i+1/2}
        g += (flux - _shift(flux, ax, -1)) / h              # F_{i+1/2} - F_{i-1/2}
    return np.where(m_plus, g, 0.0)


def pks_rhs(rho, c, m_plus, h, dt, chi):
    """(f_rho, f_c) on M+ (zero elsewhere)."""
    g = convective_term(rho, c, m_plus, h, chi)
    f_rho = np.where(m_plus, rho - dt * g, 0.0)
    f_c = np.where(m_plus, (1.0 - dt) * c + dt * rho, 0.0)
    return f_rho, f_c


def face_gradient_max(c: np.ndarray, m_plus: np.ndarray, h: float) -> float:
    """max |grad_h c| over the six faces of every M+ node (eq cfl_condition)."""
    gmax = 0.0
    for ax in range(3):
        for k in (1, -1):
            gr = np.abs(_shift(c, ax, k) - c) / h
            gmax = max(gmax, float(np.max(np.where(m_plus, gr, 0.0))))
    return gmax


def cfl_dt(c: np.ndarray, m_plus: np.ndarray, h: float, chi: float) -> float:
    """Largest dt allowed by the CFL-type condition of the positivity theorem."""
    gmax = face_gradient_max(c, m_plus, h)
    return np.inf if gmax == 0.0 or chi == 0.0 else h / (6.0 * chi * gmax)


def dpm_step(rho, c, ps: PointSets, basis: np.ndarray, A: np.ndarray, h: float, dt: float,
             chi: float):
    """One time step; returns (rho_new, c_new) on N+ (zero elsewhere) and the coefficients."""
    sigma = 1.0 / dt
    f_rho, f_c = pks_rhs(rho, c, ps.m_plus, h, dt, chi)
    out, coefs = [], []
    for f in (f_rho, f_c):
        Gf = particular_solution(f, ps, sigma, h)                 # Step 4a
        C = least_squares(A, trace(Gf, ps.idx_in))                # Step 5
        u_gamma = basis.T @ C                                     # Step 5 (density)
        Pu = difference_potential(u_gamma, ps, sigma, h)          # Step 6
        u = np.where(ps.n_plus, Pu + Gf, 0.0)                     # Step 7
        out.append(u)
        coefs.append(C)
    return out[0], out[1], coefs


def adaptive_run(rho, c, ps: PointSets, basis: np.ndarray, h: float, sigma0: float, chi: float,
                 t_final: float, rho_cap: float = np.inf, max_steps: int = 1000,
                 rho_jump_cap: float = 0.0):
    """Steps 3-8 from dt_0 = 1/sigma0 (the step of Step 2's matrix).

    Returns (rho, c, summary) with summary keys steps, rebuilds, stop, t, dt, rho_max,
    grad_max, dt_hist, rebuilt and cfl_hist (the CFL-type bound of each step's state)."""
    dt_prev = 1.0 / sigma0
    A = bep_matrix(basis, ps, sigma0, h)                               # Step 2
    t, dts, rebuilt, cfls, stop = 0.0, [], [], [], "max_steps"
    gmax = rmax = rprev = 0.0
    while True:
        if t >= t_final:
            stop = "t_final"
            break
        if len(dts) >= max_steps:
            stop = "max_steps"
            break
        gmax = face_gradient_max(c, ps.m_plus, h)                      # Step 3
        rmax = float(np.max(np.where(ps.m_plus, np.abs(rho), 0.0)))    # Step 8
        if not (np.isfinite(gmax) and np.isfinite(rmax)):
            stop = "nonfinite"
            break
        if rmax > rho_cap:
            stop = "rho_cap"
            break
        # Sec. 4, Test B: stop once ||rho||_inf has grown by rho_jump_cap over one step
        if rho_jump_cap > 0 and dts and rmax - rprev >= rho_jump_cap:
            stop = "rho_jump"
            break
        rprev = rmax
        cfl = cfl_dt(c, ps.m_plus, h, chi)
        dt = min(cfl, dt_prev)
        rb = dt < dt_prev
        if rb:                                                         # Step 4b
            A = bep_matrix(basis, ps, 1.0 / dt, h)
        rho, c, _ = dpm_step(rho, c, ps, basis, A, h, dt, chi)         # Steps 4a-7
        dts.append(dt)
        rebuilt.append(rb)
        cfls.append(cfl)
        t += dt
        dt_prev = dt
    return rho, c, {"steps": len(dts), "rebuilds": int(sum(rebuilt)), "stop": stop, "t": t,
                    "dt": dt_prev, "rho_max": rmax, "grad_max": gmax, "dt_hist": dts,
                    "rebuilt": rebuilt, "cfl_hist": cfls}
