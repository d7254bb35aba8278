"""Oracle: the domain-decomposition approach, one IMEX time step: Case 1 (the interface Z inside
Omega, Z cap Gamma empty; DDCase, dd_matrix, dd_step) and Case 2 (Z meets Gamma; DDCase2,
dd2_matrix, dd2_step, below).

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


# ---------------------------------------------------------------------------------------------
# Case 2: the interface Z meets Gamma (paper Sec. 3, "Case 2" and "BEPs for Case 2", eqs
# DD2_BEP and reduced_DD2_BEP, and the remark on effective densities).
#
# Omega is the unit ball; Z is the sphere of radius r_z about q = (0, 0, q_z), a point of Gamma
# (the blow-up point of Test B), Omega_1 = Omega cap {|x - q| < r_z} (the cap around q),
# Omega_2 = Omega cap {|x - q| > r_z}.  On the mesh of subdomain l:
#   gamma   = the discrete grid boundary of the whole ball Omega (as in the single domain),
#   zeta    = the discrete grid boundary of {|x - q| < r_z} (l = 1) or of {|x - q| > r_z} (l = 2),
#   gamma_l = nodes of gamma whose projection onto Gamma has polar angle theta in
#             [0, theta* + eps] (l = 1) or [theta* - eps, pi] (l = 2),
#   zeta_l  = nodes of zeta whose projection onto Z has angle psi, measured at q from the
#             direction towards the centre of Omega, in [0, psi* + eps_z],
# theta*, psi* the angles of the circle where Z meets Gamma.  Readings: the tolerances are
# eps_layers mesh widths of the subdomain, as angles eps = eps_layers h_l / 1 on Gamma and
# eps_z = eps_layers h_l / r_z on Z; every node of the subdomain's own discrete grid boundary
# must fall in gamma_l or zeta_l (checked); one zonal expansion on the whole of Gamma (shared
# by gamma_1 and gamma_2) and one on Z (shared by zeta_1 and zeta_2, 3-term, as in Case 1).
# A node of gamma_l cap zeta_l carries the average of its two densities (the effective density)
# in the difference potential, and two equations of the reduced BEP (one per density), in the
# order Gamma row, then Z row; rows follow gamma_in of the subdomain in ascending index.
# ---------------------------------------------------------------------------------------------


def _gamma_of(mask: np.ndarray) -> np.ndarray:
    return PointSets(mask).gamma


class DDCase2:
    """Grids, point sets, parts and effective densities of the two subdomains of Case 2."""

    def __init__(self, n1: int, half1: float, zc1: float, n2: int, q_z: float, r_z: float,
                 m_gamma: int, m_z: int, beta: int = 0, eps_layers: float = 2.0,
                 rcond: float | None = None):
        self.q_z, self.r_z = q_z, r_z
        # least squares of the coupled BEPs: None plain, > 0 truncated minimum norm (dpm.least_squares)
        self.rcond = rcond
        self.n1, self.n2 = n1, n2
        self.m_gamma, self.m_z, self.beta = m_gamma, m_z, beta
        self.n_gamma_cols = (beta + 1) * (m_gamma + 1)
        self.n_z_cols = 3 * (m_z + 1)
        self.n_cols = self.n_gamma_cols + self.n_z_cols
        # the circle where Z meets Gamma: |x| = 1 and |x - q| = r_z
        z_star = (1.0 + q_z * q_z - r_z * r_z) / (2.0 * q_z)
        self.theta_star = float(np.arccos(z_star))
        self.psi_star = float(np.arccos((q_z - z_star) / r_z))
        self.sub = []
        for l, (n, half, zc) in enumerate(((n1, half1, zc1), (n2, inp.HALF_WIDTH, 0.0))):
            h, x0 = inp.grid(n, half)
            z, y, x = inp.mesh(n, half)
            z = z + zc
            r2 = x * x + y * y + z * z
            q2 = x * x + y * y + (z - q_z) * (z - q_z)
            ball = r2 < 1.0
            zin = q2 < r_z * r_z if l == 0 else q2 > r_z * r_z
            ps = PointSets(ball & zin)
            g_ball = _gamma_of(ball).ravel()[ps.idx]
            g_z = _gamma_of(zin).ravel()[ps.idx]
            gx, gy, gz = x.ravel()[ps.idx], y.ravel()[ps.idx], z.ravel()[ps.idx]
            rho = np.sqrt(gx * gx + gy * gy)
            rr = np.sqrt(gx * gx + gy * gy + gz * gz)
            theta = np.arctan2(rho, gz)
            rq = np.sqrt(gx * gx + gy * gy + (gz - q_z) * (gz - q_z))
            psi = np.arctan2(rho, q_z - gz)
            eps_g, eps_z = eps_layers * h, eps_layers * h / r_z
            win_g = theta <= self.theta_star + eps_g if l == 0 else theta >= self.theta_star - eps_g
            in_g = g_ball & win_g
            in_z = g_z & (psi <= self.psi_star + eps_z)
            cover = in_g | in_z
            k = in_g.astype(float) + in_z.astype(float)
            w = np.where(cover, 1.0 / np.maximum(k, 1.0), 0.0)
            bg = zonal_basis_matrix(rr - 1.0, theta, m_gamma, beta)
            dz = rq - r_z
            p = zonal_basis_matrix(dz, psi, m_z, 0)
            bz = np.concatenate([p, dz[None, :] * p, 0.5 * dz[None, :] ** 2 * p], axis=0)
            B_eff = np.concatenate([bg * (in_g * w)[None, :], bz * (in_z * w)[None, :]], axis=0)
            # reduced-BEP rows of this subdomain: (position in gamma_in, part)
            pos_in = np.flatnonzero(ps.is_in)
            rows = []
            for i, j in enumerate(pos_in):
                if in_g[j]:
                    rows.append((i, 0))
                if in_z[j]:
                    rows.append((i, 1))
            self.sub.append(dict(
                h=h, x0=x0, zc=zc, mesh=(z, y, x), ps=ps, in_g=in_g, in_z=in_z, cover=cover,
                theta=theta, psi=psi, eps_g=eps_g, eps_z=eps_z, bg=bg, bz=bz, B_eff=B_eff,
                rows=np.array(rows, dtype=np.int64).reshape(-1, 2)))

    @property
    def covered(self) -> bool:
        return all(bool(s["cover"].all()) for s in self.sub)


def dd2_matrix(case: DDCase2, sigma: float) -> np.ndarray:
    """The coupled reduced BEPs of Case 2, rows [Omega_1's ; Omega_2's], columns [C ; A].
    A row of part Gamma at node p: phi^Gamma_nu(p) on the Gamma columns (zero on the Z columns)
    minus Tr_p P (effective density of column nu); part Z likewise."""
    blocks = []
    ng = case.n_gamma_cols
    for s in case.sub:
        ps = s["ps"]
        pos_in = np.flatnonzero(ps.is_in)
        PT = np.empty((ps.n_gamma_in, case.n_cols))
        for nu in range(case.n_cols):
            PT[:, nu] = trace(difference_potential(s["B_eff"][nu], ps, sigma, s["h"]), ps.idx_in)
        A = np.empty((len(s["rows"]), case.n_cols))
        for r, (i, part) in enumerate(s["rows"]):
            own = np.zeros(case.n_cols)
            j = pos_in[i]
            if part == 0:
                own[:ng] = s["bg"][:, j]
            else:
                own[ng:] = s["bz"][:, j]
            A[r] = own - PT[i]
        blocks.append(A)
    return np.concatenate(blocks, axis=0)


def dd2_step(rho1, c1, rho2, c2, case: DDCase2, A: np.ndarray, dt: float, chi: float):
    """One step on both subdomains of Case 2 (sigma = 1/dt); returns the four new states (each
    on its N+, zero elsewhere) and the coefficients of both species."""
    sigma = 1.0 / dt
    s1, s2 = case.sub
    f1r, f1c = pks_rhs(rho1, c1, s1["ps"].m_plus, s1["h"], dt, chi)
    f2r, f2c = pks_rhs(rho2, c2, s2["ps"].m_plus, s2["h"], dt, chi)
    out, coefs = [], []
    for f1, f2 in ((f1r, f2r), (f1c, f2c)):
        G = [particular_solution(f, s["ps"], sigma, s["h"]) for f, s in ((f1, s1), (f2, s2))]
        g = np.concatenate([trace(Gl, s["ps"].idx_in)[s["rows"][:, 0]] for Gl, s in zip(G, case.sub)])
        C = least_squares(A, g, case.rcond)
        u = []
        for Gl, s in zip(G, case.sub):
            ug = s["B_eff"].T @ C
            u.append(np.where(s["ps"].n_plus, difference_potential(ug, s["ps"], sigma, s["h"]) + Gl, 0.0))
        out.append(u)
        coefs.append(C)
    (r1, r2), (cc1, cc2) = out
    return r1, cc1, r2, cc2, coefs


def dd_adaptive_run(state, case, sigma0: float, chi: float, t_final: float,
                    rho_cap: float = np.inf, max_steps: int = 1000, rho_jump_cap: float = 0.0):
    """Steps 3-8 on the decomposed domain (either case) from dt_0 = 1/sigma0: each subdomain's
    CFL-type bound on its own mesh, dt the smallest of them and of the previous dt, Step 4b (a new
    coupled matrix) when dt shrinks, Step 8 on max |rho| over both M+.  state = (rho_1, c_1,
    rho_2, c_2).  Returns (state, summary) with the keys of pks.adaptive_run."""
    from .pks import cfl_dt
    if isinstance(case, DDCase2):
        subs = [(s["ps"], s["h"]) for s in case.sub]
        matrix, step = dd2_matrix, dd2_step
    else:
        subs = [(case.ps1, case.h1), (case.ps2, case.h2)]
        matrix, step = dd_matrix, dd_step
    state = list(state)
    dt_prev = 1.0 / sigma0
    A = matrix(case, sigma0)                                               # Step 2
    t, dts, rebuilt, stop = 0.0, [], [], "max_steps"
    rmax = rprev = 0.0
    while True:
        if t >= t_final:
            stop = "t_final"
            break
        if len(dts) >= max_steps:
            stop = "max_steps"
            break
        vals = [float(np.max(np.where(ps.m_plus, np.abs(state[2 * l]), 0.0)))
                for l, (ps, h) in enumerate(subs)]
        cfls = [cfl_dt(state[2 * l + 1], ps.m_plus, h, chi) for l, (ps, h) in enumerate(subs)]
        rmax = max(vals)
        if not all(np.isfinite(v) for v in vals) or any(np.isnan(x) for x in cfls):
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
        dt = min(min(cfls), dt_prev)                                       # Step 3
        rb = dt < dt_prev
        if rb:                                                             # Step 4b
            A = matrix(case, 1.0 / dt)
        state = list(step(*state, case, A, dt, chi)[:4])                   # Steps 4a-7
        dts.append(dt)
        rebuilt.append(rb)
        t += dt
        dt_prev = dt
    return state, {"steps": len(dts), "rebuilds": int(sum(rebuilt)), "stop": stop, "t": t,
                   "dt": dt_prev, "rho_max": rmax, "dt_hist": dts, "rebuilt": rebuilt}
