"""Pins of the domain-decomposition oracle (oracle/dd.py), Case 1: Omega_1 = {|x| < 0.5} on its
own cube (half-width 0.75), Omega_2 = {0.5 < |x| < 1} on the full cube, both meshes with the same
spacing and aligned nodes, so the DD step can be compared with the single-domain step node by
node.

- A constant state is an exact discrete solution (P_0 on both surfaces represents it).
- Data symmetric about the origin keep the symmetries that zonal densities preserve.
- The DD and single-domain steps approximate the same problem: without convection (chi = 0) their
  difference falls at second order as both meshes are refined together (the coupled BEP and the
  interface extension are consistent).
"""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import basis as ob
from oracle import dd
from oracle import dpm
from oracle import geometry as og
from oracle import pks


def _data(mesh, ps):
    z, y, x = mesh
    r2 = x * x + y * y + z * z
    return np.where(ps.n_plus, 10 * np.exp(-2 * r2), 0.0), np.where(ps.n_plus, 5 * np.exp(-r2), 0.0)


@pytest.fixture(scope="module")
def small():
    case = dd.DDCase(15, 0.75, 31, 0.5, 2, 2, beta=1)
    assert case.ps1.margin_ok and case.ps2.margin_ok
    assert case.h1 == case.h2
    return case


def test_dd_constant_state(small):
    case = small
    dt = 0.5 * case.h2**2
    A = dd.dd_matrix(case, 1.0 / dt)
    r1 = np.where(case.ps1.n_plus, 3.0, 0.0)
    c1 = np.where(case.ps1.n_plus, 5.0, 0.0)
    r2 = np.where(case.ps2.n_plus, 3.0, 0.0)
    c2 = np.where(case.ps2.n_plus, 5.0, 0.0)
    o1, oc1, o2, oc2, _ = dd.dd_step(r1, c1, r2, c2, case, A, dt, 1.0)
    cn = (1 - dt) * 5.0 + dt * 3.0
    assert np.allclose(o1[case.ps1.n_plus], 3.0, rtol=1e-12)
    assert np.allclose(o2[case.ps2.n_plus], 3.0, rtol=1e-12)
    assert np.allclose(oc1[case.ps1.n_plus], cn, rtol=1e-12)
    assert np.allclose(oc2[case.ps2.n_plus], cn, rtol=1e-12)
    assert np.all(o1[~case.ps1.n_plus] == 0) and np.all(o2[~case.ps2.n_plus] == 0)


def test_dd_symmetry(small):
    case = small
    dt = 1e-3
    A = dd.dd_matrix(case, 1.0 / dt)
    r1, c1 = _data(case.mesh1, case.ps1)
    r2, c2 = _data(case.mesh2, case.ps2)
    out = dd.dd_step(r1, c1, r2, c2, case, A, dt, 1.0)
    for f in out[:4]:
        tol = 1e-12 * np.abs(f).max()
        assert np.max(np.abs(f - f[:, :, ::-1])) < tol      # x -> -x
        assert np.max(np.abs(f - f[:, ::-1, :])) < tol      # y -> -y
        assert np.max(np.abs(f - f[::-1])) < tol            # z -> -z (P_nu of both parities)
        assert np.max(np.abs(f - np.transpose(f, (0, 2, 1)))) < tol   # x <-> y


def _dd_minus_sd(n1, n2, chi):
    case = dd.DDCase(n1, 0.75, n2, 0.5, 2, 2, beta=1)
    dt = 1e-3
    A = dd.dd_matrix(case, 1.0 / dt)
    r1, c1 = _data(case.mesh1, case.ps1)
    r2, c2 = _data(case.mesh2, case.ps2)
    o = dd.dd_step(r1, c1, r2, c2, case, A, dt, chi)
    h, x0 = inp.grid(n2)
    z, y, x = inp.mesh(n2)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, _ = og.project_sphere(gz, gy, gx)
    B = ob.zonal_basis_matrix(d, th, 2, 1)
    rs, cs = _data((z, y, x), ps)
    rsd, csd, _ = pks.dpm_step(rs, cs, ps, B, dpm.bep_matrix(B, ps, 1 / dt, h), h, dt, chi)
    k = (n2 - n1) // 2
    sl = (slice(k, k + n1),) * 3
    m1, m2 = case.ps1.m_plus, case.ps2.m_plus
    return [np.max(np.abs(o[0][m1] - rsd[sl][m1])) / np.abs(rsd).max(),
            np.max(np.abs(o[2][m2] - rsd[m2])) / np.abs(rsd).max(),
            np.max(np.abs(o[1][m1] - csd[sl][m1])) / np.abs(csd).max(),
            np.max(np.abs(o[3][m2] - csd[m2])) / np.abs(csd).max()]


def test_dd_converges_to_single_domain():
    coarse = _dd_minus_sd(15, 31, 0.0)
    fine = _dd_minus_sd(31, 63, 0.0)
    for a, b in zip(coarse, fine):
        assert a < 1e-4 and a / b > 2.5, (a, b)


# ---- Case 2: Z (radius 0.5 about the north pole q = (0, 0, 1)) meets Gamma -------------------

def _data2(mesh, ps):
    z, y, x = mesh
    r2 = x * x + y * y + (z - 0.5) ** 2
    return np.where(ps.n_plus, 10 * np.exp(-2 * r2), 0.0), np.where(ps.n_plus, 5 * np.exp(-r2), 0.0)


@pytest.fixture(scope="module")
def small2():
    case = dd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0)
    assert all(s["ps"].margin_ok for s in case.sub)
    return case


def test_dd2_parts_cover_the_discrete_boundaries(small2):
    """The wedge angles follow from the two radii, every node of each subdomain's discrete
    boundary falls in gamma_l or zeta_l, the wedge carries nodes in both, and the part decisions
    are far from rounding ties."""
    case = small2
    assert np.isclose(np.cos(case.theta_star), 0.875) and np.isclose(np.cos(case.psi_star), 0.25)
    assert case.covered
    for l, s in enumerate(case.sub):
        both = s["in_g"] & s["in_z"]
        assert 0 < both.sum() < 0.5 * s["cover"].sum()
        edge = case.theta_star + (s["eps_g"] if l == 0 else -s["eps_g"])
        assert np.min(np.abs(s["theta"] - edge)) > 1e-4
        assert np.min(np.abs(s["psi"] - (case.psi_star + s["eps_z"]))) > 1e-4
        # effective densities: the average of the two at the wedge nodes
        j = np.flatnonzero(both)[0]
        assert np.allclose(s["B_eff"][: case.n_gamma_cols, j], 0.5 * s["bg"][:, j])
        assert np.allclose(s["B_eff"][case.n_gamma_cols:, j], 0.5 * s["bz"][:, j])
        # one BEP row per part: wedge nodes of gamma_in carry two
        n_in_both = int((both & s["ps"].is_in).sum())
        assert len(s["rows"]) == s["ps"].n_gamma_in + n_in_both


def test_dd2_constant_state(small2):
    case = small2
    dt = 0.5 * case.sub[1]["h"] ** 2
    A = dd.dd2_matrix(case, 1.0 / dt)
    st = []
    for s in case.sub:
        st += [np.where(s["ps"].n_plus, 3.0, 0.0), np.where(s["ps"].n_plus, 5.0, 0.0)]
    out = dd.dd2_step(*st, case, A, dt, 1.0)
    cn = (1 - dt) * 5.0 + dt * 3.0
    for (r, c), s in ((out[:2], case.sub[0]), (out[2:4], case.sub[1])):
        assert np.allclose(r[s["ps"].n_plus], 3.0, rtol=1e-11)
        assert np.allclose(c[s["ps"].n_plus], cn, rtol=1e-11)


def test_dd2_axial_symmetry(small2):
    case = small2
    dt = 1e-3
    A = dd.dd2_matrix(case, 1.0 / dt)
    st = []
    for s in case.sub:
        st += list(_data2(s["mesh"], s["ps"]))
    out = dd.dd2_step(*st, case, A, dt, 1.0)
    for f in out[:4]:
        tol = 1e-11 * np.abs(f).max()
        assert np.max(np.abs(f - f[:, :, ::-1])) < tol
        assert np.max(np.abs(f - f[:, ::-1, :])) < tol
        assert np.max(np.abs(f - np.transpose(f, (0, 2, 1)))) < tol


def _dd2_minus_sd(n1, n2, chi):
    case = dd.DDCase2(n1, 0.75, 0.75, n2, 1.0, 0.5, 4, 4, beta=0)
    dt = 1e-3
    A = dd.dd2_matrix(case, 1.0 / dt)
    s1, s2 = case.sub
    st = list(_data2(s1["mesh"], s1["ps"])) + list(_data2(s2["mesh"], s2["ps"]))
    o = dd.dd2_step(*st, case, A, dt, chi)
    h, x0 = inp.grid(n2)
    z, y, x = inp.mesh(n2)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, _ = og.project_sphere(gz, gy, gx)
    B = ob.zonal_basis_matrix(d, th, 4, 0)
    rs, cs = _data2((z, y, x), ps)
    rsd, csd, _ = pks.dpm_step(rs, cs, ps, B, dpm.bep_matrix(B, ps, 1 / dt, h), h, dt, chi)
    # Omega_1's cube [-0.75, 0.75]^2 x [0, 1.5]: its nodes are Omega_2's, shifted
    kz, kx = int(round(1.5 / h)), (n2 - n1) // 2
    sl = (slice(kz, kz + n1), slice(kx, kx + n1), slice(kx, kx + n1))
    m1, m2 = s1["ps"].m_plus, s2["ps"].m_plus
    assert np.array_equal(s1["mesh"][0][m1], z[sl][m1])
    return [np.max(np.abs(o[0][m1] - rsd[sl][m1])) / np.abs(rsd).max(),
            np.max(np.abs(o[2][m2] - rsd[m2])) / np.abs(rsd).max(),
            np.max(np.abs(o[1][m1] - csd[sl][m1])) / np.abs(csd).max(),
            np.max(np.abs(o[3][m2] - csd[m2])) / np.abs(csd).max()]


def test_dd2_converges_to_single_domain():
    """The decomposed and single-domain steps approximate the same problem: their difference,
    dominated by the wedge, falls by more than 3.5x per halving of h (with convection)."""
    coarse = _dd2_minus_sd(15, 31, 1.0)
    fine = _dd2_minus_sd(31, 63, 1.0)
    for a, b in zip(coarse, fine):
        assert b < 2e-3 and a / b > 3.5, (a, b)


def test_dd2_least_squares_well_posed_at_test_sizes(small2):
    """The coupled least squares of the Case 2 configurations the GPU tests use is well posed:
    LAPACK's solution and a Householder QR's give the same step to 1e-10 (with too many harmonics
    on Z's partial arc they do not, even when the rank test passes)."""
    from scipy.linalg import solve_triangular
    case = small2
    dt = 1e-3
    A = dd.dd2_matrix(case, 1 / dt)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(A.shape[0])
    c1 = np.linalg.lstsq(A, g, rcond=None)[0]
    q, r = np.linalg.qr(A)
    c2 = solve_triangular(r, q.T @ g)
    for s in case.sub:
        u1, u2 = s["B_eff"].T @ c1, s["B_eff"].T @ c2
        assert np.max(np.abs(u1 - u2)) <= 1e-10 * np.max(np.abs(u1))


def test_dd2_truncated_least_squares_with_twenty_harmonics_on_z():
    """The paper's 20 harmonics per term on Z make the coupled matrix of Case 2 numerically rank
    deficient (singular values fall smoothly to 1e-19 of the largest).  With the truncated
    minimum-norm reading (rcond = 1e-7, inside the gap 3.4e-7 -> 4.1e-8 of this configuration) two
    different SVD-based LAPACK solvers, gelsd (numpy) and gelss (scipy), give the same densities
    to 1e-9.  The constant state is a consistent right-hand side; truncation keeps it to the
    level of the dropped singular values, not to rounding (1e-5 relative; measured 2.8e-7 on
    Omega_1 and 1.4e-6 on Omega_2, against 1e-11 untruncated)."""
    from scipy.linalg import lstsq as sp_lstsq
    case = dd.DDCase2(31, 0.75, 0.75, 31, 1.0, 0.5, 19, 19, beta=0, rcond=1e-7)
    dt = 1e-3
    A = dd.dd2_matrix(case, 1 / dt)
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[-1] < 1e-15 * sv[0]  # rank deficient without truncation
    rng = np.random.default_rng(5)
    g = rng.standard_normal(A.shape[0])
    c1 = dpm.least_squares(A, g, case.rcond)
    c2 = sp_lstsq(A, g, cond=case.rcond, lapack_driver="gelss")[0]
    for s in case.sub:
        u1, u2 = s["B_eff"].T @ c1, s["B_eff"].T @ c2
        assert np.max(np.abs(u1 - u2)) <= 1e-9 * np.max(np.abs(u1))
    st = []
    for s in case.sub:
        st += [np.where(s["ps"].n_plus, 3.0, 0.0), np.where(s["ps"].n_plus, 5.0, 0.0)]
    out = dd.dd2_step(*st, case, A, dt, 1.0)
    for (r, _), s in ((out[:2], case.sub[0]), (out[2:4], case.sub[1])):
        assert np.max(np.abs(r[s["ps"].n_plus] - 3.0)) <= 3e-5
