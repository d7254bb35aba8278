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
