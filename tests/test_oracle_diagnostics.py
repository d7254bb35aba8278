"""Pins of the run diagnostics (oracle/diagnostics.py; Sec. 4, "Error metrics and quantities of
interest"): Gaussian data inside the unit ball, whose sums on the grid approach closed-form
integrals (spectrally for the pointwise terms, at second order for the central-difference
gradient term), the exact maximum at the centre node, and the decomposed domain's sums equal to
the single domain's on aligned meshes."""
import math

import numpy as np
import pytest

import dpm_inputs as inp
from oracle import dd as odd
from oracle import diagnostics as dg
from oracle import geometry as og

A, B = 7.0, 20.0      # rho = A exp(-B r^2): below 2e-9 of its peak on the boundary
A2, B2 = 3.0, 15.0    # c = A2 exp(-B2 r^2)


def _closed_forms():
    pi32 = math.pi ** 1.5
    moment = 1.5 * A * pi32 * B ** -2.5
    mass = A * (math.pi / B) ** 1.5
    rho_ln_rho = mass * math.log(A) - A * B * 1.5 * pi32 * B ** -2.5
    rho_c = A * A2 * (math.pi / (B + B2)) ** 1.5
    c2 = 0.5 * A2 * A2 * (math.pi / (2 * B2)) ** 1.5
    grad = 0.5 * 4 * A2 * A2 * B2 * B2 * 1.5 * pi32 * (2 * B2) ** -2.5
    return moment, rho_ln_rho - rho_c + c2 + grad, grad


def _fields(n):
    h, _ = inp.grid(n)
    z, y, x = inp.mesh(n)
    r2 = x * x + y * y + z * z
    mp = og.inside_sphere(z, y, x)
    return A * np.exp(-B * r2), A2 * np.exp(-B2 * r2), mp, h, (z, y, x)


def test_diagnostics_against_closed_forms():
    moment, energy, grad = _closed_forms()
    errs = []
    for n in (63, 127):
        rho, c, mp, h, mesh = _fields(n)
        mx, m2, e = dg.diagnostics(rho, c, mp, h, mesh)
        assert mx == A                                   # the centre is a node (N odd)
        # trapezoidal sums of a Gaussian: what is left is the part beyond the ball (1.5e-7)
        assert abs(m2 - moment) <= 5e-7 * moment
        errs.append(abs(e - energy))
    # the free energy's error is the central-difference gradient term's, second order in h
    assert errs[0] < 0.05 * grad and 3.8 < errs[0] / errs[1] < 4.2, errs


def test_free_energy_terms_and_nonpositive_density():
    """Constant rho = a, c = b on M+: E = |M+| h^3 (a ln a - a b + b^2/2) (no gradient inside, and
    the cube's edges are not reached); rho ln rho is 0 for rho <= 0 (a rounding-level negative
    rho still enters -rho c); a NaN rho gives NaN."""
    n = 31
    h, _ = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    a, b = 2.5, 0.75
    rho = np.where(ps.n_plus, a, 0.0)
    c = np.where(ps.n_plus, b, 0.0)
    e = dg.free_energy(rho, c, ps.m_plus, h)
    vol = ps.m_plus.sum() * h**3
    assert np.isclose(e, vol * (a * math.log(a) - a * b + 0.5 * b * b), rtol=1e-13)
    assert dg.free_energy(np.zeros_like(rho), c, ps.m_plus, h) == pytest.approx(vol * 0.5 * b * b, rel=1e-13)
    k = tuple(v[0] for v in ps.m_plus.nonzero())
    rho[k] = -1e-17
    e2 = dg.free_energy(rho, c, ps.m_plus, h)
    assert np.isclose(e2, e - h**3 * (a * math.log(a) - a * b) + h**3 * 1e-17 * b, rtol=1e-13)
    rho[k] = np.nan
    assert math.isnan(dg.free_energy(rho, c, ps.m_plus, h))


def test_decomposed_sums_equal_single_domain():
    """Ball r < 0.5 at N = 15 on [-0.75, 0.75]^3 and the shell at N = 31 share the single domain's
    nodes (no node lies on Z): the same sampled fields give the single domain's diagnostics."""
    case = odd.DDCase(15, 0.75, 31, 0.5, 0, 0, 1)
    parts = []
    for ps, h, mesh in ((case.ps1, case.h1, case.mesh1), (case.ps2, case.h2, case.mesh2)):
        z, y, x = mesh
        r2 = x * x + y * y + z * z
        parts.append((A * np.exp(-B * r2), A2 * np.exp(-B2 * r2), ps.m_plus, h, mesh))
    rho, c, mp, h, mesh = _fields(31)
    sd = dg.diagnostics(rho, c, mp, h, mesh)
    dd = dg.dd_diagnostics(parts)
    assert dd[0] == sd[0]
    assert np.allclose(dd[1:], sd[1:], rtol=1e-13, atol=0)
