"""Pins of the point sets, projections and basis (oracle/geometry.py, oracle/basis.py).

Paper: Def. "point sets" (Sec. 2); extension operator and spherical-harmonic expansion
(Sec. 2, "Spectral Approach").
"""
import itertools

import numpy as np
import pytest

import dpm_inputs as inp
from oracle import basis as ob
from oracle import geometry as og

STENCIL = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def _bruteforce_sets(m_plus):
    """Literal set algebra with Python sets over padded coordinates (ghosts included)."""
    n = m_plus.shape[0]
    M0 = {(z, y, x) for z in range(1, n + 1) for y in range(1, n + 1) for x in range(1, n + 1)}
    Mp = {(z + 1, y + 1, x + 1) for z, y, x in zip(*np.nonzero(m_plus))}
    Mm = M0 - Mp

    def N(S):
        return {(z + a, y + b, x + c) for (z, y, x) in S for (a, b, c) in STENCIL}

    gamma = N(Mp) & N(Mm)
    return gamma, gamma & Mp, gamma & Mm


@pytest.mark.parametrize("n,radius,shape", [(7, 1.0, "sphere"), (9, 1.1, "sphere"), (11, 1.0, "ellipsoid")])
def test_point_sets_bruteforce(n, radius, shape):
    z, y, x = inp.mesh(n)
    if shape == "sphere":
        mp = og.inside_sphere(z, y, x, radius=radius)
    else:
        mp = og.inside_ellipsoid(z, y, x)
    ps = og.PointSets(mp)
    gamma, gin, gex = _bruteforce_sets(mp)
    lin = lambda p: ((p[0] - 1) * n + (p[1] - 1)) * n + (p[2] - 1)
    assert sorted(lin(p) for p in gamma) == list(ps.idx)
    assert sorted(lin(p) for p in gin) == list(ps.idx_in)
    assert sorted(lin(p) for p in gex) == sorted(set(ps.idx) - set(ps.idx_in))
    assert ps.margin_ok


def test_gamma_neighbour_characterisation():
    """gamma_in = M+ nodes with an M- neighbour; gamma_ex = M- nodes with an M+ neighbour."""
    n = 31
    z, y, x = inp.mesh(n)
    mp = og.inside_sphere(z, y, x)
    ps = og.PointSets(mp)
    P = np.pad(mp, 1, constant_values=False)
    nb_minus = np.zeros_like(mp)
    nb_plus = np.zeros_like(mp)
    for a, b, c in STENCIL[1:]:
        sl = P[1 + a:n + 1 + a, 1 + b:n + 1 + b, 1 + c:n + 1 + c]
        nb_plus |= sl
        inner_m = ~sl
        # ghosts are not in M-: mask them out
        gz = np.arange(n)[:, None, None] + a
        gy = np.arange(n)[None, :, None] + b
        gx = np.arange(n)[None, None, :] + c
        inside = (gz >= 0) & (gz < n) & (gy >= 0) & (gy < n) & (gx >= 0) & (gx < n)
        nb_minus |= inner_m & inside
    assert np.array_equal(ps.gamma_in, mp & nb_minus)
    assert np.array_equal(ps.gamma_ex, ~mp & nb_plus)
    # the reduced BEP has about half of the rows of the full one (remark after Thm "reduced BEP")
    assert 0.4 < ps.n_gamma_in / ps.n_gamma < 0.6


def test_margin_violation_detected():
    n = 15
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x, radius=1.45))
    assert not ps.margin_ok


def test_sphere_projection_closed_form():
    pts = np.array([[0.3, -0.2, 1.1], [0.0, 0.0, -0.9], [1.05, 0.0, 0.0], [-0.5, 0.6, 0.7]])
    x, y, z = pts.T
    d, th, ph = og.project_sphere(z, y, x, radius=1.0)
    r = np.linalg.norm(pts, axis=1)
    assert np.allclose(d, r - 1.0)
    back = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    assert np.allclose(back * (r[:, None]), pts)


def test_ellipsoid_projection_properties():
    axes = (1.0, 0.8, 0.6)
    rng = np.random.default_rng(1)
    # random points near the surface
    u = rng.normal(size=(40, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    surf = u * np.array(axes)
    pts = surf * (1.0 + rng.uniform(-0.05, 0.05, size=(40, 1)))
    x, y, z = pts.T
    d, th, ph = og.project_ellipsoid(z, y, x, axes=axes)
    a = np.array(axes)
    q = np.stack([a[0] * np.sin(th) * np.cos(ph), a[1] * np.sin(th) * np.sin(ph), a[2] * np.cos(th)], 1)
    # foot point on the surface, |p - q| = |d|, and p - q along the normal grad(q^2/a^2) ~ q/a^2
    assert np.allclose(np.sum(q * q / a**2, 1), 1.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(pts - q, axis=1), np.abs(d), atol=1e-12)
    nrm = q / a**2
    cross = np.cross(pts - q, nrm)
    assert np.max(np.abs(cross)) < 1e-12
    outside = np.sum(pts * pts / a**2, 1) > 1
    assert np.all((d > 0) == outside)
    # brute force: no sampled surface point is closer
    tt, pp = np.meshgrid(np.linspace(0, np.pi, 400), np.linspace(-np.pi, np.pi, 800), indexing="ij")
    S = np.stack([a[0] * np.sin(tt) * np.cos(pp), a[1] * np.sin(tt) * np.sin(pp), a[2] * np.cos(tt)], -1).reshape(-1, 3)
    for p, dd in zip(pts[:8], d[:8]):
        assert np.min(np.linalg.norm(S - p, axis=1)) >= abs(dd) - 1e-12


def test_ellipsoid_with_equal_axes_is_sphere():
    rng = np.random.default_rng(2)
    pts = rng.uniform(-1.2, 1.2, size=(30, 3))
    x, y, z = pts.T
    d1, t1, p1 = og.project_sphere(z, y, x, radius=0.9)
    d2, t2, p2 = og.project_ellipsoid(z, y, x, axes=(0.9, 0.9, 0.9))
    assert np.allclose(d1, d2, atol=1e-12) and np.allclose(t1, t2, atol=1e-10)
    assert np.allclose(np.cos(p1 - p2), 1.0, atol=1e-12)


def test_real_harmonics_closed_forms():
    th = np.array([0.3, 1.1, 2.0, 2.9])
    ph = np.array([-2.5, -0.4, 0.7, 3.0])
    c, s = np.cos(th), np.sin(th)
    k1 = np.sqrt(3 / (4 * np.pi))
    table = {
        (0, 0): np.full_like(th, 0.5 / np.sqrt(np.pi)),
        (1, -1): k1 * s * np.sin(ph),
        (1, 0): k1 * c,
        (1, 1): k1 * s * np.cos(ph),
        (2, 0): np.sqrt(5 / (16 * np.pi)) * (3 * c**2 - 1),
        (2, 1): np.sqrt(15 / (4 * np.pi)) * s * c * np.cos(ph),
        (2, -2): np.sqrt(15 / (16 * np.pi)) * s**2 * np.sin(2 * ph),
    }
    for (l, m), ref in table.items():
        assert np.allclose(ob.real_sph_harm(l, m, th, ph), ref, atol=1e-14), (l, m)


def test_real_harmonics_orthonormal():
    L = 10
    xg, wg = np.polynomial.legendre.leggauss(L + 2)
    nphi = 2 * L + 3
    ph = 2 * np.pi * np.arange(nphi) / nphi
    TH, PH = np.meshgrid(np.arccos(xg), ph, indexing="ij")
    W = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    Y = np.array([ob.real_sph_harm(l, m, TH.ravel(), PH.ravel()) for (l, m) in ob.lm_list(L)])
    G = (Y * W) @ Y.T
    assert np.max(np.abs(G - np.eye(len(Y)))) < 1e-12


def test_basis_matrix_layout():
    d = np.array([0.1, -0.2, 0.05])
    th = np.array([0.5, 1.5, 2.5])
    ph = np.array([0.0, 1.0, -1.0])
    B = ob.basis_matrix(d, th, ph, lmax=2, beta=1)
    assert B.shape == (18, 3)
    assert np.allclose(B[9:], 0.5 * d**2 * B[:9])
    assert np.allclose(B[4], ob.real_sph_harm(2, -2, th, ph))


def test_zonal_basis_closed_forms_and_endpoints():
    th = np.array([0.0, 0.4, 1.3, 2.2, np.pi])
    x = np.cos(th)
    d = np.array([0.1, -0.05, 0.2, 0.0, -0.3])
    B = ob.zonal_basis_matrix(d, th, 3, beta=1)
    ref = [np.ones_like(x), x, 0.5 * (3 * x**2 - 1), 0.5 * (5 * x**3 - 3 * x)]
    assert B.shape == (8, 5)
    for nu in range(4):
        assert np.allclose(B[nu], ref[nu], atol=1e-15)
        assert np.allclose(B[4 + nu], 0.5 * d**2 * ref[nu], atol=1e-15)
    # P_nu(1) = 1 and P_nu(-1) = (-1)^nu up to the degrees of the paper's Test B
    P = ob.zonal_basis_matrix(np.zeros(2), np.array([0.0, np.pi]), 499, beta=0)
    assert np.allclose(P[:, 0], 1.0, atol=1e-12)
    assert np.allclose(P[:, 1], (-1.0) ** np.arange(500), atol=1e-12)


def test_zonal_basis_orthogonal_and_matches_real_harmonics():
    """int_{-1}^{1} P_l P_m dx = 2/(2l+1) delta_lm (Gauss-Legendre, exact for these degrees), and
    P_l(cos theta) = sqrt(4 pi/(2l+1)) Y_l0 from the independent spherical-harmonic routine."""
    L = 300
    xg, wg = np.polynomial.legendre.leggauss(L + 2)
    P = ob.zonal_basis_matrix(np.zeros_like(xg), np.arccos(xg), L, beta=0)
    G = (P * wg) @ P.T
    assert np.max(np.abs(G - np.diag(2.0 / (2 * np.arange(L + 1) + 1)))) < 1e-12
    th = np.linspace(0.05, 3.1, 9)
    Z = ob.zonal_basis_matrix(np.zeros_like(th), th, 10, beta=0)
    for l in range(11):
        y = ob.real_sph_harm(l, 0, th, np.zeros_like(th))
        assert np.allclose(Z[l], np.sqrt(4 * np.pi / (2 * l + 1)) * y, atol=1e-13), l
