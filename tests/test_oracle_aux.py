"""Pins of the AP oracle (oracle/aux.py) against mathematics that does not use its code path.

Paper: the AP (Sec. 2, eqs discrete_ap / discrete_ap_boundary) with the 7-point Laplacian
(eq stencil:7-point; coefficients in the proof of the positivity theorem).
"""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import aux


def _assembled_matrix(n, sigma, h):
    """(sigma I - Lap_h) assembled node by node from the stencil, zero Dirichlet ghosts."""
    N = n**3
    A = np.zeros((N, N))

    def lin(z, y, x):
        return (z * n + y) * n + x

    for z in range(n):
        for y in range(n):
            for x in range(n):
                r = lin(z, y, x)
                A[r, r] = sigma + 6.0 / h**2
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    zz, yy, xx = z + dz, y + dy, x + dx
                    if 0 <= zz < n and 0 <= yy < n and 0 <= xx < n:
                        A[r, lin(zz, yy, xx)] = -1.0 / h**2
    return A


@pytest.mark.parametrize("n", [1, 2, 4, 7, 15, 16])
def test_dst_matrix_symmetric_orthogonal(n):
    S = aux.dst1_matrix(n)
    assert np.allclose(S, S.T, atol=0)
    assert np.max(np.abs(S @ S - np.eye(n))) < 1e-14


@pytest.mark.parametrize("sigma", [0.0, 1.0, 35.0 / 3.0, 1e4])
def test_bruteforce_dense_solve_7(sigma):
    n = 7
    h, _ = inp.grid(n)
    A = _assembled_matrix(n, sigma, h)
    b = inp.rhs_normal(n, 1, seed=3)[0]
    u_ref = np.linalg.solve(A, b.ravel()).reshape(n, n, n)
    u = aux.aux_solve(b, sigma, h)
    assert aux.rel_err_inf(u, u_ref) < 1e-13
    # the stencil application equals the assembled matrix
    assert np.max(np.abs(aux.apply_operator(b, sigma, h).ravel() - A @ b.ravel())) < 1e-10


@pytest.mark.parametrize("n", [7, 15, 31, 63])
def test_eigenmodes_closed_form(n):
    """b = s_k1 (x) s_k2 (x) s_k3 with s_k(j) = sin(pi j k/(n+1)) gives u = b / (sigma + sum lambda)."""
    h, _ = inp.grid(n)
    sigma = 2.5
    j = np.arange(1, n + 1)
    rng = np.random.default_rng(n)
    for _ in range(3):
        k1, k2, k3 = rng.integers(1, n + 1, size=3)
        s = [np.sin(np.pi * j * k / (n + 1)) for k in (k1, k2, k3)]
        b = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = [4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3)]
        expect = b / (sigma + sum(lam))
        assert aux.rel_err_inf(aux.aux_solve(b, sigma, h), expect) < 1e-12
        # the stencil reproduces the eigenvalue (independent of the DST path)
        assert aux.rel_err_inf(aux.apply_operator(b, sigma, h), (sigma + sum(lam)) * b) < 1e-12


@pytest.mark.parametrize("n", [7, 15, 31, 63])
@pytest.mark.parametrize("sigma", [0.0, 1.0, 1e4])
def test_residual(n, sigma):
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 1, seed=n)[0]
    u = aux.aux_solve(b, sigma, h)
    r = b - aux.apply_operator(u, sigma, h)
    norm_A = sigma + 12.0 / h**2
    assert np.max(np.abs(r)) / (norm_A * np.max(np.abs(u))) < 1e-15 * n


def test_inverse_symmetric_and_positive():
    n = 15
    h, _ = inp.grid(n)
    b1, b2 = inp.rhs_normal(n, 2, seed=11)
    u1, u2 = aux.aux_solve(b1, 3.0, h), aux.aux_solve(b2, 3.0, h)
    assert abs(np.vdot(u1, b2) - np.vdot(b1, u2)) < 1e-12 * abs(np.vdot(u1, b2)) + 1e-14
    # M-matrix: b >= 0 implies u >= 0 (positivity theorem, the non-negative inverse)
    bpos = np.abs(b1)
    assert np.min(aux.aux_solve(bpos, 0.0, h)) > -1e-14


def test_second_order_convergence():
    """u** = prod sin(pi (x_d + 1.5)/3) vanishes on the faces; (sigma - Lap) u** = (sigma + pi^2/3) u**."""
    sigma = 1.0
    errs = []
    ns = [15, 31, 63, 127]
    for n in ns:
        h, _ = inp.grid(n)
        z, y, x = inp.mesh(n)
        ue = np.sin(np.pi * (x + 1.5) / 3) * np.sin(np.pi * (y + 1.5) / 3) * np.sin(np.pi * (z + 1.5) / 3)
        u = aux.aux_solve((sigma + np.pi**2 / 3) * ue, sigma, h)
        errs.append(np.max(np.abs(u - ue)))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.7 < r < 4.3 for r in ratios), ratios


def test_config1_manufactured_exact():
    """Noise-free b = A_D u*_grid is solved back to u*_grid (exact discrete solution)."""
    n = 31
    h, _ = inp.grid(n)
    dt = h
    sigma = 1.0 / dt + 1.0
    ustar = inp.manufactured_c1(n, dt)
    b = aux.apply_operator(ustar, sigma, h)
    assert aux.rel_err_inf(aux.aux_solve(b, sigma, h), ustar) < 1e-13
    b_noisy = b + inp.noise_uniform(n, seed=0)
    u = aux.aux_solve(b_noisy, sigma, h)
    assert np.max(np.abs(aux.apply_operator(u, sigma, h) - b_noisy)) < 1e-11 * np.max(np.abs(b_noisy))


def test_batched_shapes():
    n = 7
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 3, seed=5)
    u = aux.aux_solve(b, 2.0, h)
    for i in range(3):
        assert np.max(np.abs(u[i] - aux.aux_solve(b[i], 2.0, h))) < 1e-14


def test_dst_matrix_accuracy_against_high_precision():
    """Entries of the sine matrix agree with a long-double evaluation to ~1 ulp at n = 255."""
    n = 255
    S = aux.dst1_matrix(n)
    j = np.arange(1, n + 1)
    r = (np.outer(j, j) % (2 * (n + 1))).astype(np.longdouble)
    pi = np.longdouble("3.14159265358979323846264338327950288")
    ref = np.sqrt(np.longdouble(2) / (n + 1)) * np.sin(pi * r / (n + 1))
    assert float(np.max(np.abs(S - ref))) < 4e-16
