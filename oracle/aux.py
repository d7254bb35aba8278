"""Oracle: the discrete auxiliary problem (AP).

Paper, Sec. 2, "The Discrete Auxiliary Problem" (eqs discrete_ap, discrete_ap_boundary):
L v = q on M0, v = 0 on N0 \\ M0, with L = I - dt*Lap_h and Lap_h the standard second-order
7-point Laplacian (eq stencil:7-point; the explicit coefficients appear in the proof of the
positivity theorem).  The library states it in sigma-form, (sigma I - Lap_h) u = b; the paper's
AP(q) is this solve with sigma = 1/dt and b = q/dt.

The exact solution is written out through the textbook eigen-decomposition of the zero-Dirichlet
second difference: eigenvectors sin(pi j k/(N+1)) and eigenvalues -(4/h^2) sin^2(pi k/(2(N+1))).
The paper only says "Fast Poisson Solver" (Sec. 4, "Choice of Meshes"); the oracle applies the
dense orthonormal DST-I matrix along each axis, O(N^4), so that every step can be read by eye.

TEST INFRASTRUCTURE: imported only by tests/, smoke() and bench.py's cpu_baseline.
"""
from __future__ import annotations

import numpy as np


def dst1_matrix(n: int) -> np.ndarray:
    """Orthonormal DST-I matrix S[j-1,k-1] = sqrt(2/(n+1)) sin(pi j k/(n+1)), j,k = 1..n.

    sin is 2 pi-periodic, so j k is first reduced modulo 2(n+1) in exact integer arithmetic;
    the argument passed to sin then stays below 2 pi (unreduced arguments reach ~pi n and lose
    up to ~1e-14 of accuracy at n = 255).
    """
    j = np.arange(1, n + 1, dtype=np.int64)
    r = np.outer(j, j) % (2 * (n + 1))
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * r.astype(np.float64) / (n + 1))


def eigenvalues(n: int, h: float) -> np.ndarray:
    """lambda_k = (4/h^2) sin^2(pi k / (2(n+1))), k = 1..n: eigenvalues of -Lap_h in 1D."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return 4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2


def apply_operator(u: np.ndarray, sigma: float, h: float) -> np.ndarray:
    """(sigma I - Lap_h) u with the 7-point stencil and zero values on the ghost layer.

    u has shape (..., n, n, n) in [z][y][x] order.
    """
    pad = [(0, 0)] * (u.ndim - 3) + [(1, 1)] * 3
    p = np.pad(u, pad)
    c = p[..., 1:-1, 1:-1, 1:-1]
    nb = (p[..., 2:, 1:-1, 1:-1] + p[..., :-2, 1:-1, 1:-1]
          + p[..., 1:-1, 2:, 1:-1] + p[..., 1:-1, :-2, 1:-1]
          + p[..., 1:-1, 1:-1, 2:] + p[..., 1:-1, 1:-1, :-2])
    lap = (nb - 6.0 * c) / h**2
    return sigma * c - lap


def apply_s3(v: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Apply the symmetric matrix S along x, then y, then z of v (..., n, n, n)."""
    n = S.shape[0]
    lead = v.shape[:-3]
    w = v.reshape(-1, n, n, n)
    w = w @ S                                              # along x (last axis)
    w = np.matmul(S, w)                                    # along y: S @ w[b, z]
    w = (S @ w.reshape(w.shape[0], n, n * n)).reshape(w.shape)  # along z
    return w.reshape(lead + (n, n, n))


def aux_solve(b: np.ndarray, sigma: float, h: float) -> np.ndarray:
    """Exact FP64 solution u of (sigma I - Lap_h) u = b, zero Dirichlet ghosts.

    u = S3 D^{-1} S3 b with S3 the orthonormal DST-I along each axis (S3 is its own inverse)
    and D the diagonal sigma + lambda_kx + lambda_ky + lambda_kz.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[-1]
    S = dst1_matrix(n)
    lam = eigenvalues(n, h)
    denom = sigma + lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    return apply_s3(apply_s3(b, S) / denom, S)


def rel_err_inf(u: np.ndarray, ref: np.ndarray) -> float:
    """||u - ref||_inf / ||ref||_inf (max norm, as the paper's error measures)."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(np.asarray(u, dtype=np.float64) - ref)) / np.max(np.abs(ref)))
