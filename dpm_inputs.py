"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and the benchmark.

This module only draws random numbers and lays out coordinates of the auxiliary cube.  It
holds none of the method's arithmetic (no operator, transform, point-set rule, projection or
basis): both the CPU oracle and the HIP path receive these arrays as plain inputs.

Cube convention: the auxiliary cube is [-a, a]^3 with N interior nodes per axis, spacing
h = 2a/(N+1), node i (0-based) at x0 + i*h with x0 = -a + h; the zero Dirichlet ghosts sit on
the faces.  Arrays are C-ordered [z][y][x] (x fastest).
"""
from __future__ import annotations

import numpy as np

HALF_WIDTH = 1.5  # the cube [-1.5, 1.5]^3 of every workload below


def grid(n: int, half_width: float = HALF_WIDTH) -> tuple[float, float]:
    """Spacing h and coordinate x0 of the first interior node for N interior nodes."""
    h = 2.0 * half_width / (n + 1)
    return h, -half_width + h


def node_coords(n: int, half_width: float = HALF_WIDTH) -> np.ndarray:
    h, x0 = grid(n, half_width)
    return x0 + h * np.arange(n, dtype=np.float64)


def mesh(n: int, half_width: float = HALF_WIDTH):
    """Coordinate volumes (Z, Y, X), each [z][y][x]."""
    c = node_coords(n, half_width)
    return np.meshgrid(c, c, c, indexing="ij")


def rhs_normal(n: int, nrhs: int, seed: int = 0) -> np.ndarray:
    """nrhs right-hand sides with i.i.d. N(0,1) FP64 entries, shape (nrhs, n, n, n)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, n, n, n))


def noise_uniform(n: int, amp: float = 1e-3, seed: int = 0) -> np.ndarray:
    """i.i.d. U(-amp, amp) FP64 volume, shape (n, n, n)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(n, n, n))


def manufactured_c1(n: int, t: float, half_width: float = HALF_WIDTH) -> np.ndarray:
    """Samples of sin(pi x/3) sin(pi y/3) sin(pi z/3) e^{-t} at the interior nodes."""
    z, y, x = mesh(n, half_width)
    return np.sin(np.pi * x / 3) * np.sin(np.pi * y / 3) * np.sin(np.pi * z / 3) * np.exp(-t)


def random_density(n_gamma: int, seed: int = 0) -> np.ndarray:
    """A random grid function on the discrete boundary, U(0,1)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=n_gamma)


def serving_mix(n_sims: int = 64, seed: int = 0, sizes=(31, 63, 127, 255),
                sigma_range=(1.0, 1e4)):
    """Per-simulation grid size (uniform over `sizes`) and sigma (log-uniform over the range)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=n_sims)
    lo, hi = np.log(sigma_range[0]), np.log(sigma_range[1])
    sig = np.exp(rng.uniform(lo, hi, size=n_sims))
    return ns.astype(int), sig


def poisson_arrivals(n: int, qps: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process with rate qps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


def serving_workload(n_sims: int = 64, n_requests: int = 2000, qps: float = 1000.0, seed: int = 0,
                     sizes=(31, 63, 127, 255), step_fraction: float = 0.5,
                     closed_loop: bool = False):
    """Request mix of a serving run: simulations from `serving_mix`, the first
    step_fraction of them advancing DPM steps and the rest issuing aux solves; each request
    picks a simulation uniformly and, for aux solves, its own log-uniform sigma on [1, 1e4];
    Poisson arrivals at qps (all at time 0 when closed_loop).
    Returns (sim_n, sim_sigma, sim_is_step, req_sim, req_sigma, req_arrival)."""
    ns, sig = serving_mix(n_sims, seed=seed, sizes=sizes)
    is_step = np.arange(n_sims) < int(step_fraction * n_sims)
    rng = np.random.default_rng(seed + 1)
    req_sim = rng.integers(0, n_sims, size=n_requests)
    req_sig = np.exp(rng.uniform(0.0, np.log(1e4), size=n_requests))
    arr = np.zeros(n_requests) if closed_loop else poisson_arrivals(n_requests, qps, seed=seed + 2)
    return ns, sig, is_step, req_sim, req_sig, arr


def rhs_normal_device(n: int, nrhs: int, seed: int = 0, device="cuda"):
    """nrhs i.i.d. N(0,1) FP64 right-hand sides drawn on the device by torch's seeded generator,
    shape (nrhs, n, n, n).  Used where the batch is too large to draw on the host."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((nrhs, n, n, n), dtype=torch.float64, device=device, generator=g)
