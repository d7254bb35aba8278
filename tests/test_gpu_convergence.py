"""Accuracy of the whole GPU path against an exact solution, at sizes the oracle cannot reach.

With rho = 0 and chi = 0 the system reduces to c_t = Lap c - c with zero Neumann data on the unit
sphere, solved exactly by c = exp(-(k^2 + 1) t) sin(k r)/(k r) with tan k = k (k the first positive
root).  The scheme is first order in time and second order in space (paper Sec. 2: IMEX step,
7-point Laplacian, the 3-term extension; Prop. "discrete generalized Green's formula"), so with
dt ~ h^2 (dt = T / ceil(T / (0.5 h^2))) the error at T = 0.01 must fall by about 4 per halving of
h: in the single domain (N = 31 ... 255), and on both decomposed domains (Case 1 and Case 2, both
meshes refined together), where it must also match the single domain's accuracy; at a fixed mesh
the dependence on dt is first order.
"""
import math

import numpy as np
import pytest

import dpm_inputs as inp
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

K = 4.493409457909064   # first positive root of tan k = k
T = 0.01
MESHES = (31, 63, 127, 255)


def _j0(r):
    return np.sinc(K * r / np.pi)   # sin(K r) / (K r)


def _dt(h):
    steps = math.ceil(T / (0.5 * h * h))
    return T / steps, steps


def _sd_errors():
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    geo = api.geometry("sphere", axes=(1.0,))
    errs = []
    for n in MESHES:
        h, x0 = inp.grid(n)
        dt, steps = _dt(h)
        m = api.classify(n, h, x0, geo, device=dev)
        idx, _ = api.gamma_points(m, h, x0)
        B, _ = api.basis_zonal(n, h, x0, geo, idx, 0, 1)
        bep = api.build_boundary_matrix(m, B, n, h, 1.0 / dt, x0)
        z, y, x = inp.mesh(n)
        c0 = _j0(np.sqrt(x * x + y * y + z * z))
        c = torch.from_numpy(c0).to(dev)
        rho = torch.zeros_like(c)
        st = api.Stepper(bep, dt, 0.0, rho, c)
        st.run(steps)
        mp = m.cpu().numpy().astype(bool)
        exact = math.exp(-(K * K + 1) * T) * c0
        err = np.max(np.abs(c.cpu().numpy() - exact)[mp]) / np.max(np.abs(exact[mp]))
        say(f"  single domain N = {n}: {steps} steps, rel max err {err:.3e}")
        assert float(rho.abs().max()) == 0.0
        errs.append(err)
        st.close()
        bep.close()
    return errs


@pytest.fixture(scope="module")
def sd_errors():
    return _sd_errors()


def test_single_domain_second_order(sd_errors):
    e = sd_errors
    say("ratios " + ", ".join(f"{a / b:.2f}" for a, b in zip(e, e[1:])))
    for a, b in zip(e[1:], e[2:]):
        assert a / b > 3.2, (a, b)
    assert e[-1] < 3e-4


def _dd_errors(case):
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    errs = []
    for n2 in MESHES:
        n1 = (n2 - 1) // 2     # Omega_1's cube has half the width: the same spacing
        h1, x01 = inp.grid(n1, 0.75)
        h2, x02 = inp.grid(n2)
        dt, steps = _dt(h2)
        if case == 1:
            prm = api.dd_params(n1, h1, x01, n2, h2, x02, 1.0 / dt, 0.5, 1.0, 0.75, 0, 1, 0)
            oz = 0.0
        else:
            prm = api.dd2_params(n1, h1, x01, (0.0, 0.0, 0.75), n2, h2, x02, (0.0, 0.0, 0.0),
                                 1.0 / dt, 1.0, 1.0, 0.5, 2.0, 2, 1, 6)
            oz = 0.75
        dd = api.dd_build(prm, device=dev)
        state, exact, masks = [], [], []
        for l, (n, half, zo) in enumerate(((n1, 0.75, oz), (n2, inp.HALF_WIDTH, 0.0))):
            z, y, x = inp.mesh(n, half)
            c0 = _j0(np.sqrt(x * x + y * y + (z + zo) ** 2))
            state += [torch.zeros((n,) * 3, dtype=torch.float64, device=dev),
                      torch.from_numpy(c0).to(dev)]
            exact.append(math.exp(-(K * K + 1) * T) * c0)
            masks.append(dd.masks(l)[0].cpu().numpy().astype(bool))
        ws = torch.empty(dd.workspace_size(api.opts("fp64")), dtype=torch.uint8, device=dev)
        for _ in range(steps):
            api.dd_step(dd, dt, 0.0, state, out=state, workspace=ws)
        scale = max(np.max(np.abs(e[m])) for e, m in zip(exact, masks))
        err = max(np.max(np.abs(state[2 * l + 1].cpu().numpy() - exact[l])[masks[l]]) / scale
                  for l in (0, 1))
        say(f"  case {case} {n1}/{n2}: {steps} steps, rel max err {err:.3e}")
        errs.append(err)
        dd.close()
    return errs


@pytest.mark.parametrize("case", [1, 2])
def test_decomposed_domain_second_order(case, sd_errors):
    """Case 1: the ball r < 0.5 and the shell, one harmonic per term; Case 2: the cap around the
    north pole and the rest, 3 harmonics (3-term) on Gamma and 7 (3-term) on Z (3 on Z leave the
    truncation of the solution's trace on Z, j0(k sqrt(1.25 - cos psi)), above the mesh error)."""
    e = _dd_errors(case)
    say("ratios " + ", ".join(f"{a / b:.2f}" for a, b in zip(e, e[1:])))
    for a, b in zip(e[1:], e[2:]):
        assert a / b > 3.2, (a, b)
    # as accurate as the single domain on the same spacing
    for a, b in zip(e, sd_errors):
        assert a <= 1.05 * b, (a, b)


def test_single_domain_first_order_in_time():
    """At a fixed mesh (N = 63) the IMEX step is first order in dt: the differences between the
    states at T = 0.02 reached with dt = T/4, T/8, T/16, T/32 halve with dt."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    geo = api.geometry("sphere", axes=(1.0,))
    n = 63
    h, x0 = inp.grid(n)
    m = api.classify(n, h, x0, geo, device=dev)
    idx, _ = api.gamma_points(m, h, x0)
    B, _ = api.basis_zonal(n, h, x0, geo, idx, 0, 1)
    z, y, x = inp.mesh(n)
    c0 = _j0(np.sqrt(x * x + y * y + z * z))
    mp = m.cpu().numpy().astype(bool)
    tt = 0.02
    finals = []
    for steps in (4, 8, 16, 32):
        dt = tt / steps
        bep = api.build_boundary_matrix(m, B, n, h, 1.0 / dt, x0)
        c = torch.from_numpy(c0).to(dev)
        rho = torch.zeros_like(c)
        st = api.Stepper(bep, dt, 0.0, rho, c)
        st.run(steps)
        finals.append(c.cpu().numpy()[mp])
        st.close()
        bep.close()
    d = [np.max(np.abs(a - b)) for a, b in zip(finals, finals[1:])]
    say("time differences " + ", ".join(f"{v:.3e}" for v in d) + "; ratios "
        + ", ".join(f"{a / b:.2f}" for a, b in zip(d, d[1:])))
    for a, b in zip(d, d[1:]):
        assert 1.7 < a / b < 2.3, (a, b)
