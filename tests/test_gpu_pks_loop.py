"""The graph-captured time loop (dpm_stepper): replays equal eager steps bitwise, the finiteness
guard names the first non-finite step, and the ellipsoid time loop at 127^3 (dt = h/4, Test A
data, l <= 4, beta = 1) follows the oracle over its first steps."""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import basis as ob
from oracle import dpm as odpm
from oracle import geometry as og
from oracle import pks as opks
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _setup(n, shape, lmax, dt, dev, prec="fp64"):
    import torch
    from paper_1811_03557_amd import api
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    if shape == "sphere":
        mp = og.inside_sphere(z, y, x)
        proj = og.project_sphere
        axes = np.array([1.0, 1.0, 1.0])
    else:
        mp = og.inside_ellipsoid(z, y, x)
        proj = og.project_ellipsoid
        axes = np.array([1.0, 0.8, 0.6])
    ps = og.PointSets(mp)
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = proj(gz, gy, gx)
    Bref = ob.basis_matrix(d, th, ph, lmax, 1)
    m_gpu = torch.from_numpy(mp.astype(np.uint8)).to(dev)
    bep = api.build_boundary_matrix(m_gpu, torch.from_numpy(Bref).to(dev), n, h, 1.0 / dt, x0,
                                    prec=prec)
    # Test A data: point values on M+, values at the projection onto Gamma on gamma
    r2 = x**2 + y**2 + z**2
    q = np.stack([axes[0] * np.sin(th) * np.cos(ph), axes[1] * np.sin(th) * np.sin(ph),
                  axes[2] * np.cos(th)], 1)
    q2 = np.sum(q * q, 1)
    rho = np.where(mp, 1000.0 * np.exp(-100.0 * r2), 0.0).ravel()
    c = np.where(mp, 500.0 * np.exp(-50.0 * r2), 0.0).ravel()
    rho[ps.idx] = 1000.0 * np.exp(-100.0 * q2)
    c[ps.idx] = 500.0 * np.exp(-50.0 * q2)
    return h, ps, Bref, bep, rho.reshape(mp.shape), c.reshape(mp.shape)


def test_stepper_replays_equal_eager_steps():
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 31
    h, _ = inp.grid(n)
    dt = 0.5 * h * h
    say(f"stepper n={n} sphere dt={dt:.3e}")
    _, ps, _, bep, rho0, c0 = _setup(n, "sphere", 2, dt, dev)
    re = torch.from_numpy(rho0).to(dev)
    ce = torch.from_numpy(c0).to(dev)
    rs, cs = re.clone(), ce.clone()
    st = api.Stepper(bep, dt, 1.0, rs, cs)
    eager = []
    for _ in range(5):
        re, ce = api.dpm_step(bep, dt, 1.0, re, ce)
        eager.append((re.clone(), ce.clone()))
    done = 0
    for k in (1, 2, 1):
        st.run(k)
        done += k
        torch.cuda.synchronize()
        assert torch.equal(rs, eager[done - 1][0]) and torch.equal(cs, eager[done - 1][1]), done
        # unrelated eager work between replays
        api.aux_solve(torch.randn((n, n, n), dtype=torch.float64, device=dev), 3.0, h)
        torch.cuda.synchronize()
    assert st.first_nonfinite() == 0
    # a non-finite value planted in the state shows up in the outputs of the next step
    i = np.flatnonzero(ps.m_plus.ravel())[0]
    rs.view(-1)[int(i)] = float("nan")
    st.run(1)
    assert st.first_nonfinite() == done + 1
    st.close()
    bep.close()


def test_ellipsoid_time_loop_127():
    """C4 configuration: ellipsoid (1, 0.8, 0.6), N = 127, dt = h/4, chi = 1; the HIP time loop
    (FP64, and FP32 transforms) against the oracle step by step while the state is finite."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 127
    h, _ = inp.grid(n)
    dt = h / 4
    say(f"time loop n={n} ellipsoid dt={dt:.4e}")
    _, ps, Bref, bep, rho0, c0 = _setup(n, "ellipsoid", 4, dt, dev)
    assert (bep.n_gamma_in, bep.n_basis) == (ps.n_gamma_in, 50)
    A = odpm.bep_matrix(Bref, ps, 1.0 / dt, h)
    say("oracle boundary matrix done")
    bep32 = api.build_boundary_matrix(
        torch.from_numpy(ps.m_plus.astype(np.uint8)).to(dev), torch.from_numpy(Bref).to(dev), n, h,
        1.0 / dt, inp.grid(n)[1], prec="fp32", max_refine=0)
    r64, c64 = torch.from_numpy(rho0).to(dev), torch.from_numpy(c0).to(dev)
    r32, c32 = r64.clone(), c64.clone()
    s64 = api.Stepper(bep, dt, 1.0, r64, c64)
    s32 = api.Stepper(bep32, dt, 1.0, r32, c32, prec="fp32", max_refine=0)
    ro, co = rho0, c0
    for k in range(1, 4):
        ro, co, _ = opks.dpm_step(ro, co, ps, Bref, A, h, dt, 1.0)
        if not (np.all(np.isfinite(ro)) and np.max(np.abs(ro)) < 1e30):
            say(f"step {k}: oracle state left the finite window")
            break
        s64.run(1)
        s32.run(1)
        torch.cuda.synchronize()
        e = []
        for (rg, cg) in ((r64, c64), (r32, c32)):
            rg, cg = rg.cpu().numpy(), cg.cpu().numpy()
            e.append(max(np.max(np.abs(rg - ro)) / np.max(np.abs(ro)),
                         np.max(np.abs(cg - co)) / np.max(np.abs(co))))
        say(f"step {k}: max|rho| {np.max(np.abs(ro)):.3e}, rel err fp64 {e[0]:.2e}, fp32 {e[1]:.2e}")
        assert e[0] < 1e-10, k
        assert e[1] < 1e-5, k
    assert s64.first_nonfinite() == 0
    s64.close()
    s32.close()
    bep.close()
    bep32.close()
