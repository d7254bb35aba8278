"""The adaptive time loop (Algorithm "Main Steps", Steps 3-8: dt from the CFL-type condition,
Step 4b rebuilds of the boundary matrix, Step 8 threshold) through the C ABI, against the
oracle's loop on the same data: the same decisions (dt sequence, rebuild flags, stop reason)
and the same states.  Also: the CFL scan against the oracle's, and a rebuild equal bitwise to a
fresh build at the same sigma."""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import basis as ob
from oracle import geometry as og
from oracle import pks as opks
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _case(n, lmax, c_amp, dev, sigma0):
    import torch
    from paper_1811_03557_amd import api
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.basis_matrix(d, th, ph, lmax=lmax, beta=1)
    r2 = x**2 + y**2 + z**2
    rho = np.where(ps.n_plus, 1000.0 * np.exp(-100.0 * r2), 0.0)
    c = np.where(ps.n_plus, c_amp * np.exp(-50.0 * r2), 0.0)
    m = torch.from_numpy(ps.m_plus.astype(np.uint8)).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    bep = api.build_boundary_matrix(m, Bd, n, h, sigma0, x0)
    return h, ps, B, rho, c, m, Bd, bep


def _compare(res, ref, rg, cg, ro, co):
    assert res["stop"] == ref["stop"], (res["stop"], ref["stop"])
    assert res["steps"] == ref["steps"] and res["rebuilt"] == ref["rebuilt"]
    for a, b in zip(res["dt_hist"], ref["dt_hist"]):
        assert abs(a - b) <= 1e-10 * b, (a, b)
    assert abs(res["t"] - ref["t"]) <= 1e-10 * ref["t"]
    for g, o in ((rg, ro), (cg, co)):
        g = g.cpu().numpy()
        assert np.max(np.abs(g - o)) <= 1e-10 * np.max(np.abs(o))


def test_cfl_scan_matches_oracle():
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 63
    h, ps, B, rho, c, *_ , bep = _case(n, 1, 500.0, dev, 1.0)
    say(f"cfl scan n={n}")
    rng = np.random.default_rng(5)
    c = c + np.where(ps.n_plus, rng.normal(size=c.shape), 0.0)
    out = api.cfl_scan(bep, torch.from_numpy(rho).to(dev), torch.from_numpy(c).to(dev)).cpu().numpy()
    # the same face differences and division in both: equal bitwise
    assert out[0] == opks.face_gradient_max(c, ps.m_plus, h)
    assert out[1] == np.max(np.abs(rho[ps.m_plus]))
    # a NaN in the scanned entries shows up
    i = int(np.flatnonzero(ps.m_plus.ravel())[7])
    rn = rho.copy().ravel()
    rn[i] = np.nan
    out = api.cfl_scan(bep, torch.from_numpy(rn.reshape(rho.shape)).to(dev),
                       torch.from_numpy(c).to(dev)).cpu().numpy()
    assert np.isnan(out[1]) and out[0] == opks.face_gradient_max(c, ps.m_plus, h)
    bep.close()


def test_adaptive_run_rebuilds_every_step():
    """c0 = 0 and chi = 1000 from dt0 = 1e-3 at 31^3: no bound at step 1, then the gradient of c
    grows every step, so every later step shrinks dt (by >= 0.19%) and rebuilds the matrix."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n, lmax, chi, dt0, steps = 31, 2, 1000.0, 1e-3, 10
    h, ps, B, rho, c, m, Bd, bep = _case(n, lmax, 0.0, dev, 1.0 / dt0)
    say(f"adaptive run n={n} chi={chi} dt0={dt0} steps={steps}")
    ro, co, ref = opks.adaptive_run(rho, c, ps, B, h, 1.0 / dt0, chi, 1.0, max_steps=steps)
    assert ref["rebuilt"] == [False] + [True] * (steps - 1)
    for a, b in zip(ref["dt_hist"][1:], ref["dt_hist"][2:]):
        assert b < a * (1 - 1e-3)  # decisions well separated from rounding
    rg, cg = torch.from_numpy(rho).to(dev), torch.from_numpy(c).to(dev)
    res = api.run(bep, chi, rg, cg, t_final=1.0, max_steps=steps)
    say(f"  rebuilds {res['rebuilds']}, dt {res['dt_hist'][0]:.3e} .. {res['dt']:.3e}")
    _compare(res, ref, rg, cg, ro, co)
    assert res["rebuilds"] == steps - 1 and abs(bep.sigma * res["dt"] - 1) < 1e-15
    # the handle now holds the last dt's matrix: equal bitwise to a fresh build at that sigma
    fresh = api.build_boundary_matrix(m, Bd, n, h, bep.sigma, inp.grid(n)[1])
    g = torch.from_numpy(np.random.default_rng(1).normal(size=(2, bep.n_gamma_in))).to(dev)
    assert torch.equal(api.bep_solve(bep, g), api.bep_solve(fresh, g))
    # and a rebuild back to the first sigma equals the first build
    bep.rebuild(1.0 / dt0)
    first = api.build_boundary_matrix(m, Bd, n, h, 1.0 / dt0, inp.grid(n)[1])
    assert torch.equal(api.bep_solve(bep, g), api.bep_solve(first, g))
    for b in (bep, fresh, first):
        b.close()


def test_adaptive_run_stops():
    """Test A data (chi = 1) from dt0 = 0.5 h^2: step 1 takes the CFL bound and rebuilds, later
    steps keep it.  Stops at t_final (after 3 steps) and at the Step 8 threshold (2 steps)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 31
    h = inp.grid(n)[0]
    sigma0 = 1.0 / (0.5 * h * h)
    h, ps, B, rho, c, m, Bd, bep = _case(n, 2, 500.0, dev, sigma0)
    t_final = 2.5 * opks.cfl_dt(c, ps.m_plus, h, 1.0)
    for kw in ({"t_final": t_final}, {"t_final": 1.0, "rho_cap": 2000.0}):
        say(f"adaptive run n={n} Test A {kw}")
        ro, co, ref = opks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, max_steps=10, **kw)
        assert ref["stop"] == ("t_final" if "rho_cap" not in kw else "rho_cap")
        rg, cg = torch.from_numpy(rho).to(dev), torch.from_numpy(c).to(dev)
        bep.rebuild(sigma0)
        res = api.run(bep, 1.0, rg, cg, max_steps=10, **kw)
        say(f"  {res['stop']} after {res['steps']} steps, rebuilt {res['rebuilt']}")
        _compare(res, ref, rg, cg, ro, co)
        assert abs(res["rho_max"] - ref["rho_max"]) <= 1e-10 * ref["rho_max"]
    bep.close()


def test_adaptive_run_stops_on_nonfinite_state():
    """Step 8's guard: a NaN planted at one M+ node stops the loop before any step, the handle
    keeps its matrix (no rebuild), and the state is left as it was."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 31
    h = inp.grid(n)[0]
    sigma0 = 1.0 / (0.5 * h * h)
    h, ps, B, rho, c, m, Bd, bep = _case(n, 1, 500.0, dev, sigma0)
    i = int(np.flatnonzero(ps.m_plus.ravel())[11])
    rho.ravel()[i] = np.nan
    rg, cg = torch.from_numpy(rho).to(dev), torch.from_numpy(c).to(dev)
    res = api.run(bep, 1.0, rg, cg, t_final=1.0, max_steps=5)
    say(f"nonfinite stop: {res['stop']} after {res['steps']} steps")
    assert res["stop"] == "nonfinite" and res["steps"] == 0 and res["rebuilds"] == 0
    assert np.isnan(res["rho_max"]) and bep.sigma == sigma0
    assert np.array_equal(cg.cpu().numpy(), c)
    bep.close()


def test_adaptive_run_test_b():
    """Test B data (rho0 = 2000 exp(-100 (x^2 + y^2 + (z - 0.25)^2)), c0 = 0: blow-up at the
    boundary) with the zonal 2-term extension (M = 10, beta = 0) from dt0 = 0.5 h^2 at 31^3: the
    oracle's decisions (a rebuild at step 2, when c has grown) and states, step by step."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n, steps = 31, 6
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.zonal_basis_matrix(d, th, 10, beta=0)
    rho = np.where(ps.n_plus, 2000.0 * np.exp(-100.0 * (x**2 + y**2 + (z - 0.25) ** 2)), 0.0)
    c = np.zeros_like(rho)
    sigma0 = 1.0 / (0.5 * h * h)
    say(f"adaptive run n={n} Test B zonal M=10")
    ro, co, ref = opks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, 1.0, max_steps=steps)
    assert ref["rebuilt"][1] and ref["rebuilds"] >= 1
    prev = 1.0 / sigma0
    for cfl, dt in zip(ref["cfl_hist"], ref["dt_hist"]):
        assert abs(cfl / prev - 1.0) > 1e-6  # every decision far from a rounding tie
        prev = dt
    m = torch.from_numpy(ps.m_plus.astype(np.uint8)).to(dev)
    bep = api.build_boundary_matrix(m, torch.from_numpy(B).to(dev), n, h, sigma0, x0)
    rg, cg = torch.from_numpy(rho).to(dev), torch.from_numpy(c).to(dev)
    res = api.run(bep, 1.0, rg, cg, t_final=1.0, max_steps=steps)
    say(f"  {res['steps']} steps, rebuilt {res['rebuilt']}, max rho {res['rho_max']:.4e}")
    _compare(res, ref, rg, cg, ro, co)
    bep.close()


def test_adaptive_run_jump_rule_test_b():
    """The Test B termination rule (Sec. 4: stop once max |rho| grows by a cap over one step) on
    Test B data at 31^3 (max |rho| 1814 -> 780 -> 948: the second step grows it by 168): with a
    cap of 150 the loop stops after 2 steps, like the oracle's."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 31
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.zonal_basis_matrix(d, th, 10, beta=0)
    rho = np.where(ps.n_plus, 2000.0 * np.exp(-100.0 * (x**2 + y**2 + (z - 0.25) ** 2)), 0.0)
    c = np.zeros_like(rho)
    sigma0 = 1.0 / (0.5 * h * h)
    ro, co, ref = opks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, 1.0, max_steps=10,
                                    rho_jump_cap=150.0)
    assert ref["stop"] == "rho_jump" and ref["steps"] == 2
    m = torch.from_numpy(ps.m_plus.astype(np.uint8)).to(dev)
    bep = api.build_boundary_matrix(m, torch.from_numpy(B).to(dev), n, h, sigma0, x0)
    rg, cg = torch.from_numpy(rho).to(dev), torch.from_numpy(c).to(dev)
    say("adaptive run n=31 Test B, jump cap 150")
    res = api.run(bep, 1.0, rg, cg, t_final=1.0, max_steps=10, rho_jump_cap=150.0)
    say(f"  {res['stop']} after {res['steps']} steps, max rho {res['rho_max']:.1f}")
    _compare(res, ref, rg, cg, ro, co)
    bep.close()
