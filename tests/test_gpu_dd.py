"""Domain decomposition, Case 1 (Sec. 3, eqs interface_condition, reduced_DD1_BEP1,
reduced_DD1_BEP2) and Case 2 (eqs DD2_BEP, reduced_DD2_BEP, effective densities) through the C
ABI, against the oracle (oracle/dd.py) on the same data:

- the point sets of both subdomains (bit-exact) and the stacked coupled-BEP matrix;
- one step on both subdomains (forcing, particular solutions, the coupled least squares, the
  Green's formula of each subdomain), also in place and on meshes of different spacing;
- the exact constant state and the node-sampled Gaussian initial data.

Tolerance: the matrix and the states come from FP64 AP solves (FFT form, relative error ~1e-14
per solve) and an FP64 QR, so 1e-10 relative to the largest entry leaves four orders of margin.
"""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import dd as odd
from oracle import geometry as og
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _params(case, sigma, m_gamma, beta, m_z):
    from paper_1811_03557_amd import api
    return api.dd_params(case.n1, case.h1, case.x01, case.n2, case.h2, case.x02, sigma,
                         case.r_z, 1.0, 0.5 * (case.r_z + 1.0), m_gamma, beta, m_z)


def _data(mesh, ps):
    z, y, x = mesh
    r2 = x * x + y * y + z * z
    return (np.where(ps.n_plus, 10 * np.exp(-2 * r2), 0.0),
            np.where(ps.n_plus, 5 * np.exp(-r2), 0.0))


CASES = [
    # n1, half-width of Omega_1's cube, n2, r_z, m_gamma, m_z, beta
    (15, 0.75, 31, 0.5, 2, 2, 1),    # the same spacing on both meshes
    (31, 0.75, 31, 0.5, 3, 2, 1),    # Omega_1's mesh twice as fine
    (63, 0.75, 31, 0.5, 0, 0, 1),    # Omega_1's mesh four times as fine, one harmonic per term
]


@pytest.mark.parametrize("n1,half1,n2,r_z,mg,mz,beta", CASES)
def test_dd_matrix_and_point_sets(n1, half1, n2, r_z, mg, mz, beta):
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase(n1, half1, n2, r_z, mg, mz, beta)
    assert case.ps1.margin_ok and case.ps2.margin_ok
    dt = 1e-3
    say(f"dd matrix n1={n1} half1={half1} n2={n2} mg={mg} mz={mz} beta={beta}")
    dd, A = api.dd_build(_params(case, 1.0 / dt, mg, beta, mz), return_A=True, device=dev)
    for l, ps in enumerate((case.ps1, case.ps2)):
        mp, np_ = dd.masks(l)
        assert np.array_equal(mp.cpu().numpy().astype(bool), ps.m_plus)
        assert np.array_equal(np_.cpu().numpy().astype(bool), ps.n_plus)
        assert dd.n_gamma[l] == ps.n_gamma and dd.n_gamma_in[l] == ps.n_gamma_in
    # no gamma node of Omega_2 near the Gamma/Z split radius: the split is a clean decision
    gz, gy, gx = og.gamma_coords(case.ps2, case.x02, case.h2)
    rr = np.sqrt(gx * gx + gy * gy + gz * gz)
    assert np.min(np.abs(rr - 0.5 * (r_z + 1.0))) > 0.5 * case.h2
    ref = odd.dd_matrix(case, 1.0 / dt)
    assert A.shape == ref.shape and dd.n_cols == case.n_cols
    err = np.max(np.abs(A.cpu().numpy() - ref)) / np.max(np.abs(ref))
    say(f"  rows {ref.shape[0]}, cols {ref.shape[1]}, rel err {err:.2e}")
    assert err <= TOL
    dd.close()


@pytest.mark.parametrize("n1,half1,n2,r_z,mg,mz,beta", CASES)
def test_dd_step_matches_oracle(n1, half1, n2, r_z, mg, mz, beta):
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase(n1, half1, n2, r_z, mg, mz, beta)
    dt, chi = 1e-3, 1.0
    say(f"dd step n1={n1} half1={half1} n2={n2} mg={mg} mz={mz} beta={beta}")
    A = odd.dd_matrix(case, 1.0 / dt)
    r1, c1 = _data(case.mesh1, case.ps1)
    r2, c2 = _data(case.mesh2, case.ps2)
    ref = odd.dd_step(r1, c1, r2, c2, case, A, dt, chi)[:4]
    dd = api.dd_build(_params(case, 1.0 / dt, mg, beta, mz), device=dev)
    state = [torch.from_numpy(v).to(dev) for v in (r1, c1, r2, c2)]
    out = api.dd_step(dd, dt, chi, state)
    for k, (g, o) in enumerate(zip(out, ref)):
        err = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
        say(f"  output {k}: rel err {err:.2e}")
        assert err <= TOL, (k, err)
    # a second step in place against the oracle's second step
    ref2 = odd.dd_step(*ref, case, A, dt, chi)[:4]
    api.dd_step(dd, dt, chi, out, out=list(out))
    for k, (g, o) in enumerate(zip(out, ref2)):
        err = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
        assert err <= TOL, ("second step", k, err)
    dd.close()


def test_dd_constant_state_and_gauss_data():
    """A constant state is an exact discrete solution of the coupled problem (P_0 represents it
    on both surfaces): rho stays 3, c moves to (1 - dt) 5 + 3 dt, on both N+; the node-sampled
    Gaussian data equal the formula at the N+ nodes and zero elsewhere."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase(15, 0.75, 31, 0.5, 2, 2, 1)
    dt = 0.5 * case.h2 ** 2
    dd = api.dd_build(_params(case, 1.0 / dt, 2, 1, 2), device=dev)
    say("dd constant state 15/31")
    state = []
    for ps in (case.ps1, case.ps2):
        state += [torch.from_numpy(np.where(ps.n_plus, 3.0, 0.0)).to(dev),
                  torch.from_numpy(np.where(ps.n_plus, 5.0, 0.0)).to(dev)]
    out = [v.cpu().numpy() for v in api.dd_step(dd, dt, 1.0, state)]
    cn = (1 - dt) * 5.0 + dt * 3.0
    for (r, c), ps in ((out[:2], case.ps1), (out[2:], case.ps2)):
        assert np.allclose(r[ps.n_plus], 3.0, rtol=1e-12, atol=0)
        assert np.allclose(c[ps.n_plus], cn, rtol=1e-12, atol=0)
        assert np.all(r[~ps.n_plus] == 0) and np.all(c[~ps.n_plus] == 0)
    for l, (mesh, ps) in enumerate(((case.mesh1, case.ps1), (case.mesh2, case.ps2))):
        z, y, x = mesh
        ref = np.where(ps.n_plus, 7.0 * np.exp(-3.0 * ((x - 0.1) ** 2 + y * y + z * z)), 0.0)
        g = dd.gauss_state(l, 7.0, 3.0, (0.1, 0.0, 0.0)).cpu().numpy()
        assert np.max(np.abs(g - ref)) <= 1e-14 * 7.0
    dd.close()


def test_dd_rejects_wrong_dt_and_shapes():
    import torch
    from paper_1811_03557_amd import api
    from paper_1811_03557_amd._lib import DPMError
    dev = need_gpu()
    case = odd.DDCase(15, 0.75, 31, 0.5, 0, 0, 1)
    dd = api.dd_build(_params(case, 1000.0, 0, 1, 0), device=dev)
    say("dd rejections")
    state = [torch.zeros((n,) * 3, dtype=torch.float64, device=dev) for n in (15, 15, 31, 31)]
    with pytest.raises(DPMError, match="sigma"):
        api.dd_step(dd, 2e-3, 1.0, state)
    with pytest.raises(ValueError, match="hold"):
        api.dd_step(dd, 1e-3, 1.0, state[::-1])
    dd.close()


# ---- Case 2: Z (radius 0.5 about the north pole) meets Gamma ---------------------------------
# The coupled matrices here have condition numbers up to 1e6 (zonal densities on both surfaces
# meet at the wedge), so the least-squares coefficients carry relative errors up to ~1e6 x 1e-16
# from either side's rounding: the steps are compared at 1e-9, the matrices (no solve) at 1e-10.

CASES2 = [
    # n1, n2, m_gamma, m_z, beta (Omega_1's cube [-0.75, 0.75]^2 x [0, 1.5])
    (15, 31, 4, 2, 0),    # the same spacing on both meshes, 2-term extension on Gamma
    (31, 31, 6, 3, 1),    # Omega_1's mesh twice as fine, 3-term extension on Gamma
    (63, 31, 2, 2, 0),    # four times as fine
]


def _params2(case, sigma):
    from paper_1811_03557_amd import api
    s1, s2 = case.sub
    return api.dd2_params(case.n1, s1["h"], s1["x0"], (0.0, 0.0, s1["zc"]), case.n2, s2["h"],
                          s2["x0"], (0.0, 0.0, 0.0), sigma, 1.0, case.q_z, case.r_z, 2.0,
                          case.m_gamma, case.beta, case.m_z, case.rcond or 0.0)


def _data2(mesh, ps):
    z, y, x = mesh
    r2 = x * x + y * y + (z - 0.5) ** 2
    return (np.where(ps.n_plus, 10 * np.exp(-2 * r2), 0.0),
            np.where(ps.n_plus, 5 * np.exp(-r2), 0.0))


@pytest.mark.parametrize("n1,n2,mg,mz,beta", CASES2)
def test_dd2_matrix_and_point_sets(n1, n2, mg, mz, beta):
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(n1, 0.75, 0.75, n2, 1.0, 0.5, mg, mz, beta=beta)
    assert case.covered
    dt = 1e-3
    say(f"dd2 matrix n1={n1} n2={n2} mg={mg} mz={mz} beta={beta}")
    dd, A = api.dd_build(_params2(case, 1.0 / dt), return_A=True, device=dev)
    for l, s in enumerate(case.sub):
        mp, np_ = dd.masks(l)
        assert np.array_equal(mp.cpu().numpy().astype(bool), s["ps"].m_plus)
        assert np.array_equal(np_.cpu().numpy().astype(bool), s["ps"].n_plus)
        assert dd.n_gamma_in[l] == s["ps"].n_gamma_in and dd.n_rows[l] == len(s["rows"])
    ref = odd.dd2_matrix(case, 1.0 / dt)
    assert A.shape == ref.shape
    err = np.max(np.abs(A.cpu().numpy() - ref)) / np.max(np.abs(ref))
    say(f"  rows {ref.shape[0]}, cols {ref.shape[1]}, rel err {err:.2e}")
    assert err <= 1e-10
    dd.close()


@pytest.mark.parametrize("n1,n2,mg,mz,beta", CASES2)
def test_dd2_step_matches_oracle(n1, n2, mg, mz, beta):
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(n1, 0.75, 0.75, n2, 1.0, 0.5, mg, mz, beta=beta)
    dt, chi = 1e-3, 1.0
    say(f"dd2 step n1={n1} n2={n2} mg={mg} mz={mz} beta={beta}")
    A = odd.dd2_matrix(case, 1.0 / dt)
    s1, s2 = case.sub
    st = list(_data2(s1["mesh"], s1["ps"])) + list(_data2(s2["mesh"], s2["ps"]))
    ref = odd.dd2_step(*st, case, A, dt, chi)[:4]
    dd = api.dd_build(_params2(case, 1.0 / dt), device=dev)
    state = [torch.from_numpy(v).to(dev) for v in st]
    out = api.dd_step(dd, dt, chi, state)
    for k, (g, o) in enumerate(zip(out, ref)):
        err = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
        say(f"  output {k}: rel err {err:.2e}")
        assert err <= 1e-9, (k, err)
    for l, s in enumerate(case.sub):
        z, y, x = s["mesh"]
        g0 = np.where(s["ps"].n_plus, 7.0 * np.exp(-3.0 * (x * x + y * y + (z - 0.4) ** 2)), 0.0)
        g = dd.gauss_state(l, 7.0, 3.0, (0.0, 0.0, 0.4)).cpu().numpy()
        assert np.max(np.abs(g - g0)) <= 1e-14 * 7.0
    dd.close()


def test_dd2_constant_state():
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0)
    dt = 0.5 * case.sub[1]["h"] ** 2
    dd = api.dd_build(_params2(case, 1.0 / dt), device=dev)
    say("dd2 constant state 15/31")
    state = []
    for s in case.sub:
        state += [torch.from_numpy(np.where(s["ps"].n_plus, 3.0, 0.0)).to(dev),
                  torch.from_numpy(np.where(s["ps"].n_plus, 5.0, 0.0)).to(dev)]
    out = [v.cpu().numpy() for v in api.dd_step(dd, dt, 1.0, state)]
    cn = (1 - dt) * 5.0 + dt * 3.0
    for (r, c), s in ((out[:2], case.sub[0]), (out[2:], case.sub[1])):
        assert np.allclose(r[s["ps"].n_plus], 3.0, rtol=1e-11, atol=0)
        assert np.allclose(c[s["ps"].n_plus], cn, rtol=1e-11, atol=0)
    dd.close()


def _adaptive_compare(res, ref, out, ref_state):
    assert res["stop"] == ref["stop"] and res["steps"] == ref["steps"]
    assert res["rebuilt"] == ref["rebuilt"]
    for a, b in zip(res["dt_hist"], ref["dt_hist"]):
        assert abs(a - b) <= 1e-10 * b, (a, b)
    for k, (g, o) in enumerate(zip(out, ref_state)):
        # scale by the largest entry (a state left at zero must come back exactly zero)
        err = np.max(np.abs(g.cpu().numpy() - o)) / max(np.max(np.abs(o)), 1e-300)
        assert err <= 1e-9, (k, err)


def test_dd_adaptive_run_rebuilds():
    """Case 1, rho of Test A with c0 = 0 and chi = 1000 from dt0 = 1e-3: the gradient of c grows
    every step, each subdomain's CFL-type bound shrinks dt and the coupled matrix is rebuilt;
    the same decisions and states as the oracle's loop."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase(15, 0.75, 31, 0.5, 1, 1, 1)
    dt0, chi, steps = 1e-3, 1000.0, 5
    st = []
    for mesh, ps in ((case.mesh1, case.ps1), (case.mesh2, case.ps2)):
        z, y, x = mesh
        st += [np.where(ps.n_plus, 1000.0 * np.exp(-100.0 * (x * x + y * y + z * z)), 0.0),
               np.zeros_like(x)]
    say(f"dd adaptive run 15/31 chi={chi} steps={steps}")
    ref_state, ref = odd.dd_adaptive_run(st, case, 1.0 / dt0, chi, 1.0, max_steps=steps)
    assert ref["rebuilt"][1:] == [True] * (steps - 1)
    for a, b in zip(ref["dt_hist"][1:], ref["dt_hist"][2:]):
        assert b < a * (1 - 1e-3)
    dd = api.dd_build(_params(case, 1.0 / dt0, 1, 1, 1), device=dev)
    state = [torch.from_numpy(v).to(dev) for v in st]
    res = api.dd_run(dd, chi, state, t_final=1.0, max_steps=steps)
    say(f"  rebuilds {res['rebuilds']}, dt {res['dt_hist'][0]:.3e} .. {res['dt']:.3e}")
    _adaptive_compare(res, ref, state, ref_state)
    # the handle holds the last dt's matrix: a step with it matches a fresh build's
    fresh = api.dd_build(_params(case, dd.sigma, 1, 1, 1), device=dev)
    a = api.dd_step(dd, 1.0 / dd.sigma, chi, state)
    b = api.dd_step(fresh, 1.0 / dd.sigma, chi, state)
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    dd.close()
    fresh.close()


def test_dd2_adaptive_run_test_b():
    """Case 2 with Test B data (rho0 = 2000 exp(-100 (x^2 + y^2 + (z - 0.25)^2)), c0 = 0) from
    dt0 = 0.5 h^2 against the oracle's loop (a rebuild at step 2, when c has grown), and the
    Step 8 stop at a threshold below the initial max |rho| (1814 at these nodes)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0)
    dt0 = 0.5 * case.sub[1]["h"] ** 2
    st = []
    for s in case.sub:
        z, y, x = s["mesh"]
        st += [np.where(s["ps"].n_plus, 2000.0 * np.exp(-100.0 * (x * x + y * y + (z - 0.25) ** 2)), 0.0),
               np.zeros_like(x)]
    for kw in ({"t_final": 1.0, "max_steps": 4}, {"t_final": 1.0, "max_steps": 10, "rho_cap": 1500.0}):
        say(f"dd2 adaptive run 15/31 Test B {kw}")
        ref_state, ref = odd.dd_adaptive_run(st, case, 1.0 / dt0, 1.0, **kw)
        dd = api.dd_build(_params2(case, 1.0 / dt0), device=dev)
        state = [torch.from_numpy(v).to(dev) for v in st]
        res = api.dd_run(dd, 1.0, state, **kw)
        say(f"  {res['stop']} after {res['steps']} steps, rebuilt {res['rebuilt']}")
        _adaptive_compare(res, ref, state, ref_state)
        assert abs(res["rho_max"] - ref["rho_max"]) <= 1e-9 * ref["rho_max"]
        assert res["stop"] == ("max_steps" if "rho_cap" not in kw else "rho_cap")
        dd.close()


def test_dd_meshes_off_powers_of_two_dense_form():
    """Both cases on meshes with N + 1 not a power of two (N1/N2 = 20/36: h1 = 1.5/21, h2 = 3/37,
    so the meshes do not align), solved by the dense FP64 transform form: one step against the
    oracle (no node lies within 1e-3 of a classification radius, so the masks are decided
    identically whatever the rounding)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    dt, chi = 1e-3, 1.0
    case = odd.DDCase(20, 0.75, 36, 0.5, 2, 2, 1)
    case2 = odd.DDCase2(20, 0.75, 0.75, 36, 1.0, 0.5, 4, 2, beta=0)
    runs = [("case 1", _params(case, 1.0 / dt, 2, 1, 2), odd.dd_matrix(case, 1.0 / dt),
             list(_data(case.mesh1, case.ps1)) + list(_data(case.mesh2, case.ps2)),
             lambda st, A: odd.dd_step(*st, case, A, dt, chi)[:4]),
            ("case 2", _params2(case2, 1.0 / dt), odd.dd2_matrix(case2, 1.0 / dt),
             list(_data2(case2.sub[0]["mesh"], case2.sub[0]["ps"]))
             + list(_data2(case2.sub[1]["mesh"], case2.sub[1]["ps"])),
             lambda st, A: odd.dd2_step(*st, case2, A, dt, chi)[:4])]
    for label, prm, A, st, step in runs:
        say(f"dd {label} 20/36 fp64_gemm")
        ref = step(st, A)
        dd = api.dd_build(prm, prec="fp64_gemm", device=dev)
        out = api.dd_step(dd, dt, chi, [torch.from_numpy(v).to(dev) for v in st], prec="fp64_gemm")
        for k, (g, o) in enumerate(zip(out, ref)):
            err = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
            say(f"  output {k}: rel err {err:.2e}")
            assert err <= 1e-9, (label, k, err)
        dd.close()


def test_dd2_uncovered_nodes_rejected():
    """With a tolerance of 0.2 mesh widths, 8 nodes of Omega_2's discrete boundary at the wedge
    fall in neither part (the oracle counts them): the build fails with DPM_EGEOM and names the
    count and the subdomain, and at 0.5 mesh widths it succeeds."""
    from paper_1811_03557_amd import api
    from paper_1811_03557_amd._lib import DPMError, DPM_EGEOM
    dev = need_gpu()
    case = odd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0, eps_layers=0.2)
    missing = [int((~s["cover"]).sum()) for s in case.sub]
    assert missing == [0, 8]
    s1, s2 = case.sub
    say("dd2 eps_layers 0.2 and 0.5")
    for eps, ok in ((0.2, False), (0.5, True)):
        prm = api.dd2_params(15, s1["h"], s1["x0"], (0.0, 0.0, 0.75), 31, s2["h"], s2["x0"],
                             (0.0, 0.0, 0.0), 1000.0, 1.0, 1.0, 0.5, eps, 4, 0, 2)
        if ok:
            api.dd_build(prm, device=dev).close()
        else:
            with pytest.raises(DPMError, match="8 nodes of subdomain 2") as e:
                api.dd_build(prm, device=dev)
            assert e.value.status == DPM_EGEOM


@pytest.mark.parametrize("prec,max_refine,tol", [("fp32", 3, 1e-9), ("fp32", 0, 1e-5)])
def test_dd_step_fp32_transforms(prec, max_refine, tol):
    """Both cases with FP32 transforms: the columns and both steps' solves refined in FP64 to
    1e-10 match the oracle at 1e-9; unrefined, at 1e-5 (FP32 rounding through ~8 solves)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    dt, chi = 1e-3, 1.0
    case = odd.DDCase(15, 0.75, 31, 0.5, 2, 2, 1)
    case2 = odd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0)
    runs = [("case 1", _params(case, 1.0 / dt, 2, 1, 2), odd.dd_matrix(case, 1.0 / dt),
             list(_data(case.mesh1, case.ps1)) + list(_data(case.mesh2, case.ps2)),
             lambda st, A: odd.dd_step(*st, case, A, dt, chi)[:4]),
            ("case 2", _params2(case2, 1.0 / dt), odd.dd2_matrix(case2, 1.0 / dt),
             list(_data2(case2.sub[0]["mesh"], case2.sub[0]["ps"]))
             + list(_data2(case2.sub[1]["mesh"], case2.sub[1]["ps"])),
             lambda st, A: odd.dd2_step(*st, case2, A, dt, chi)[:4])]
    for label, prm, A, st, step in runs:
        say(f"dd {label} 15/31 {prec} max_refine={max_refine}")
        ref = step(st, A)
        dd = api.dd_build(prm, prec=prec, max_refine=max_refine, device=dev)
        out = api.dd_step(dd, dt, chi, [torch.from_numpy(v).to(dev) for v in st], prec=prec,
                          max_refine=max_refine)
        for k, (g, o) in enumerate(zip(out, ref)):
            err = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
            say(f"  output {k}: rel err {err:.2e}")
            assert err <= tol, (label, k, err)
        dd.close()


def test_dd_positivity_per_subdomain():
    """The positivity theorem holds in each subdomain (Sec. 3 remark on Cases 1 and 2) when its
    conditions hold, among them non-negative values on the discrete boundary: Case 1 from Test A
    data, ten adaptive steps (dt at each subdomain's CFL-type bound) leave rho and c non-negative
    on both M+ up to rounding (1e-12 of the maximum).  (Case 2's truncated expansion on Z
    undershoots by about 5e-4 of the maximum on Test B data; the oracle does the same.)"""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase(31, 0.75, 31, 0.5, 0, 0, 1)
    dd = api.dd_build(_params(case, 1.0 / (0.5 * case.h2 ** 2), 0, 1, 0), device=dev)
    masks = [case.ps1.m_plus, case.ps2.m_plus]
    state = [dd.gauss_state(l, a, r) for l in (0, 1) for a, r in ((1000.0, 100.0), (500.0, 50.0))]
    say("dd positivity case 1")
    res = api.dd_run(dd, 1.0, state, t_final=1.0, max_steps=10)
    assert res["steps"] == 10 and res["rebuilds"] >= 1
    for l in (0, 1):
        for v in state[2 * l: 2 * l + 2]:
            a = v.cpu().numpy()[masks[l]]
            say(f"  subdomain {l + 1}: min {a.min():.3e}, max {a.max():.3e}")
            assert a.min() >= -1e-12 * a.max()
    dd.close()


def test_dd_cube_without_margin_rejected():
    """A subdomain whose N+ reaches its cube's ghost layer (Case 1: the ball r < 0.5 on a cube of
    half-width 0.55 at N = 15; Case 2: the cap's cube shifted down to z in [-0.45, 1.05]) is
    rejected with DPM_EGEOM, as the oracle's point sets report no margin."""
    from paper_1811_03557_amd import api
    from paper_1811_03557_amd._lib import DPMError, DPM_EGEOM
    dev = need_gpu()
    say("dd geometry without margin")
    h1, x01 = inp.grid(15, 0.55)
    h2, x02 = inp.grid(31)
    z, y, x = inp.mesh(15, 0.55)
    assert not og.PointSets(x * x + y * y + z * z < 0.25).margin_ok
    with pytest.raises(DPMError) as e:
        api.dd_build(api.dd_params(15, h1, x01, 31, h2, x02, 1e3, 0.5, 1.0, 0.75, 0, 1, 0), device=dev)
    assert e.value.status == DPM_EGEOM
    h1, x01 = inp.grid(15, 0.75)
    with pytest.raises(DPMError) as e:
        api.dd_build(api.dd2_params(15, h1, x01, (0.0, 0.0, 0.3), 31, h2, x02, (0.0, 0.0, 0.0), 1e3,
                                    1.0, 1.0, 0.5, 2.0, 2, 0, 1), device=dev)
    assert e.value.status == DPM_EGEOM


@pytest.mark.parametrize("case_no", [1, 2])
def test_dd_stepper_replays_equal_eager_steps(case_no):
    """The graph-captured decomposed step (both meshes, the side stream's branch inside the graph)
    replayed three times, with eager steps and synchronisations between the replays, equals the
    eager steps bitwise after every replay."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    dt, chi = 1e-3, 1.0
    if case_no == 1:
        case = odd.DDCase(15, 0.75, 31, 0.5, 2, 2, 1)
        prm = _params(case, 1.0 / dt, 2, 1, 2)
        st = list(_data(case.mesh1, case.ps1)) + list(_data(case.mesh2, case.ps2))
    else:
        case = odd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0)
        prm = _params2(case, 1.0 / dt)
        st = list(_data2(case.sub[0]["mesh"], case.sub[0]["ps"])) + list(_data2(case.sub[1]["mesh"], case.sub[1]["ps"]))
    dd = api.dd_build(prm, device=dev)
    eager = [torch.from_numpy(v).to(dev) for v in st]
    graph_state = [v.clone() for v in eager]
    say(f"dd stepper case {case_no}")
    stepper = api.DDStepper(dd, dt, chi, graph_state)
    ws = torch.empty(dd.workspace_size(api.opts("fp64")), dtype=torch.uint8, device=dev)
    for k in range(3):
        api.dd_step(dd, dt, chi, eager, out=eager, workspace=ws)
        torch.cuda.synchronize()
        stepper.run(1)
        torch.cuda.synchronize()
        for a, b in zip(eager, graph_state):
            assert torch.equal(a, b), (case_no, k)
    stepper.close()
    dd.close()


def test_dd2_adaptive_run_jump_rule():
    """The Test B termination rule on the decomposed domain (Case 2, Test B data at 15/31): the
    same stop and states as the oracle's loop."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(15, 0.75, 0.75, 31, 1.0, 0.5, 4, 2, beta=0)
    dt0 = 0.5 * case.sub[1]["h"] ** 2
    st = []
    for s in case.sub:
        z, y, x = s["mesh"]
        st += [np.where(s["ps"].n_plus, 2000.0 * np.exp(-100.0 * (x * x + y * y + (z - 0.25) ** 2)), 0.0),
               np.zeros_like(x)]
    maxes = [odd.dd_adaptive_run(st, case, 1.0 / dt0, 1.0, 1.0, max_steps=k)[1]["rho_max"]
             for k in range(1, 6)]
    jumps = np.diff(maxes)
    first = int(np.argmax(jumps > 0))
    cap = 0.5 * jumps[first]
    ref_state, ref = odd.dd_adaptive_run(st, case, 1.0 / dt0, 1.0, 1.0, max_steps=10, rho_jump_cap=cap)
    assert ref["stop"] == "rho_jump" and ref["steps"] == first + 1
    dd = api.dd_build(_params2(case, 1.0 / dt0), device=dev)
    state = [torch.from_numpy(v).to(dev) for v in st]
    say(f"dd2 adaptive run, jump cap {cap:.1f}")
    res = api.dd_run(dd, 1.0, state, t_final=1.0, max_steps=10, rho_jump_cap=cap)
    say(f"  {res['stop']} after {res['steps']} steps")
    _adaptive_compare(res, ref, state, ref_state)
    dd.close()


@pytest.mark.parametrize("case_no", [1, 2])
def test_dd_full_size_constant_state(case_no):
    """The timed configurations at full size, 127/63: Case 1 (ball r < 0.5 on [-0.75, 0.75]^3, the
    shell on [-1.5, 1.5]^3, one zonal harmonic per term) and Case 2 (the cap around the north pole
    with the paper's 150 zonal harmonics on Gamma and 6 on Z, tolerance 2 mesh widths).  A
    constant state is an exact discrete solution whatever the size (P_0 represents it on Gamma
    and on Z): rho stays 3 and c moves to (1 - dt) 5 + 3 dt on both N+, zero elsewhere.  Bound:
    the coupled least squares is consistent here, so the error is rounding amplified by the
    matrix's conditioning (min/max |R_ii| 1e-7 for Case 2): 1e-8 relative."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n1, n2 = 127, 63
    h1, h2 = 1.5 / (n1 + 1), 3.0 / (n2 + 1)
    dt = 0.5 * h1 * h1
    if case_no == 1:
        prm = api.dd_params(n1, h1, -0.75 + h1, n2, h2, -1.5 + h2, 1.0 / dt, 0.5, 1.0, 0.75, 0, 1, 0)
    else:
        prm = api.dd2_params(n1, h1, -0.75 + h1, (0.0, 0.0, 0.75), n2, h2, -1.5 + h2,
                             (0.0, 0.0, 0.0), 1.0 / dt, 1.0, 1.0, 0.5, 2.0, 149, 0, 5)
    say(f"dd case {case_no} full size 127/63 constant state")
    dd = api.dd_build(prm, device=dev)
    npl = [dd.masks(l)[1].bool() for l in (0, 1)]
    state = []
    for m in npl:
        state += [torch.where(m, 3.0, 0.0).to(torch.float64), torch.where(m, 5.0, 0.0).to(torch.float64)]
    out = api.dd_step(dd, dt, 1.0, state)
    cn = (1 - dt) * 5.0 + dt * 3.0
    for l, m in enumerate(npl):
        r, c = out[2 * l], out[2 * l + 1]
        er = float((r[m] - 3.0).abs().max()) / 3.0
        ec = float((c[m] - cn).abs().max()) / cn
        say(f"  subdomain {l + 1}: rel err rho {er:.2e}, c {ec:.2e}")
        assert er <= 1e-8 and ec <= 1e-8, (l, er, ec)
        assert int((r[~m] != 0).sum()) == 0 and int((c[~m] != 0).sum()) == 0
    dd.close()


def _full_size_case(case_no):
    """The timed configurations: Case 1 with one zonal harmonic per term, Case 2 with the
    paper's 150 zonal harmonics on Gamma and 6 on Z, both on the 127/63 meshes."""
    n1, n2 = 127, 63
    if case_no == 1:
        case = odd.DDCase(n1, 0.75, n2, 0.5, 0, 0, 1)
        h1 = case.h1
    else:
        case = odd.DDCase2(n1, 0.75, 0.75, n2, 1.0, 0.5, 149, 5, beta=0)
        h1 = case.sub[0]["h"]
    return case, 0.5 * h1 * h1


@pytest.mark.parametrize("case_no", [1, 2])
def test_dd_full_size_matches_oracle(case_no):
    """Full-size parity at 127/63 (the configurations the bench times): point sets bit-exact, the
    stacked matrix, and one step of Gaussian data, all against the oracle.
    Tolerances: the matrix comes from FP64 AP solves (1e-14 each), so 1e-10 as at small sizes.
    The step goes through the coupled least squares. Case 1 (5 columns) is well conditioned:
    1e-10. Case 2 has min/max |R_ii| near 1e-7, which amplifies rounding (1e-16) to about 1e-9:
    the step gets 1e-9 (measured 2e-12)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case, dt = _full_size_case(case_no)
    chi = 1.0
    say(f"dd case {case_no} full size 127/63 against the oracle")
    if case_no == 1:
        prm = _params(case, 1.0 / dt, 0, 1, 0)
        subs = [(case.mesh1, case.ps1), (case.mesh2, case.ps2)]
        A_ref = odd.dd_matrix(case, 1.0 / dt)
        data, step, tol_step = _data, odd.dd_step, 1e-10
    else:
        prm = _params2(case, 1.0 / dt)
        subs = [(s["mesh"], s["ps"]) for s in case.sub]
        A_ref = odd.dd2_matrix(case, 1.0 / dt)
        data, step, tol_step = _data2, odd.dd2_step, 1e-9
    dd, A = api.dd_build(prm, return_A=True, device=dev)
    for l, (_, ps) in enumerate(subs):
        mp, np_ = dd.masks(l)
        assert np.array_equal(mp.cpu().numpy().astype(bool), ps.m_plus)
        assert np.array_equal(np_.cpu().numpy().astype(bool), ps.n_plus)
    assert A.shape == A_ref.shape
    err = np.max(np.abs(A.cpu().numpy() - A_ref)) / np.max(np.abs(A_ref))
    say(f"  matrix {A_ref.shape}: rel err {err:.2e}; min/max |R_ii| {dd.rdiag[0] / dd.rdiag[1]:.2e}")
    assert err <= 1e-10
    del A
    st = []
    for mesh, ps in subs:
        st += list(data(mesh, ps))
    ref = step(*st, case, A_ref, dt, chi)[:4]
    out = api.dd_step(dd, dt, chi, [torch.from_numpy(v).to(dev) for v in st])
    for k, (g, o) in enumerate(zip(out, ref)):
        e = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
        say(f"  step output {k}: rel err {e:.2e}")
        assert e <= tol_step, (k, e)
    dd.close()


def test_dd2_ill_conditioned_system_takes_householder_qr():
    """Case 2 with 6 harmonics per term on Z: the coupled matrix has full rank but widely
    different column norms (min / max |R_ii| about 5e-7, kappa 8e7), below the CholeskyQR2
    threshold of 1e-5, so the plain least squares is factored by the Householder QR; the solution
    matches LAPACK's (one step against the oracle is the subject of the Case 2 parity tests)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(31, 0.75, 0.75, 31, 1.0, 0.5, 19, 5, beta=0)
    dt = 0.5 * case.sub[0]["h"] ** 2
    dd = api.dd_build(_params2(case, 1.0 / dt), device=dev)
    info = dd.lsq_info()
    say(f"dd2 31/31 with 6 harmonics on Z: QR {info['method']}, min/max |R_ii| "
        f"{dd.rdiag[0] / dd.rdiag[1]:.2e}")
    assert info["method"] == "householder" and info["rank"] == dd.n_cols
    dd.close()


def test_dd2_plain_least_squares_rejects_rank_deficient_matrix():
    """Case 2 with 20 harmonics per term on Z and the plain least squares (rcond = 0): the
    stacked matrix is numerically rank deficient (singular values down to 1e-19 of the largest),
    so the CholeskyQR2 factorisation breaks down or fails its orthogonality check, the
    Householder QR takes over on the untouched matrix, and its rank test rejects the build."""
    from paper_1811_03557_amd import api
    from paper_1811_03557_amd._lib import DPMError
    dev = need_gpu()
    case = odd.DDCase2(31, 0.75, 0.75, 31, 1.0, 0.5, 19, 19, beta=0)
    dt = 0.5 * case.sub[0]["h"] ** 2
    say("dd2 plain least squares, 20 harmonics on Z: expect DPM_ERANK")
    with pytest.raises(DPMError) as ei:
        api.dd_build(_params2(case, 1.0 / dt), device=dev)
    assert "rank deficient" in str(ei.value), str(ei.value)


# Truncated minimum-norm least squares (rcond > 0): the paper's 20 harmonics per term on Z.
# The coupled matrix is numerically rank deficient (its singular values fall smoothly to 1e-19
# of the largest); rcond sits in a gap of each configuration's spectrum (31/31: 3.4e-7 -> 4.1e-8;
# 127/63: 7.7e-7 -> 1.0e-7), so both sides keep the same singular triplets.  The kept part has
# condition up to 1/rcond, which amplifies rounding (1e-16) to about 1e-16/rcond: steps compared
# at 1e-8 (31/31) and 1e-7 (127/63).
TRUNC = [(31, 31, 19, 19, 1e-7, 1e-8), (127, 63, 149, 19, 3e-7, 1e-7)]


@pytest.mark.parametrize("n1,n2,mg,mz,rcond,tol", TRUNC)
def test_dd2_truncated_least_squares_matches_oracle(n1, n2, mg, mz, rcond, tol):
    """Case 2 with 20 harmonics per term on Z and the truncated least squares: the numerical
    rank and the smallest kept singular value of the GPU's Jacobi SVD of R agree with LAPACK's SVD
    of the stacked matrix, and one step of Test B-like data matches the oracle's step with the
    same rcond (gelsd)."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    case = odd.DDCase2(n1, 0.75, 0.75, n2, 1.0, 0.5, mg, mz, beta=0, rcond=rcond)
    s1, s2 = case.sub
    dt, chi = 0.5 * s1["h"] ** 2, 1.0
    say(f"dd2 truncated least squares n1={n1} n2={n2} mg={mg} mz={mz} rcond={rcond:g}")
    A = odd.dd2_matrix(case, 1.0 / dt)
    sv = np.linalg.svd(A, compute_uv=False)
    rank = int(np.sum(sv > rcond * sv[0]))
    dd = api.dd_build(_params2(case, 1.0 / dt), device=dev)
    info = dd.lsq_info()
    say(f"  rank {info['rank']} (LAPACK {rank} of {A.shape[1]}), smallest kept "
        f"{info['smin_ratio']:.3e} (LAPACK {sv[rank - 1] / sv[0]:.3e})")
    assert info["rcond"] == rcond and info["rank"] == rank
    assert info["method"] == "householder_truncated"
    assert abs(info["smin_ratio"] / (sv[rank - 1] / sv[0]) - 1.0) < 1e-6
    st = list(_data2(s1["mesh"], s1["ps"])) + list(_data2(s2["mesh"], s2["ps"]))
    ref = odd.dd2_step(*st, case, A, dt, chi)[:4]
    out = api.dd_step(dd, dt, chi, [torch.from_numpy(v).to(dev) for v in st])
    for k, (g, o) in enumerate(zip(out, ref)):
        err = np.max(np.abs(g.cpu().numpy() - o)) / np.max(np.abs(o))
        say(f"  output {k}: rel err {err:.2e}")
        assert err <= tol, (k, err)
    dd.close()
