"""Pins of the DPM oracle (oracle/dpm.py, oracle/pks.py) against the paper's theorems.

Paper, Sec. 2: P_gamma is a projection; Thm "BEP" (full BEP <=> trace of a solution),
Prop. "rank" (rank = |gamma_in|), Thm "reduced BEP", Prop. "discrete generalized Green's
formula"; positivity theorem (CFL-type condition); Sec. 4 initial data of Test A.
"""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import aux, dpm, pks
from oracle import basis as ob
from oracle import geometry as og


@pytest.fixture(scope="module")
def small():
    n = 15
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x, radius=1.0))
    assert ps.margin_ok
    sigma = 1.0 / (0.5 * h * h)
    P = dpm.projection_matrix(ps, sigma, h)
    return dict(n=n, h=h, x0=x0, ps=ps, sigma=sigma, P=P)


def test_projection_idempotent(small):
    P = small["P"]
    assert np.max(np.abs(P @ P - P)) < 1e-12 * max(1.0, np.max(np.abs(P)))


def test_rank_is_gamma_in(small):
    ps, P = small["ps"], small["P"]
    I = np.eye(ps.n_gamma)
    s = np.linalg.svd(I - P, compute_uv=False)
    rank = int(np.sum(s > 1e-10 * s[0]))
    assert rank == ps.n_gamma_in
    # reduced BEP rows (gamma_in) are independent and span the full BEP row space
    rows_in = (I - P)[ps.is_in]
    s_in = np.linalg.svd(rows_in, compute_uv=False)
    assert int(np.sum(s_in > 1e-10 * s_in[0])) == ps.n_gamma_in


def _random_solution(small, seed=0):
    """A random grid function u on N+ and its right-hand side f with L u = f on M+."""
    ps, sigma, h = small["ps"], small["sigma"], small["h"]
    rng = np.random.default_rng(seed)
    u = np.where(ps.n_plus, rng.uniform(-1, 1, size=ps.m_plus.shape), 0.0)
    f = np.where(ps.m_plus, aux.apply_operator(u, sigma, h) / sigma, 0.0)   # L = dt (sigma - Lap)
    return u, f


def test_bep_identity_and_green_formula(small):
    ps, sigma, h, P = small["ps"], small["sigma"], small["h"], small["P"]
    u, f = _random_solution(small)
    u_g = dpm.trace(u, ps.idx)
    Gf = dpm.particular_solution(f, ps, sigma, h)
    # Thm BEP: u_gamma - P_gamma u_gamma = Tr_gamma G f
    assert np.max(np.abs(u_g - P @ u_g - dpm.trace(Gf, ps.idx))) < 1e-12
    # Green's formula reproduces u on N+
    w = dpm.green_formula(u_g, f, ps, sigma, h)
    assert np.max(np.abs(np.where(ps.n_plus, w - u, 0.0))) < 1e-12
    # a density that is not a trace violates the BEP on gamma_in (reduced BEP detects it)
    bad = u_g + np.where(ps.is_in, 0.0, 1.0)
    r = bad - P @ bad - dpm.trace(Gf, ps.idx)
    assert np.max(np.abs(r[ps.is_in])) > 1e-3


def test_bep_matrix_and_lsq(small):
    ps, sigma, h, x0, P = small["ps"], small["sigma"], small["h"], small["x0"], small["P"]
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.basis_matrix(d, th, ph, lmax=2, beta=1)
    A = dpm.bep_matrix(B, ps, sigma, h)
    # columns equal Tr_gin (I - P_gamma) phi computed through the dense projection
    ref = ((np.eye(ps.n_gamma) - P) @ B.T)[ps.is_in]
    assert np.max(np.abs(A - ref)) < 1e-12
    g = np.random.default_rng(4).normal(size=ps.n_gamma_in)
    C = dpm.least_squares(A, g)
    assert np.max(np.abs(A.T @ (A @ C - g))) < 1e-9 * np.linalg.norm(A) ** 2 * np.linalg.norm(C)
    Q, R = np.linalg.qr(A)
    assert np.allclose(C, np.linalg.solve(R, Q.T @ g), atol=1e-10)


# ----------------------------------------------------------------------------- PKS forcing

def test_truncated_least_squares_closed_form():
    """The truncated minimum-norm least squares (rcond > 0) against its closed form on a matrix
    built from chosen singular triplets, A = 7.3 U diag(s) V^T with s spanning 1 .. 1e-13: the
    solution is V_k diag(1 / (7.3 s_k)) U_k^T g over the kept triplets (s > rcond, relative to the
    largest, which is why A is scaled), it has no component along the dropped right singular
    vectors, and without truncation it is the plain least-squares solution."""
    rng = np.random.default_rng(11)
    m, n = 60, 9
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.array([1.0, 0.6, 0.2, 3e-2, 1e-4, 2e-6, 5e-9, 1e-11, 1e-13])
    A = 7.3 * (U * s) @ V.T
    g = rng.standard_normal(m)
    for rcond, kept in ((1e-5, 5), (1e-7, 6), (1e-10, 7)):
        C = dpm.least_squares(A, g, rcond)
        ref = V[:, :kept] @ ((U[:, :kept].T @ g) / (7.3 * s[:kept]))
        # rounding of A is amplified by the smallest kept singular value's inverse
        tol = 1e-13 / s[kept - 1]
        assert np.max(np.abs(C - ref)) <= tol * np.max(np.abs(ref)), rcond
        assert np.max(np.abs(V[:, kept:].T @ C)) <= tol * np.max(np.abs(C))
    B = rng.standard_normal((m, n))  # well conditioned: truncation changes nothing
    assert np.allclose(dpm.least_squares(B, g, 1e-7), dpm.least_squares(B, g), rtol=1e-12)


def test_minmod():
    a = np.array([1.0, -1.0, 1.0, 0.0, 3.0, -3.0])
    b = np.array([2.0, -2.0, -1.0, 1.0, 2.0, -5.0])
    c = np.array([3.0, -0.5, 1.0, 1.0, 1.0, -4.0])
    assert np.array_equal(pks.minmod3(a, b, c), [1.0, -0.5, 0.0, 0.0, 1.0, -3.0])


def _line_volume(vals, axis):
    """A 7^3 volume that varies along one axis only, with the values of `vals` along it."""
    v = np.asarray(vals, dtype=np.float64)
    shape = [1, 1, 1]
    shape[axis] = v.size
    return np.broadcast_to(v.reshape(shape), (v.size,) * 3).copy()


def test_limited_slopes_hand_table():
    """Slope limiter (Sec. 2, eq slope_limiter and the slope formula above it): each case below
    was worked out by hand, and each of the three minmod arguments -- the doubled forward
    difference, the centred difference over 2h and the doubled backward difference -- is the
    selected one at some node.  h = 0.5, values along the axis (ghosts outside read 0):

      node  rho_{j-1} rho_j rho_{j+1}   2(fwd)/h  central/(2h)  2(bwd)/h   slope
        1     0.0     1.0    2.0          4.0       2.0           4.0      2.0   central
        2     1.0     2.0    2.25         1.0       1.25          4.0      1.0   forward
        3     2.0     2.25   3.25         4.0       1.25          1.0      1.0   backward
        4     2.25    3.25   3.0         -1.0       -0.25         4.0      0.0   signs differ
        5     3.25    3.0    1.0         -8.0       -2.25        -1.0     -1.0   backward (max)
    """
    h = 0.5
    vals = [0.0, 1.0, 2.0, 2.25, 3.25, 3.0, 1.0]
    expect = {1: 2.0, 2: 1.0, 3: 1.0, 4: 0.0, 5: -1.0}
    m_plus = np.ones((7, 7, 7), dtype=bool)
    for axis in range(3):
        rho = _line_volume(vals, axis)
        slopes = pks.limited_slopes(rho, m_plus, h)
        idx = [3, 3, 3]
        for j, s in expect.items():
            idx[axis] = j
            assert slopes[axis][tuple(idx)] == pytest.approx(s, abs=1e-14), (axis, j)
        # the other two axes see a constant profile: zero slope
        for other in range(3):
            if other != axis:
                idx[axis] = 3
                assert slopes[other][tuple(idx)] == 0.0
    # outside M+ the slope is zero by definition
    rho = _line_volume(vals, 2)
    mask = m_plus.copy()
    mask[:, :, 2] = False
    assert pks.limited_slopes(rho, mask, h)[2][3, 3, 2] == 0.0


def test_convective_term_quadratic_rho_linear_c():
    """Closed form that fixes the three minmod arguments together (Sec. 2, eqs slope_limiter and
    upwind_approximation): rho = x^2 on x > 2h, c = a x with a > 0.  The three arguments are
    2(rho' + h), rho' and 2(rho' - h) there, so the centred one, which equals rho' exactly, is
    selected; the reconstruction is exact and the upwind (left) face value is
    rho_j + (h/2) rho'_j.  Telescoping the fluxes gives
    g = chi a [(rho_j - rho_{j-1}) + (h/2)(rho'_j - rho'_{j-1})]/h = chi a rho'(x_j) = 2 chi a x_j
    exactly.  A centred difference over h instead of 2h would select 2 rho' - 2h and break the
    identity.  (A constant bias of the slope telescopes out of g, so the one-sided arguments are
    pinned by the hand table above, not here.)"""
    n, h, chi, a = 15, 0.1, 0.8, 1.7
    x = 0.3 + h * np.arange(n)                   # x > 2h everywhere (x_0 = 0.3)
    X = np.broadcast_to(x.reshape(1, 1, n), (n, n, n)).copy()
    rho = X ** 2
    c = a * X
    m_plus = np.zeros((n, n, n), dtype=bool)
    m_plus[2:-2, 2:-2, 2:-2] = True
    g = pks.convective_term(rho, c, m_plus, h, chi)
    inner = np.zeros_like(m_plus)
    inner[3:-3, 3:-3, 3:-3] = True
    assert np.allclose(g[inner], (2.0 * chi * a * X)[inner], rtol=1e-12, atol=1e-12)


def _sphere_case(n=31):
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    return h, x0, (z, y, x), ps


def test_forcing_closed_forms():
    h, _, (z, y, x), ps = _sphere_case()
    chi = 0.7
    # constant rho, quadratic c: g = chi rho0 Lap_h c = 6 chi rho0 (exact for quadratics)
    rho = np.where(ps.n_plus, 2.0, 0.0)
    c = np.where(ps.n_plus, x**2 + y**2 + z**2, 0.0)
    g = pks.convective_term(rho, c, ps.m_plus, h, chi)
    assert np.allclose(g[ps.m_plus], 6 * chi * 2.0, rtol=1e-11)
    # linear positive rho (minmod keeps the exact slope away from gamma_ex), linear c
    rho = np.where(ps.n_plus, 3.0 + 0.5 * x - 0.25 * y + 0.2 * z, 0.0)
    c = np.where(ps.n_plus, 2.0 * x + 1.5 * y - 1.0 * z, 0.0)
    g = pks.convective_term(rho, c, ps.m_plus, h, chi)
    interior = ps.m_plus & ~ps.gamma_in
    P = np.pad(interior, 1)
    deep = interior.copy()
    for s in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        deep &= P[1 + s[0]:1 + s[0] + interior.shape[0], 1 + s[1]:1 + s[1] + interior.shape[0],
                  1 + s[2]:1 + s[2] + interior.shape[0]]
    expect = chi * (2.0 * 0.5 + 1.5 * -0.25 + -1.0 * 0.2)
    assert np.allclose(g[deep], expect, rtol=1e-9, atol=1e-9)


def test_forcing_conservative():
    """Fluxes telescope: with data supported away from gamma, the sum of g over M+ vanishes."""
    h, _, (z, y, x), ps = _sphere_case()
    r2 = x**2 + y**2 + z**2
    rho = np.where(ps.n_plus, 1000 * np.exp(-100 * r2), 0.0)
    c = np.where(ps.n_plus, 500 * np.exp(-50 * r2), 0.0)
    g = pks.convective_term(rho, c, ps.m_plus, h, 1.0)
    assert abs(g.sum()) < 1e-9 * np.abs(g).sum()
    assert np.abs(g).max() > 1.0


def test_forcing_positive_under_cfl():
    """Positivity theorem: rho >= 0 and dt at the CFL bound give f_rho >= 0 (upwind choice)."""
    h, _, (z, y, x), ps = _sphere_case(23)
    rng = np.random.default_rng(7)
    for _ in range(5):
        rho = np.where(ps.n_plus, rng.uniform(0, 1, ps.m_plus.shape) ** 8, 0.0)
        c = np.where(ps.n_plus, rng.normal(size=ps.m_plus.shape), 0.0)
        dt = pks.cfl_dt(c, ps.m_plus, h, 1.0)
        f_rho, _ = pks.pks_rhs(rho, c, ps.m_plus, h, dt, 1.0)
        assert f_rho[ps.m_plus].min() > -1e-12 * rho.max()
        # beyond the bound the same data goes negative (the check has power)
        f_big, _ = pks.pks_rhs(rho, c, ps.m_plus, h, 20 * dt, 1.0)
        assert f_big[ps.m_plus].min() < 0


def test_forcing_reflection_symmetry():
    h, _, (z, y, x), ps = _sphere_case()
    r2 = x**2 + y**2 + z**2
    rho = np.where(ps.n_plus, 1000 * np.exp(-100 * r2), 0.0)
    c = np.where(ps.n_plus, 500 * np.exp(-50 * r2), 0.0)
    f_rho, f_c = pks.pks_rhs(rho, c, ps.m_plus, h, 1e-6, 1.0)
    for f in (f_rho, f_c):
        assert np.allclose(f, f[::-1, :, :], rtol=1e-12, atol=1e-9)
        assert np.allclose(f, f[:, :, ::-1], rtol=1e-12, atol=1e-9)
        assert np.allclose(f, np.transpose(f, (2, 1, 0)), rtol=1e-12, atol=1e-9)


def test_dpm_step_constant_state():
    """A constant state is an exact discrete Neumann solution, representable by Y_00."""
    n = 15
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.basis_matrix(d, th, ph, lmax=2, beta=1)
    dt = 0.01
    A = dpm.bep_matrix(B, ps, 1.0 / dt, h)
    rho0, c0 = 3.0, 5.0
    rho = np.where(ps.n_plus, rho0, 0.0)
    c = np.where(ps.n_plus, c0, 0.0)
    r1, c1, _ = pks.dpm_step(rho, c, ps, B, A, h, dt, 1.0)
    assert np.allclose(r1[ps.n_plus], rho0, rtol=1e-11)
    assert np.allclose(c1[ps.n_plus], (1 - dt) * c0 + dt * rho0, rtol=1e-11)
    assert np.all(r1[~ps.n_plus] == 0)


def test_dpm_step_symmetry_and_positivity():
    """Test A data on a centred sphere stays symmetric and non-negative for a CFL-sized step."""
    n = 15
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.basis_matrix(d, th, ph, lmax=0, beta=1)
    r2 = x**2 + y**2 + z**2
    rho = np.where(ps.n_plus, 10 * np.exp(-2 * r2), 0.0)
    c = np.where(ps.n_plus, 5 * np.exp(-1 * r2), 0.0)
    dt = min(pks.cfl_dt(c, ps.m_plus, h, 1.0), 0.5 * h * h)
    A = dpm.bep_matrix(B, ps, 1.0 / dt, h)
    r1, c1, coefs = pks.dpm_step(rho, c, ps, B, A, h, dt, 1.0)
    for f in (r1, c1):
        assert np.allclose(f, f[::-1], atol=1e-10) and np.allclose(f, np.transpose(f, (1, 2, 0)), atol=1e-10)
        assert f[ps.n_plus].min() >= -1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cfl_scan_linear_field(axis):
    """eq cfl_condition on a field linear along one axis (values on N+, zero beyond): every face of
    an M+ node sees the slope s, so max |grad_h c| = |s| and the bound is h / (6 chi |s|); faces
    of nodes outside M+ (which reach the zeros beyond N+) must not count."""
    h, _, mesh, ps = _sphere_case(15)
    s, chi = -3.25, 0.8
    c = np.where(ps.n_plus, s * mesh[axis], 0.0)
    g = pks.face_gradient_max(c, ps.m_plus, h)
    assert abs(g - abs(s)) < 1e-12 * abs(s)
    assert abs(pks.cfl_dt(c, ps.m_plus, h, chi) - h / (6 * chi * abs(s))) < 1e-12 * h
    # a field constant on N+ gives no bound
    assert pks.cfl_dt(np.where(ps.n_plus, 2.0, 0.0), ps.m_plus, h, chi) == np.inf


def _adaptive_case(n, lmax):
    h, x0, (z, y, x), ps = _sphere_case(n)
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, ph = og.project_sphere(gz, gy, gx)
    B = ob.basis_matrix(d, th, ph, lmax=lmax, beta=1)
    return h, (z, y, x), ps, B


def test_adaptive_constant_state():
    """Constant data: no CFL bound, so dt stays 1/sigma0 with no rebuild; the state is the exact
    discrete solution (rho constant, c_{k+1} = (1 - dt) c_k + dt rho) and the loop ends at the
    first t >= t_final."""
    h, _, ps, B = _adaptive_case(15, 1)
    dt0 = 0.5 * h * h
    rho = np.where(ps.n_plus, 3.0, 0.0)
    c = np.where(ps.n_plus, 5.0, 0.0)
    r, cc, s = pks.adaptive_run(rho, c, ps, B, h, 1.0 / dt0, 1.0, t_final=3.5 * dt0)
    assert s["stop"] == "t_final" and s["steps"] == 4 and s["rebuilds"] == 0
    assert s["dt_hist"] == [1.0 / (1.0 / dt0)] * 4
    assert abs(s["t"] - 4 * (1.0 / (1.0 / dt0))) < 1e-15
    ck = 5.0
    for _ in range(4):
        ck = (1 - s["dt"]) * ck + s["dt"] * 3.0
    assert np.allclose(r[ps.n_plus], 3.0, rtol=1e-11)
    assert np.allclose(cc[ps.n_plus], ck, rtol=1e-11)


def test_adaptive_rules_test_a():
    """Test A data on a centred sphere: the CFL bound is far below 0.5 h^2, so step 1 takes
    exactly that bound and rebuilds; dt never grows; rebuilds happen exactly when dt shrinks;
    the state keeps the sphere's symmetries; max_steps and rho_cap stop the loop."""
    h, (z, y, x), ps, B = _adaptive_case(15, 1)
    r2 = x**2 + y**2 + z**2
    rho = np.where(ps.n_plus, 1000 * np.exp(-100 * r2), 0.0)
    c = np.where(ps.n_plus, 500 * np.exp(-50 * r2), 0.0)
    sigma0 = 1.0 / (0.5 * h * h)
    r, cc, s = pks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, t_final=1.0, max_steps=4)
    assert s["stop"] == "max_steps" and s["steps"] == 4
    assert s["dt_hist"][0] == pks.cfl_dt(c, ps.m_plus, h, 1.0) < 1.0 / sigma0
    assert s["rebuilt"][0]
    prev = 1.0 / sigma0
    for dt, rb in zip(s["dt_hist"], s["rebuilt"]):
        assert dt <= prev and rb == (dt < prev)
        prev = dt
    assert s["rebuilds"] == sum(s["rebuilt"])
    assert abs(s["t"] - sum(s["dt_hist"])) < 1e-15
    for f in (r, cc):
        assert np.allclose(f, f[::-1], atol=1e-9 * np.abs(f).max())
        assert np.allclose(f, np.transpose(f, (1, 2, 0)), atol=1e-9 * np.abs(f).max())
    # Step 8: a threshold below the initial max |rho| stops before the first step
    _, _, s2 = pks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, t_final=1.0, rho_cap=100.0)
    assert s2["stop"] == "rho_cap" and s2["steps"] == 0 and s2["rho_max"] == np.max(rho[ps.m_plus])


def test_adaptive_run_jump_rule():
    """The Test B termination rule (Sec. 4): the loop stops at the first scan whose max |rho|
    exceeds the previous scan's by at least the cap, and never when the cap is disabled.  On Test
    B data at 15^3 max |rho| first falls (the first step is the large dt0) and then rises."""
    n = 15
    h, x0 = inp.grid(n)
    z, y, x = inp.mesh(n)
    ps = og.PointSets(og.inside_sphere(z, y, x))
    gz, gy, gx = og.gamma_coords(ps, x0, h)
    d, th, _ = og.project_sphere(gz, gy, gx)
    B = ob.zonal_basis_matrix(d, th, 4, beta=0)
    rho = np.where(ps.n_plus, 2000.0 * np.exp(-100.0 * (x**2 + y**2 + (z - 0.25) ** 2)), 0.0)
    c = np.zeros_like(rho)
    sigma0 = 1.0 / (0.5 * h * h)
    # the run stopped by max_steps = k reports the scan of the state after k - 1 steps
    maxes = [pks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, 1.0, max_steps=k)[2]["rho_max"]
             for k in range(1, 7)]
    jumps = np.diff(maxes)         # jumps[j]: the change over step j + 1
    first = int(np.argmax(jumps > 0))
    cap = 0.5 * jumps[first]
    _, _, ref = pks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, 1.0, max_steps=10, rho_jump_cap=cap)
    assert ref["stop"] == "rho_jump" and ref["steps"] == first + 1
    _, _, ref = pks.adaptive_run(rho, c, ps, B, h, sigma0, 1.0, 1.0, max_steps=5, rho_jump_cap=0.0)
    assert ref["stop"] == "max_steps"
