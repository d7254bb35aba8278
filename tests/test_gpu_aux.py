"""GPU parity of aux_solve / aux_solve_batched against the FP64 oracle.

Tolerances (relative max-norm per right-hand side): FP64 transforms 1e-12, FP32 transforms
1e-5, FP32 transforms + FP64 refinement 1e-10.
"""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import aux as oaux
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "refined": 1e-10}


def _solve(b_np, sigma, h, dev, **kw):
    import torch
    from paper_1811_03557_amd import api
    b = torch.from_numpy(np.ascontiguousarray(b_np)).to(dev)
    u = api.aux_solve_batched(b, sigma, h, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _max_rel(u, ref):
    return max(oaux.rel_err_inf(u[i], ref[i]) for i in range(ref.shape[0]))


@pytest.mark.parametrize("n", [7, 15, 31, 63, 127])
@pytest.mark.parametrize("sigma", [0.0, 1.0, 1e4])
def test_fp64_parity(n, sigma):
    dev = need_gpu()
    say(f"fp64 parity n={n} sigma={sigma}")
    h, _ = inp.grid(n)
    nrhs = 3 if n <= 63 else 2
    b = inp.rhs_normal(n, nrhs, seed=n)
    ref = oaux.aux_solve(b, sigma, h)
    u = _solve(b, sigma, h, dev, prec="fp64")
    assert _max_rel(u, ref) < TOL["fp64"]


@pytest.mark.parametrize("n", [7, 31, 127])
def test_fp32_io_parity(n):
    import torch
    dev = need_gpu()
    say(f"fp32 io parity n={n}")
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 2, seed=1)
    ref = oaux.aux_solve(b, 1.0, h)
    bf = torch.from_numpy(b.astype(np.float32)).to(dev)
    from paper_1811_03557_amd import api
    u = api.aux_solve_batched(bf, 1.0, h, prec="fp32").cpu().numpy().astype(np.float64)
    assert _max_rel(u, ref) < TOL["fp32"]


@pytest.mark.parametrize("n", [15, 63, 127])
@pytest.mark.parametrize("sigma", [1.0, 1e4])
def test_fp32_refined_parity(n, sigma):
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    say(f"fp32+refinement parity n={n} sigma={sigma}")
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 3, seed=2)
    ref = oaux.aux_solve(b, sigma, h)
    # without refinement: FP32 accuracy
    u0 = _solve(b, sigma, h, dev, prec="fp32", max_refine=0)
    assert _max_rel(u0, ref) < TOL["fp32"]
    bt = torch.from_numpy(b).to(dev)
    u, info = api.aux_solve_batched(bt, sigma, h, prec="fp32", max_refine=4, rtol=1e-10, info=True)
    u = u.cpu().numpy()
    assert _max_rel(u, ref) < TOL["refined"]
    assert 1 <= info["refine_iters"] <= 3


@pytest.mark.parametrize("n", [31, 255])
def test_fp64_refined_parity(n):
    """FP64 transforms with FP64 refinement (residual and update sweeps in double)."""
    dev = need_gpu()
    say(f"fp64 refined n={n}")
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 2, seed=11)
    ref = oaux.aux_solve(b, 1.0, h)
    u = _solve(b, 1.0, h, dev, prec="fp64", max_refine=2, rtol=1e-14)
    assert _max_rel(u, ref) < TOL["fp64"]


@pytest.mark.parametrize("prec,kw,modes,tol", [
    ("fp64", {}, [(1, 2, 3), (511, 300, 77)], 1e-12),
    ("fp32", {"max_refine": 4, "rtol": 1e-10}, [(1, 2, 3), (511, 300, 77)], 1e-10),
    ("fp32", {}, [(1, 2, 3), (5, 9, 2)], 1e-5)])
def test_eigenmode_closed_form_511(prec, kw, modes, tol):
    """N = 511 (a 256-point complex FFT per line): sine modes are solved exactly.  Plain FP32 is
    held to 1e-5 on low modes only: for a high mode the transforms' rounding (~eps32 log2 M of
    |b|) lands in low-frequency coefficients, divided by sigma + lambda_min = 4.3 while the
    solution is divided by sigma + lambda_mode = 2e5, so its relative error grows with that
    ratio (5e-5 measured for (511, 300, 77)); refinement brings it to 1e-10."""
    dev = need_gpu()
    n = 511
    say(f"eigenmode n=511 {prec} {kw}")
    h, _ = inp.grid(n)
    j = np.arange(1, n + 1)
    for (k1, k2, k3) in modes:
        s = [np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1)) for k in (k1, k2, k3)]
        b = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
        u = _solve(b[None], 1.0, h, dev, prec=prec, **kw)[0]
        assert oaux.rel_err_inf(u, b / (1.0 + lam)) < tol, (k1, k2, k3)


def test_eigenmode_closed_form_1023():
    """N = 1023, the largest grid the solver takes (8.6 GB per FP64 volume, 8-line tiles, a
    512-point complex FFT per line): a sine mode is solved exactly.  The separable right-hand
    side and its closed-form solution are formed on the device from FP64 sine vectors."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 1023
    say("eigenmode n=1023")
    h, _ = inp.grid(n)
    j = np.arange(1, n + 1)
    k1, k2, k3 = 5, 1000, 333
    s = [torch.from_numpy(np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1))).to(dev)
         for k in (k1, k2, k3)]
    lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
    b = (s[2][:, None, None] * s[1][None, :, None]) * s[0][None, None, :]
    u = api.aux_solve_batched(b[None], 1.0, h)[0]
    b.div_(1.0 + lam)  # the exact solution, in place
    err = (u - b).abs().max().item() / b.abs().max().item()
    say(f"n=1023 rel err {err:.2e}")
    assert err < 1e-12


def test_eigenmode_closed_form_full_size():
    """At N = 255 a single sine mode is solved exactly (property at any size)."""
    dev = need_gpu()
    n = 255
    say("eigenmode n=255")
    h, _ = inp.grid(n)
    j = np.arange(1, n + 1)
    sigma = 1.0
    out = []
    for (k1, k2, k3) in [(1, 1, 1), (255, 3, 128), (17, 200, 64)]:
        # exact integer reduction of j k keeps sin's argument below 2 pi
        s = [np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1)) for k in (k1, k2, k3)]
        b = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
        out.append((b, b / (sigma + lam)))
    b = np.stack([o[0] for o in out])
    ref = np.stack([o[1] for o in out])
    u = _solve(b, sigma, h, dev, prec="fp64")
    assert _max_rel(u, ref) < TOL["fp64"]


@pytest.mark.parametrize("sigma", [1.0, 1e4])
@pytest.mark.parametrize("prec,kw,tol", [("fp64", {}, 1e-12),
                                         ("fp32", {"max_refine": 4, "rtol": 1e-10}, 1e-10)])
def test_full_size_255_parity(prec, kw, tol, sigma):
    """The benchmark's launch configuration (N = 255) against the oracle on 2 right-hand sides,
    at both ends of the workload's sigma range (1 and 1e4)."""
    dev = need_gpu()
    n = 255
    say(f"n=255 parity {prec} sigma={sigma:g}")
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 2, seed=0)
    ref = oaux.aux_solve(b, sigma, h)
    u = _solve(b, sigma, h, dev, prec=prec, **kw)
    err = _max_rel(u, ref)
    say(f"  rel err {err:.2e}")
    assert err < tol


def test_random_rhs_511_fp64():
    """N = 511 (the paper's largest single-domain mesh of its speed-up table) on a random
    right-hand side against the oracle, FP64 at 1e-12."""
    dev = need_gpu()
    n = 511
    say("n=511 random right-hand side, fp64")
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 1, seed=5)
    ref = oaux.aux_solve(b, 1.0, h)
    u = _solve(b, 1.0, h, dev, prec="fp64")
    err = _max_rel(u, ref)
    say(f"  rel err {err:.2e}")
    assert err < TOL["fp64"]


def test_config1_manufactured():
    dev = need_gpu()
    n = 31
    h, _ = inp.grid(n)
    dt = h
    sigma = 1.0 / dt + 1.0
    ustar = inp.manufactured_c1(n, dt)
    b = oaux.apply_operator(ustar, sigma, h) + inp.noise_uniform(n, seed=0)
    ref = oaux.aux_solve(b, sigma, h)
    u = _solve(b[None], sigma, h, dev, prec="fp64")[0]
    assert oaux.rel_err_inf(u, ref) < TOL["fp64"]
    # noise-free manufactured data come back exactly
    u2 = _solve(oaux.apply_operator(ustar, sigma, h)[None], sigma, h, dev, prec="fp64")[0]
    assert oaux.rel_err_inf(u2, ustar) < TOL["fp64"]


def test_batch_chunks_and_ragged_count():
    """Results do not depend on how the batch is chunked (chunk 1, 2, all) for 5 RHS."""
    dev = need_gpu()
    n = 63
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 5, seed=9)
    us = [_solve(b, 2.0, h, dev, prec="fp32", max_refine=2, rtol=1e-12, rhs_chunk=c)
          for c in (1, 2, 0)]
    assert np.array_equal(us[0], us[1]) and np.array_equal(us[0], us[2])
    ref = oaux.aux_solve(b, 2.0, h)
    assert _max_rel(us[0], ref) < TOL["refined"]


@pytest.mark.parametrize("n", [7, 15, 31, 63, 127])
@pytest.mark.parametrize("prec,kw,tol", [
    ("fp64", {}, 1e-12),
    ("fp64", {"max_refine": 2, "rtol": 1e-14}, 1e-12),
    ("fp32", {"max_refine": 4, "rtol": 1e-10}, 1e-10),
])
def test_plane_and_axis_sweeps(n, prec, kw, tol):
    """The fused plane sweeps (both in-plane transforms of a z-plane in one pass, three sweeps
    per solve) and the five per-axis sweeps each meet the oracle on a ragged batch of 3 at two
    shifts, and agree with each other to the same bar."""
    dev = need_gpu()
    h, _ = inp.grid(n)
    for sigma in (1.0, 1e4):
        say(f"plane vs axis n={n} {prec} {kw} sigma={sigma:g}")
        b = inp.rhs_normal(n, 3, seed=n + 17)
        ref = oaux.aux_solve(b, sigma, h)
        up = _solve(b, sigma, h, dev, prec=prec, sweeps="plane", rhs_chunk=2, **kw)
        ua = _solve(b, sigma, h, dev, prec=prec, sweeps="axis", rhs_chunk=2, **kw)
        ep, ea = _max_rel(up, ref), _max_rel(ua, ref)
        say(f"  rel err plane {ep:.2e}, axis {ea:.2e}")
        assert ep < tol and ea < tol
        assert _max_rel(up, ua) < tol


@pytest.mark.parametrize("n", [31, 127])
def test_plane_sweeps_fp32_io(n):
    """FP32 input and output through the plane sweeps: the FP32 bar (1e-5) against the
    oracle."""
    dev = need_gpu()
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 2, seed=n + 3)
    ref = oaux.aux_solve(b, 1.0, h)
    u = _solve(b.astype(np.float32), 1.0, h, dev, prec="fp32", sweeps="plane")
    assert _max_rel(u.astype(np.float64), ref) < TOL["fp32"]


def test_plane_sweeps_sine_modes_127():
    """Closed form through the plane sweeps: b = s_k1 x s_k2 x s_k3 (the DST-I eigenvectors) gives
    u = b / (sigma + lambda_k1 + lambda_k2 + lambda_k3), with k1 != k2 so that a transposed
    spectral plane read the wrong way round would show."""
    dev = need_gpu()
    n = 127
    h, _ = inp.grid(n)
    j = np.arange(1, n + 1)
    sigma = 3.0
    bs, refs = [], []
    for (k1, k2, k3) in [(1, 2, 3), (127, 5, 64), (40, 90, 1)]:
        s = [np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1)) for k in (k1, k2, k3)]
        bm = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
        bs.append(bm)
        refs.append(bm / (sigma + lam))
    u = _solve(np.stack(bs), sigma, h, dev, prec="fp64", sweeps="plane")
    assert _max_rel(u, np.stack(refs)) < TOL["fp64"]


def test_invalid_arguments_raise():
    import torch
    from paper_1811_03557_amd import api, _lib
    dev = need_gpu()
    b = torch.zeros((5, 5, 5), dtype=torch.float64, device=dev)   # n below the smallest size
    with pytest.raises(_lib.DPMError):
        api.aux_solve(b, 1.0, 0.1)
    b = torch.zeros((7, 7, 7), dtype=torch.float64, device=dev)
    with pytest.raises(_lib.DPMError):
        api.aux_solve(b, -1.0, 0.1)
    with pytest.raises(_lib.DPMError):
        api.aux_solve(b, 1.0, 0.0)


@pytest.mark.parametrize("n", [15, 63, 127, 255])
def test_bf16x3_parity(n):
    """Split-bf16 MFMA sweeps: ~1e-5 per transform unrefined (the dropped lo*lo product is
    ~2^-16 relative; six transforms -> tolerance 1e-4), 1e-10 after FP64 refinement."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    say(f"bf16x3 parity n={n}")
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 2, seed=4)
    ref = oaux.aux_solve(b, 1.0, h)
    u0 = _solve(b, 1.0, h, dev, prec="bf16x3", max_refine=0)
    assert _max_rel(u0, ref) < 1e-4
    bt = torch.from_numpy(b).to(dev)
    u, info = api.aux_solve_batched(bt, 1.0, h, prec="bf16x3", max_refine=6, rtol=1e-10, info=True)
    assert _max_rel(u.cpu().numpy(), ref) < TOL["refined"]
    assert info["refine_iters"] >= 1


def test_per_rhs_sigma_matches_single_solves():
    """A batch with one sigma per right-hand side equals the solves one at a time, bitwise."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 63
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 4, seed=8)
    sig = [1.0, 37.5, 1e4, 0.0]
    bt = torch.from_numpy(b).to(dev)
    for prec, mr in (("fp64", 0), ("fp32", 3)):
        ub = api.aux_solve_batched_sigma(bt, sig, h, prec=prec, max_refine=mr, rtol=1e-10).cpu().numpy()
        for i, s in enumerate(sig):
            ui = api.aux_solve_batched(bt[i:i + 1].contiguous(), s, h, prec=prec, max_refine=mr,
                                       rtol=1e-10).cpu().numpy()[0]
            assert np.array_equal(ub[i], ui), (prec, i)
            assert oaux.rel_err_inf(ub[i], oaux.aux_solve(b[i], s, h)) < 1e-10


@pytest.mark.parametrize("n", [7, 15, 31, 63, 127, 255, 36, 68, 132, 260])
def test_fp64_gemm_parity(n):
    """FP64 dense-DST sweeps on the FP64 matrix cores (the GEMM form): the FP64 bar, 1e-12,
    against the oracle on a ragged batch of 3 (chunk 2 at 255^3: a full and a partial launch)
    and on sine modes in closed form.  36, 68, 132 and 260 are meshes of the paper's tables,
    N + 1 not a power of two (matrix padded to 64, 96, 160 and 288)."""
    dev = need_gpu()
    say(f"fp64 gemm parity n={n}")
    h, _ = inp.grid(n)
    nrhs = 3 if n <= 127 else 2
    b = inp.rhs_normal(n, nrhs, seed=n + 1)
    ref = oaux.aux_solve(b, 1.0, h)
    u = _solve(b, 1.0, h, dev, prec="fp64_gemm")
    assert _max_rel(u, ref) < TOL["fp64"]
    if n >= 127:
        u2 = _solve(b, 1.0, h, dev, prec="fp64_gemm", rhs_chunk=1)
        assert np.array_equal(u, u2)  # the chunking does not change the arithmetic
    j = np.arange(1, n + 1)
    ks = [(1, 1, 1), (n, 2, (n + 1) // 2)]
    bs, refs = [], []
    for (k1, k2, k3) in ks:
        s = [np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1)) for k in (k1, k2, k3)]
        bm = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
        bs.append(bm)
        refs.append(bm / (1e4 + lam))
    um = _solve(np.stack(bs), 1e4, h, dev, prec="fp64_gemm")
    assert _max_rel(um, np.stack(refs)) < TOL["fp64"]


def test_fp64_gemm_rejects_refinement_and_large_n():
    import torch
    from paper_1811_03557_amd import api, _lib
    dev = need_gpu()
    b = torch.zeros((2, 7, 7, 7), dtype=torch.float64, device=dev)
    with pytest.raises(_lib.DPMError):
        api.aux_solve_batched(b, 1.0, 0.1, prec="fp64_gemm", max_refine=1)
    b = torch.zeros((1, 600, 600, 600), dtype=torch.float64, device=dev)
    with pytest.raises(_lib.DPMError) as e:  # beyond the dense sizes
        api.aux_solve_batched(b, 1.0, 3.0 / 601, prec="fp64_gemm")
    assert "n <= 543" in str(e.value)
    del b
    # the FP32 FFT form needs N + 1 a power of two, and says where to go otherwise
    b = torch.zeros((1, 36, 36, 36), dtype=torch.float64, device=dev)
    with pytest.raises(_lib.DPMError) as e:
        api.aux_solve_batched(b, 1.0, 3.0 / 37, prec="fp32", max_refine=2)
    assert "DPM_FP64_GEMM" in str(e.value) and "Bluestein" in str(e.value)


# Bluestein's sweeps: the FP64 FFT form for N + 1 not a power of two.  36, 68, 132, 260 and 516
# are meshes of the paper's tables; 9, 100 and 341 (the longest line at L = 1024) and 342 (the
# shortest at L = 2048) cover the table sizes' edges.
@pytest.mark.parametrize("n", [9, 36, 68, 100, 132, 260, 341, 342, 516])
def test_bluestein_parity(n):
    """Random right-hand sides against the oracle's dense DST-I at the FP64 bar (1e-12), at two
    shifts; a ragged batch of 3 at n <= 132."""
    dev = need_gpu()
    say(f"bluestein parity n={n}")
    h, _ = inp.grid(n)
    nrhs = 3 if n <= 132 else 1
    b = inp.rhs_normal(n, nrhs, seed=n + 7)
    for sigma in (1.0, 1e4):
        ref = oaux.aux_solve(b, sigma, h)
        u = _solve(b, sigma, h, dev, prec="fp64")
        err = _max_rel(u, ref)
        say(f"  sigma {sigma:g}: rel err {err:.2e}")
        assert err < TOL["fp64"]


@pytest.mark.parametrize("n", [36, 260, 516])
def test_bluestein_sine_modes(n):
    """Closed form through Bluestein's sweeps: b = s_k1 x s_k2 x s_k3 gives
    u = b / (sigma + lambda_k1 + lambda_k2 + lambda_k3), with the highest and middle modes."""
    dev = need_gpu()
    h, _ = inp.grid(n)
    j = np.arange(1, n + 1)
    sigma = 2.0
    bs, refs = [], []
    for (k1, k2, k3) in [(1, 2, 3), (n, (n + 1) // 2, 7)]:
        s = [np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1)) for k in (k1, k2, k3)]
        bm = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
        bs.append(bm)
        refs.append(bm / (sigma + lam))
    u = _solve(np.stack(bs), sigma, h, dev, prec="fp64")
    assert _max_rel(u, np.stack(refs)) < TOL["fp64"]


def test_bluestein_agrees_with_dense_form():
    """The two FP64 forms for N + 1 not a power of two, Bluestein's FFT sweeps and the dense
    products on the FP64 matrix cores, agree to the FP64 bar at N = 260."""
    dev = need_gpu()
    n = 260
    h, _ = inp.grid(n)
    b = inp.rhs_normal(n, 2, seed=3)
    u1 = _solve(b, 1.0, h, dev, prec="fp64")
    u2 = _solve(b, 1.0, h, dev, prec="fp64_gemm")
    assert _max_rel(u1, u2) < TOL["fp64"]
