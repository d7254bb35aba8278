"""Split layout of the FFT-form solve (n = 255, 511): the y sweeps around the z solve cut into
its segment-local elimination (fused with the forward x transforms), the separators' reduced
system, and the reconstruction (fused with the inverse x transforms).  Four passes over the
volume and a small one instead of five.

Parity: FP64 1e-12 and FP32 (FP32 I/O) 1e-5 against the oracle, per right-hand side, on ragged
batches at both ends of the sigma range; the split and per-axis layouts agree to the same bars.
The split layout is the library's choice for plain solves at 511, so the 511^3 parity tests of
test_gpu_aux.py run it too.
"""
import ctypes as C

import numpy as np
import pytest

import dpm_inputs as inp
from oracle import aux as oaux
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _solve(b_np, sigma, h, dev, **kw):
    import torch
    from paper_1811_03557_amd import api
    b = torch.from_numpy(np.ascontiguousarray(b_np)).to(dev)
    u = api.aux_solve_batched(b, sigma, h, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _max_rel(u, ref):
    return max(oaux.rel_err_inf(u[i], ref[i]) for i in range(ref.shape[0]))


@pytest.mark.parametrize("sigma", [1.0, 1e4])
def test_split_and_axis_fp64_255(sigma):
    """FP64 at 255^3, 3 right-hand sides at 2 per launch (a ragged last launch): both layouts
    meet the oracle at 1e-12 and each other."""
    dev = need_gpu()
    n = 255
    h, _ = inp.grid(n)
    say(f"split vs axis fp64 n=255 sigma={sigma:g}")
    b = inp.rhs_normal(n, 3, seed=31)
    ref = oaux.aux_solve(b, sigma, h)
    us = _solve(b, sigma, h, dev, prec="fp64", sweeps="split", rhs_chunk=2)
    ua = _solve(b, sigma, h, dev, prec="fp64", sweeps="axis", rhs_chunk=2)
    es, ea = _max_rel(us, ref), _max_rel(ua, ref)
    say(f"  rel err split {es:.2e}, axis {ea:.2e}")
    assert es < 1e-12 and ea < 1e-12
    assert _max_rel(us, ua) < 1e-12


def test_split_fp32_io_255():
    """FP32 input and output (plain FP32 transforms) through the split layout: the FP32 bar
    (1e-5) against the oracle, at one and three right-hand sides per launch."""
    dev = need_gpu()
    n = 255
    h, _ = inp.grid(n)
    say("split fp32 io n=255")
    b = inp.rhs_normal(n, 3, seed=32)
    ref = oaux.aux_solve(b, 1.0, h)
    for chunk in (1, 3):
        u = _solve(b.astype(np.float32), 1.0, h, dev, prec="fp32", sweeps="split", rhs_chunk=chunk)
        err = _max_rel(u.astype(np.float64), ref)
        say(f"  {chunk} per launch: rel err {err:.2e}")
        assert err < 1e-5


def test_split_sigma_per_rhs_255():
    """One shift per right-hand side (0, 1, 1e4) through the split layout: each right-hand side
    meets the oracle at its own sigma."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 255
    h, _ = inp.grid(n)
    sig = [0.0, 1.0, 1e4]
    say("split per-rhs sigma n=255")
    b = inp.rhs_normal(n, 3, seed=33)
    u = api.aux_solve_batched_sigma(torch.from_numpy(b).to(dev), sig, h, sweeps="split",
                                    rhs_chunk=2).cpu().numpy()
    for i, s in enumerate(sig):
        err = oaux.rel_err_inf(u[i], oaux.aux_solve(b[i:i + 1], s, h)[0])
        say(f"  sigma {s:g}: rel err {err:.2e}")
        assert err < 1e-12


def test_split_sine_modes_511():
    """Closed form at 511 through the split layout (32 segments per column, two transform rounds
    per tile): b = s_k1 x s_k2 x s_k3 gives u = b / (sigma + lambda_k1 + lambda_k2 + lambda_k3),
    with k1 != k2 so that an exchange of the x and y roles would show."""
    dev = need_gpu()
    n = 511
    h, _ = inp.grid(n)
    j = np.arange(1, n + 1)
    say("split sine modes n=511")
    for (k1, k2, k3) in [(1, 2, 3), (511, 300, 77), (17, 450, 256)]:
        s = [np.sin(np.pi * ((j * k) % (2 * (n + 1))) / (n + 1)) for k in (k1, k2, k3)]
        bm = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        lam = sum(4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 for k in (k1, k2, k3))
        u = _solve(bm[None], 2.0, h, dev, prec="fp64", sweeps="split")[0]
        err = oaux.rel_err_inf(u, bm / (2.0 + lam))
        say(f"  modes {(k1, k2, k3)}: rel err {err:.2e}")
        assert err < 1e-12


def test_split_workspace_fallback_511():
    """A workspace sized without the separator planes at 511, where the split layout is the
    library's choice: the solve runs the per-axis sweeps (bitwise equal to an explicit per-axis
    solve); an explicit split request with it is rejected."""
    import torch
    from paper_1811_03557_amd import _lib as L, api
    dev = need_gpu()
    lib = L.load()
    n = 511
    h, _ = inp.grid(n)
    say("split workspace fallback n=511")
    b = torch.randn((2, n, n, n), dtype=torch.float64, device=dev,
                    generator=torch.Generator(device=dev).manual_seed(34))
    g = api.grid(n, h, 1.0)
    small = api.workspace_size(g, 2, api.opts("fp64", sweeps="axis"))
    full = api.workspace_size(g, 2, api.opts("fp64"))
    assert full > small
    ws = torch.empty(max(small, 1), dtype=torch.uint8, device=dev)
    outs = {}
    for sw in ("auto", "split"):
        o = api.opts("fp64", sweeps=sw)
        o.workspace = C.c_void_p(ws.data_ptr())
        o.workspace_bytes = small
        u = torch.empty_like(b)
        st = lib.aux_solve_batched(C.byref(g), 2, C.c_void_p(b.data_ptr()), C.c_void_p(u.data_ptr()),
                                   C.byref(o), None, None)
        outs[sw] = (st, u)
    torch.cuda.synchronize()
    assert outs["auto"][0] == L.DPM_OK
    assert outs["split"][0] == L.DPM_EINVAL
    ua = api.aux_solve_batched(b, 1.0, h, prec="fp64", sweeps="axis")
    assert torch.equal(outs["auto"][1], ua)


def test_split_noalloc_255():
    """The allocation-free entry point at 255^3 (separator planes in the static scratch) equals
    the workspace entry point bitwise."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n = 255
    h, _ = inp.grid(n)
    say("split noalloc n=255")
    api.prepare(n)
    b = torch.from_numpy(inp.rhs_normal(n, 2, seed=35)).to(dev)
    u0 = api.aux_solve_batched(b, 1.0, h, prec="fp64", sweeps="split")
    u1 = api.aux_solve_batched_noalloc(b, 1.0, h, prec="fp64", sweeps="split")
    torch.cuda.synchronize()
    assert torch.equal(u0, u1)
