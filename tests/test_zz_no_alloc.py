"""The allocation-free entry point aux_solve_batched_noalloc against aux_solve_batched (collected
last: a failure here hides no other test).

Both entry points run the same kernels; the no-allocation one takes its workspace from the
library's static device scratch instead of the caller.  Each case runs two calls in a row through
the C ABI (the second with a smaller input, so the scratch holds the first call's contents when
the second starts) and requires the results to equal those of aux_solve_batched bit for bit, and
to meet the refined tolerance (1e-10 relative) against the FP64 oracle on the small case.
"""
import ctypes as C

import numpy as np
import pytest

import dpm_inputs as inp
from oracle import aux as oaux
from tests.gpu_util import need_gpu, say


def _pair(dev, n, nrhs, seed, sigma, prec, max_refine):
    import torch
    from paper_1811_03557_amd import api
    h, _ = inp.grid(n)
    b = torch.from_numpy(inp.rhs_normal(n, nrhs, seed=seed)).to(dev)
    kw = {"prec": prec, "max_refine": max_refine, "rtol": 1e-10}
    ref, ri = api.aux_solve_batched(b, sigma, h, info=True, **kw)
    u = torch.full_like(b, float("nan"))
    got, gi = api.aux_solve_batched_noalloc(b, sigma, h, out=u, info=True, **kw)
    torch.cuda.synchronize()
    return b.cpu().numpy(), ref.cpu().numpy(), ri, got.cpu().numpy(), gi


@pytest.mark.gpu
@pytest.mark.parametrize("prec,max_refine", [("fp32", 4), ("fp64", 0)])
def test_noalloc_equals_workspace_entry_point(prec, max_refine):
    dev = need_gpu()
    from paper_1811_03557_amd import api
    for n in (127, 63):
        api.prepare(n)
    # first call: 127^3 x 3 right-hand sides; second: 63^3 x 2 (smaller), same scratch
    for (n, nrhs, seed, sigma) in [(127, 3, 11, 1.0), (63, 2, 12, 1e4)]:
        say(f"noalloc {prec} n={n} nrhs={nrhs} sigma={sigma:g}")
        b, ref, ri, got, gi = _pair(dev, n, nrhs, seed, sigma, prec, max_refine)
        assert np.array_equal(got, ref), f"n={n}: differs from aux_solve_batched"
        assert gi == ri
        if n == 63:
            h, _ = inp.grid(n)
            orc = oaux.aux_solve(b, sigma, h)
            err = max(oaux.rel_err_inf(got[i], orc[i]) for i in range(nrhs))
            say(f"  rel err vs oracle {err:.2e}")
            assert err < (1e-10 if prec == "fp32" else 1e-12)


@pytest.mark.gpu
def test_noalloc_full_size_fp32_refined():
    """One 255^3 right-hand side with FP32 transforms and FP64 refinement: the transform volume
    (63.3 MiB) fills most of the static scratch; then a smaller call."""
    dev = need_gpu()
    from paper_1811_03557_amd import api
    api.prepare(255)
    api.prepare(31)
    for (n, nrhs, seed) in [(255, 1, 3), (31, 4, 4)]:
        say(f"noalloc fp32 refined n={n} nrhs={nrhs}")
        _, ref, ri, got, gi = _pair(dev, n, nrhs, seed, 1.0, "fp32", 4)
        assert np.array_equal(got, ref)
        assert gi == ri and gi["refine_iters"] >= 1


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    """Host-side size check, before any device call: one 511^3 FP32 transform volume (534 MB)
    exceeds the 64 MiB static scratch; so does a fixed launch width of 2 at 255^3."""
    from paper_1811_03557_amd import _lib as L
    lib = L.load()
    assert L.DPM_NOALLOC_SCRATCH_BYTES == 64 << 20
    n = 511
    g = L.Grid(n, 3.0 / (n + 1), 1.0, -1.5 + 3.0 / (n + 1))
    o = L.Opts(L.DPM_FP32, 1, 1e-10, 4, 0, None, 0)
    p = C.c_void_p(16)  # never dereferenced: the call fails in its host-side checks
    q = C.c_void_p(16 + 8 * n ** 3)
    st = lib.aux_solve_batched_noalloc(C.byref(g), 1, p, q, C.byref(o), None, None)
    assert st == L.DPM_EINVAL
    assert b"static maximum" in lib.dpm_last_error()
    n = 255
    g = L.Grid(n, 3.0 / (n + 1), 1.0, -1.5 + 3.0 / (n + 1))
    o = L.Opts(L.DPM_FP32, 1, 1e-10, 4, 2, None, 0)
    q = C.c_void_p(16 + 16 * n ** 3)
    st = lib.aux_solve_batched_noalloc(C.byref(g), 2, p, q, C.byref(o), None, None)
    assert st == L.DPM_EINVAL
    assert b"rhs_chunk = 2" in lib.dpm_last_error()
