"""The launch-shape autotuner (dpm_autotune) through the C ABI: it times every candidate width
that fits, in both sweep layouts where a fused layout exists (plane at n <= 127, split at 255
and 511), then the z pass's columns per
block at the best pair, records the fastest shape, and later solves with rhs_chunk = 0
(sweeps = auto) take it.  A solve's result depends neither on the width (each right-hand side's
arithmetic is the same) nor on the z tile (each column's is), so solves at the tuned shape are
compared bit for bit with width-1 solves and with default-shape solves, and against the oracle
at the FP64 (1e-12) and refined (1e-10) tolerances."""
import numpy as np
import pytest

import dpm_inputs as inp
from oracle import aux as oaux
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,max_refine,tol", [("fp64", 0, 1e-12), ("fp32", 3, 1e-10)])
def test_autotune_records_fastest_width(prec, max_refine, tol):
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n, nrhs = 63, 8
    h, _ = inp.grid(n)
    sigma = 1.0 / h + 1.0
    b = inp.rhs_normal(n, nrhs, seed=11)
    bt = torch.from_numpy(b).to(dev)
    say(f"autotune n={n} nrhs={nrhs} {prec} max_refine={max_refine}")
    api.autotune_reset()
    try:
        default = api.rhs_chunk(api.grid(n, h, sigma), nrhs, api.opts(prec, True, 1e-10, max_refine))
        res = api.autotune(bt, sigma, h, prec=prec, max_refine=max_refine, reps=2)
        say(f"  widths {res['widths']}, layouts {res['sweeps']}, z columns {res['zcols']}, "
            f"ms {[round(t, 3) for t in res['ms']]}, best {res['best']} {res['best_sweeps']} "
            f"z {res['best_zcols']} (default width {default})")
        # every candidate width up to nrhs (the default width at this size is far above 8), in
        # both sweep layouts (the plane sweeps exist at 63), then 16, 32 and 64 z columns per
        # block (4 segments of 16 rows per column at 63: all fit) at the best pair
        k = int(np.argmin(res["ms"][:12]))
        assert res["widths"] == [1, 2, 3, 4, 6, 8] * 2 + [res["widths"][k]] * 3
        assert res["sweeps"] == ["axis"] * 6 + ["plane"] * 6 + [res["sweeps"][k]] * 3
        assert res["zcols"] == [0] * 12 + [16, 32, 64]
        assert all(np.isfinite(t) and t > 0 for t in res["ms"])
        assert res["best"] == res["widths"][k] and res["best_sweeps"] == res["sweeps"][k]
        kz = int(np.argmin(res["ms"]))
        assert res["best_zcols"] == (res["zcols"][kz] if res["ms"][kz] < res["ms"][k] else 0)
        # solves that leave the layout to the library take the recorded one
        u_fixed = api.aux_solve_batched(bt, sigma, h, prec=prec, max_refine=max_refine,
                                        sweeps=res["best_sweeps"]).cpu().numpy()
        o = api.opts(prec, True, 1e-10, max_refine)
        assert api.rhs_chunk(api.grid(n, h, sigma), nrhs, o) == res["best"]
        u_auto = api.aux_solve_batched(bt, sigma, h, prec=prec, max_refine=max_refine).cpu().numpy()
        u_one = api.aux_solve_batched(bt, sigma, h, prec=prec, max_refine=max_refine,
                                      rhs_chunk=1).cpu().numpy()
        assert np.array_equal(u_auto, u_one)
        assert np.array_equal(u_auto, u_fixed)
        ref = oaux.aux_solve(b[:2], sigma, h)
        err = max(oaux.rel_err_inf(u_auto[i], ref[i]) for i in range(2))
        say(f"  rel err vs oracle {err:.2e}")
        assert err <= tol
    finally:
        api.autotune_reset()
    # the default shape (every z tile default) gives the same bits in the same layout
    u_def = api.aux_solve_batched(bt, sigma, h, prec=prec, max_refine=max_refine,
                                  sweeps=res["best_sweeps"]).cpu().numpy()
    assert np.array_equal(u_def, u_fixed)
    assert api.rhs_chunk(api.grid(n, h, sigma), nrhs, api.opts(prec, True, 1e-10, max_refine)) == default


def test_solve_narrows_width_to_its_workspace():
    """A solve with rhs_chunk = 0 reads the width once and narrows it to what the caller's
    workspace holds: a workspace sized for one right-hand side per launch (as one sized before a
    re-tune or a reset can be) gives the same result as the default width, with no error."""
    import ctypes as C

    import torch
    from paper_1811_03557_amd import _lib as L
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n, nrhs = 31, 6
    h, _ = inp.grid(n)
    sigma = 1.0 / h + 1.0
    b = inp.rhs_normal(n, nrhs, seed=12)
    bt = torch.from_numpy(b).to(dev)
    g = api.grid(n, h, sigma)
    api.autotune_reset()
    o1 = api.opts("fp32", True, 1e-10, 3, 1)
    small = api.workspace_size(g, nrhs, o1)
    o = api.opts("fp32", True, 1e-10, 3, 0)
    assert api.rhs_chunk(g, nrhs, o) > 1
    assert api.workspace_size(g, nrhs, o) > small
    say(f"narrowed width n={n} nrhs={nrhs}: workspace {small} bytes (one right-hand side per launch)")
    ws = torch.empty(small, dtype=torch.uint8, device=dev)
    o.workspace = C.c_void_p(ws.data_ptr())
    o.workspace_bytes = small
    u = torch.empty_like(bt)
    st = L.load().aux_solve_batched(C.byref(g), nrhs, C.c_void_p(bt.data_ptr()),
                                    C.c_void_p(u.data_ptr()), C.byref(o), None, None)
    L.check(st)
    torch.cuda.synchronize()
    u_def = api.aux_solve_batched(bt, sigma, h, prec="fp32", max_refine=3)
    assert torch.equal(u, u_def)
    # a fixed width (rhs_chunk > 0) is never narrowed: too small a workspace is an error
    o2 = api.opts("fp32", True, 1e-10, 3, 2)
    o2.workspace = C.c_void_p(ws.data_ptr())
    o2.workspace_bytes = small
    st = L.load().aux_solve_batched(C.byref(g), nrhs, C.c_void_p(bt.data_ptr()),
                                    C.c_void_p(u.data_ptr()), C.byref(o2), None, None)
    assert st == L.DPM_EINVAL


def test_autotune_times_split_layout_255():
    """At 255 the autotuner times every width in the per-axis and the split layouts (the z
    tiles only when the per-axis layout wins: the split layout has no z pass), records the
    fastest, and a later solve that leaves the layout to the library takes it: bitwise equal to
    a solve with that layout fixed, and within the FP64 bar of the oracle."""
    import torch
    from paper_1811_03557_amd import api
    dev = need_gpu()
    n, nrhs = 255, 4
    h, _ = inp.grid(n)
    sigma = 1.0
    b = inp.rhs_normal(n, nrhs, seed=13)
    bt = torch.from_numpy(b).to(dev)
    say(f"autotune n={n} nrhs={nrhs} fp64 (per-axis and split layouts)")
    api.autotune_reset()
    try:
        res = api.autotune(bt, sigma, h, prec="fp64", reps=2)
        say(f"  widths {res['widths']}, layouts {res['sweeps']}, z columns {res['zcols']}, "
            f"ms {[round(t, 3) for t in res['ms']]}, best {res['best']} {res['best_sweeps']} "
            f"z {res['best_zcols']}")
        k = int(np.argmin(res["ms"][:8]))
        assert res["widths"][:8] == [1, 2, 3, 4] * 2
        assert res["sweeps"][:8] == ["axis"] * 4 + ["split"] * 4
        if res["sweeps"][k] == "split":
            assert len(res["ms"]) == 8 and res["best_zcols"] == 0
        else:
            assert res["zcols"] == [0] * 8 + [16, 32, 64]
        assert res["best"] == res["widths"][k] and res["best_sweeps"] == res["sweeps"][k]
        u_auto = api.aux_solve_batched(bt, sigma, h, prec="fp64").cpu().numpy()
        u_fixed = api.aux_solve_batched(bt, sigma, h, prec="fp64", rhs_chunk=res["best"],
                                        sweeps=res["best_sweeps"]).cpu().numpy()
        assert np.array_equal(u_auto, u_fixed)
        ref = oaux.aux_solve(b[:2], sigma, h)
        err = max(oaux.rel_err_inf(u_auto[i], ref[i]) for i in range(2))
        say(f"  rel err vs oracle {err:.2e}")
        assert err <= 1e-12
    finally:
        api.autotune_reset()
