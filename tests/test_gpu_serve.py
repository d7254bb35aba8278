"""Continuous-batching server: every served result equals the same request run alone."""
import numpy as np
import pytest

import dpm_inputs as inp
from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lanes", [1, 2])
def test_served_results_equal_standalone_runs(lanes):
    import torch
    from paper_1811_03557_amd import api, serve
    dev = need_gpu()
    sims, reqs = serve.build_requests(*inp.serving_workload(
        n_sims=8, n_requests=48, seed=3, sizes=(15, 31, 63), closed_loop=True))
    say(f"serve: {len(sims)} simulations, {len(reqs)} requests")
    srv = serve.Server(sims, device=dev, hbm_budget=2e8, max_batch=4, lmax=2, keep_results=True,
                       lanes=lanes)
    # initial states, before any step runs
    init = {sid: (r.clone(), c.clone()) for sid, (r, c) in srv.state.items()}
    out = srv.run(reqs)
    assert all(np.isfinite(r.t_done) for r in out)
    assert any(r.batch > 1 for r in out if r.kind == "aux")
    # aux requests: a solve of the slot's right-hand side with the request's sigma, alone
    for r in out:
        if r.kind != "aux":
            continue
        c = srv.classes[r.n]
        ref = api.aux_solve_batched(c.b[r.slot:r.slot + 1], r.sigma, c.h)[0]
        assert torch.equal(r.out, ref), (r.rid, r.n, r.sigma, r.batch)
    # step requests: the simulation's steps replayed alone, in arrival order
    for sid, (rho, cc) in init.items():
        mine = [r for r in out if r.sim == sid]
        if not mine:
            continue
        bep = srv.bep[sid]
        for r in mine:
            rho, cc = api.dpm_step(bep, 1.0 / bep.sigma, srv.chi, rho, cc)
            assert torch.equal(rho, r.out[0]) and torch.equal(cc, r.out[1]), (sid, r.rid)
    s = serve.summarize(out)
    say(f"serve: {s['requests_per_s']:.0f} req/s, p50 {s['p50_ms']:.2f} ms, "
        f"p99 {s['p99_ms']:.2f} ms, mean batch {s['mean_batch']:.2f}")
