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
    _replay_steps_alone(srv, out, init)
    s = serve.summarize(out)
    say(f"serve: {s['requests_per_s']:.0f} req/s, p50 {s['p50_ms']:.2f} ms, "
        f"p99 {s['p99_ms']:.2f} ms, mean batch {s['mean_batch']:.2f}")
    assert srv.footprint() <= srv.budget


def _standalone(srv, sid):
    """A fresh handle and initial state of simulation sid, built as the server builds them."""
    from paper_1811_03557_amd import api
    s = srv.sims[sid]
    h = 3.0 / (s.n + 1)
    x0 = -1.5 + h
    geo = api.geometry("sphere", axes=(1.0,))
    m = api.classify(s.n, h, x0, geo, device=srv.device)
    idx, _ = api.gamma_points(m, h, x0)
    B, _ = api.basis(s.n, h, x0, geo, idx, srv.lmax, 1)
    bep = api.build_boundary_matrix(m, B, s.n, h, s.sigma, x0)
    return bep, api.gauss_state(bep, geo, 1000.0, 100.0), api.gauss_state(bep, geo, 500.0, 50.0)


def _replay_steps_alone(srv, out, init=None):
    import torch
    from paper_1811_03557_amd import api
    for sid, sim in srv.sims.items():
        mine = [r for r in out if r.sim == sid and r.kind == "step"]
        if not mine:
            continue
        bep, rho, cc = _standalone(srv, sid)
        if init is not None and sid in init:
            assert torch.equal(rho, init[sid][0]) and torch.equal(cc, init[sid][1])
        for r in mine:
            rho, cc = api.dpm_step(bep, 1.0 / bep.sigma, srv.chi, rho, cc)
            assert torch.equal(rho, r.out[0]) and torch.equal(cc, r.out[1]), (sid, r.rid)
        bep.close()


def test_small_budget_defers_and_evicts_simulations():
    """Admission by HBM footprint: with a budget that holds the rings' minimum and one resident
    DPM simulation, the other step simulations are deferred, made resident in turn by evicting
    idle ones (state to the host, handle rebuilt later), and every result still equals the
    simulation's steps run alone."""
    from paper_1811_03557_amd import api, serve
    dev = need_gpu()
    sims = [serve.Simulation(i, 31, 1.0 / (0.5 * (3.0 / 32) ** 2), "step") for i in range(3)]
    sims.append(serve.Simulation(3, 15, 30.0, "aux"))
    reqs = []
    for k in range(12):
        sid = k % 4
        reqs.append(serve.Request(k, sid, sims[sid].kind, sims[sid].n, sims[sid].sigma, 0.0))
    # measure one simulation's resident bytes with a generous budget, then size the budget to
    # the minimum plus that one simulation (the rest must wait)
    probe = serve.Server(sims[:1] + sims[3:], device=dev, hbm_budget=4e9, max_batch=2, lmax=2)
    one = probe.sim_bytes[0]
    step_ws = probe.lane_of[0].step_ws.numel()
    minimum = probe.footprint() - one - step_ws - (probe.classes[15].slots - 1) * 2 * 8 * 15 ** 3 \
        - (probe.classes[31].slots - 1) * 2 * 8 * 31 ** 3
    budget = minimum + one + step_ws + 1024
    say(f"serve small budget: one simulation {one} B + step workspace {step_ws} B, "
        f"budget {budget} B")
    srv = serve.Server(sims, device=dev, hbm_budget=budget, max_batch=2, lmax=2,
                       keep_results=True)
    assert len(srv.bep) == 1 and srv.deferred == {1, 2}
    out = srv.run(reqs)
    assert all(np.isfinite(r.t_done) for r in out)
    assert srv.evictions >= 2
    assert srv.footprint() <= srv.budget
    _replay_steps_alone(srv, out)
    say(f"serve small budget: {srv.evictions} evictions, footprint {srv.footprint()} B")
