"""Continuous-batching server for auxiliary-problem and DPM-step requests on one GPU.

Many simulations issue requests of uneven grid sizes.  Each grid size N is a size class with its
own HIP stream(s), so work of different classes overlaps on the device (one stream per class by
default: a second stream let two large requests of one class slow each other down, measured).  An aux
request owns a slot of its class's ring of device-resident right-hand-side/solution buffers;
ready requests in consecutive slots are launched together as one `aux_solve_batched_sigma` (each
keeps its own sigma), so requests that arrive while others run join the next launch instead of
waiting for a fixed batch.  A DPM-step request advances its simulation's resident state with its
resident boundary matrix (`dpm_step`); every simulation is pinned to one stream of its class, so
its steps run in arrival order.  Each stream has its own workspaces.

Admission by HBM footprint.  Every device byte the server keeps is charged to `hbm_budget`: each
class's minimum (one slot and its lanes' solve workspaces), the resident DPM simulations (boundary
-matrix handle, state and the step workspace of their lane), then the slot rings, which share
what is left equally.  DPM simulations are made resident in order while they fit; one that does
not is deferred: its step requests wait until it fits, which happens when an idle resident
simulation (no queued or running step) is evicted -- its state goes to host memory and its
handle is destroyed, to be rebuilt (the build is deterministic) when it is needed again.  Aux
requests are admitted per class, first come first served, when a slot of their class is free (a
full class does not hold up the others).  Completion times come from GPU events; latency is
arrival -> completion.

Host orchestration only: every arithmetic step runs in libdpm's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import api


@dataclasses.dataclass
class Request:
    rid: int
    sim: int
    kind: str            # "aux" or "step"
    n: int
    sigma: float
    arrival: float       # seconds after the start of the run
    slot: int = -1
    t_done: float = float("nan")
    batch: int = 0
    out: object = None   # copy of the solution, when the server keeps results

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclasses.dataclass
class Simulation:
    sid: int
    n: int
    sigma: float
    kind: str            # "aux" or "step"


class Lane:
    """One stream of a size class with its own solve and step workspaces."""

    def __init__(self, device, aux_ws_bytes: int):
        self.stream = torch.cuda.Stream(device=device)
        self.ws = torch.empty(max(1, aux_ws_bytes), dtype=torch.uint8, device=device)
        self.step_ws = None
        self.steps: collections.deque = collections.deque()  # step requests pinned here
        self.inflight = 0


class SizeClass:
    def __init__(self, n: int, slots: int, max_batch: int, device, prec: str, rtol: float,
                 max_refine: int, seed: int, lanes: int, ws_batch: int | None = None):
        self.n = n
        self.h = 3.0 / (n + 1)
        self.x0 = -1.5 + self.h
        self.device = device
        self.prec, self.rtol, self.max_refine = prec, rtol, max_refine
        gr = api.grid(n, self.h, 1.0)
        o = api.opts(prec, True, rtol, max_refine)
        wsb = api.workspace_size(gr, ws_batch or max_batch, o)
        self.lanes = [Lane(device, wsb) for _ in range(lanes)]
        self.grow(slots, max_batch, seed)
        self.pending: collections.deque = collections.deque()  # arrived, not yet admitted
        self.ready: collections.deque = collections.deque()    # admitted aux requests

    def grow(self, slots: int, max_batch: int, seed: int):
        """(Re)allocate the ring with `slots` resident right-hand sides (seeded N(0,1))."""
        n = self.n
        self.slots = slots
        self.max_batch = max_batch
        g = torch.Generator(device=self.device)
        g.manual_seed(seed)
        self.b = torch.randn((slots, n, n, n), dtype=torch.float64, device=self.device, generator=g)
        self.u = torch.zeros_like(self.b)
        self.free = collections.deque(range(slots))

    def footprint(self) -> int:
        """Ring and solve workspaces (the step workspaces are charged with the simulations)."""
        return 2 * self.b.numel() * 8 + sum(l.ws.numel() for l in self.lanes)


class Server:
    def __init__(self, sims, device="cuda:0", hbm_budget: float = 64e9, max_batch: int = 8,
                 prec: str = "fp64", rtol: float = 1e-10, max_refine: int = 0, lmax: int = 4,
                 chi: float = 1.0, keep_results: bool = False, lanes: int = 1, seed: int = 0):
        self.device = torch.device(device)
        self.chi = chi
        self.keep = keep_results
        self.budget = float(hbm_budget)
        self.lmax = lmax
        self.rtol = rtol
        self.sims = {s.sid: s for s in sims}
        sizes = sorted({s.n for s in sims})
        # 1. each class's minimum: one slot (b and u) and the lanes' solve workspaces
        per_slot = {n: 2 * 8 * n ** 3 for n in sizes}
        o = api.opts(prec, True, rtol, max_refine)
        lane_ws = {n: lanes * max(1, api.workspace_size(api.grid(n, 3.0 / (n + 1), 1.0),
                                                            max_batch, o)) for n in sizes}
        minimum = sum(per_slot[n] + lane_ws[n] for n in sizes)
        if minimum > self.budget:
            raise ValueError(f"hbm_budget {self.budget:.3g} B is below the servers' minimum "
                             f"{minimum} B (one slot per size class)")
        # 2. resident DPM simulations, in order, while they fit beside the minimum
        self.bep, self.state, self.lane_of, self.sim_bytes = {}, {}, {}, {}
        self.host_state = {}          # evicted simulations: (rho, c) on the host
        self.deferred = set()         # step simulations not resident
        self.inflight_of = collections.Counter()  # step launches in flight per simulation
        self.cost_of = {}             # simulation -> (device bytes, step workspace bytes)
        self.waiting: collections.deque = collections.deque()  # steps of deferred simulations
        self.evictions = 0
        self.classes = {}
        self._resident = 0            # bytes of resident simulations and step workspaces
        step_sims = [s for s in sims if s.kind == "step"]
        # rings are sized after the residents, so build the classes' lanes first (one slot each)
        for i, n in enumerate(sizes):
            self.classes[n] = SizeClass(n, 1, 1, self.device, prec, rtol, max_refine, seed + i,
                                        lanes, ws_batch=max_batch)
        for s in step_sims:
            if not self._try_resident(s.sid, evict=False):
                self.deferred.add(s.sid)
        # 3. slot rings: equal shares of what is left (at least the one slot of the minimum)
        left = self.budget - self.footprint()
        share = left / max(1, len(sizes))
        for i, n in enumerate(sizes):
            extra = int(max(0, min(4 * max_batch - 1, share // per_slot[n])))
            self.classes[n].grow(1 + extra, min(max_batch, 1 + extra), seed + i)
        torch.cuda.synchronize()

    # ------------------------------------------------------------------ memory
    def footprint(self) -> int:
        """Device bytes the server holds: rings, lanes' workspaces, resident simulations."""
        return sum(c.footprint() for c in self.classes.values()) + self._resident

    def _build_sim(self, sid: int):
        s = self.sims[sid]
        c = self.classes[s.n]
        geo = api.geometry("sphere", axes=(1.0,))
        m = api.classify(s.n, c.h, c.x0, geo, device=self.device)
        idx, _ = api.gamma_points(m, c.h, c.x0)
        B, _ = api.basis(s.n, c.h, c.x0, geo, idx, self.lmax, 1)
        bep = api.build_boundary_matrix(m, B, s.n, c.h, s.sigma, c.x0)
        if sid in self.host_state:
            rho, cc = (t.to(self.device) for t in self.host_state.pop(sid))
        else:
            rho = api.gauss_state(bep, geo, 1000.0, 100.0)
            cc = api.gauss_state(bep, geo, 500.0, 50.0)
        return bep, rho, cc

    def _lane(self, sid: int) -> Lane:
        c = self.classes[self.sims[sid].n]
        return c.lanes[sid % len(c.lanes)]

    def _try_resident(self, sid: int, evict: bool) -> bool:
        """Make simulation sid resident if its bytes fit the budget (evicting idle residents
        first when `evict`); False when it does not fit.  A simulation's bytes (handle, state,
        step workspace) are measured on its first build and remembered, so a deferred simulation
        is not rebuilt to find out that it still does not fit."""
        s = self.sims[sid]
        lane = self._lane(sid)
        built = None
        if sid not in self.cost_of:
            built = self._build_sim(sid)
            need = api.step_workspace_size(built[0], api.opts("fp64", True, self.rtol, 0))
            self.cost_of[sid] = (built[0].device_bytes() + 2 * 8 * s.n ** 3, need)
        cost, need = self.cost_of[sid]
        have = lane.step_ws.numel() if lane.step_ws is not None else 0
        ws_extra = max(0, need - have)
        while self.footprint() + cost + ws_extra > self.budget:
            victim = self._idle_resident(exclude=sid) if evict else None
            if victim is None:
                if built is not None:  # measured but does not fit: state to the host
                    bep, rho, cc = built
                    self.host_state[sid] = (rho.cpu(), cc.cpu())
                    bep.close()
                return False
            self._evict(victim)
        bep, rho, cc = built if built is not None else self._build_sim(sid)
        if ws_extra > 0:
            lane.stream.synchronize()  # steps in flight still use the old workspace
            lane.step_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._resident += ws_extra
        self.bep[sid], self.state[sid], self.lane_of[sid] = bep, (rho, cc), lane
        self.sim_bytes[sid] = cost
        self._resident += cost
        self.deferred.discard(sid)
        return True

    def _idle_resident(self, exclude: int):
        for sid in self.bep:
            if sid == exclude or self.inflight_of[sid] > 0:
                continue
            if any(r.sim == sid for r in self.lane_of[sid].steps):
                continue
            return sid
        return None

    def _evict(self, sid: int):
        lane = self.lane_of[sid]
        lane.stream.synchronize()
        self.evictions += 1
        rho, cc = self.state.pop(sid)
        self.host_state[sid] = (rho.cpu(), cc.cpu())
        self.bep.pop(sid).close()
        self.lane_of.pop(sid)
        self._resident -= self.sim_bytes.pop(sid)
        self.deferred.add(sid)

    # ------------------------------------------------------------------ launches
    def _launch_aux(self, c: SizeClass, lane: Lane, reqs, inflight):
        first = reqs[0].slot
        k = len(reqs)
        sig = [r.sigma for r in reqs]
        api.aux_solve_batched_sigma(c.b[first:first + k], sig, c.h, prec=c.prec, rtol=c.rtol,
                                    max_refine=c.max_refine, out=c.u[first:first + k],
                                    workspace=lane.ws, stream=lane.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(lane.stream)
        for i, r in enumerate(reqs):
            r.batch = k
            if self.keep:
                with torch.cuda.stream(lane.stream):
                    r.out = c.u[first + i].clone()
        inflight.append((ev, reqs, c, lane))

    def _launch_step(self, c: SizeClass, lane: Lane, r: Request, inflight):
        bep = self.bep[r.sim]
        rho, cc = self.state[r.sim]
        api.dpm_step(bep, 1.0 / bep.sigma, self.chi, rho, cc, rho, cc, workspace=lane.step_ws,
                     stream=lane.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(lane.stream)
        r.batch = 1
        self.inflight_of[r.sim] += 1
        if self.keep:
            with torch.cuda.stream(lane.stream):
                r.out = (rho.clone(), cc.clone())
        inflight.append((ev, [r], c, lane))

    # ------------------------------------------------------------------ the loop
    def run(self, requests, max_inflight_per_lane: int = 2):
        """Serve `requests` (arrival times relative to the start); returns the requests with
        their completion times filled in."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        arriving = collections.deque(reqs)
        inflight = []
        done = 0
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record()
        e0.synchronize()
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while arriving and arriving[0].arrival <= now:
                r = arriving.popleft()
                self.classes[r.n].pending.append(r)
            # steps of deferred simulations, in arrival order per simulation: a simulation
            # becomes resident once it fits, evicting idle residents if needed
            if self.waiting:
                blocked, keep = set(), collections.deque()
                for r in self.waiting:
                    if r.sim not in blocked and (r.sim in self.bep
                                                 or self._try_resident(r.sim, evict=True)):
                        self.lane_of[r.sim].steps.append(r)
                    else:
                        blocked.add(r.sim)
                        keep.append(r)
                self.waiting = keep
            for c in self.classes.values():
                # admission, first come first served within the class
                while c.pending:
                    r = c.pending[0]
                    if r.kind == "aux":
                        if not c.free:
                            break
                        r.slot = c.free.popleft()
                        c.ready.append(r)
                    elif r.sim in self.bep:
                        self.lane_of[r.sim].steps.append(r)
                    else:
                        self.waiting.append(r)  # deferred simulation: admitted when it fits
                    c.pending.popleft()
                # launches: each lane takes the older of its next step and the class's next
                # aux batch (consecutive slots, up to max_batch)
                for lane in c.lanes:
                    while lane.inflight < max_inflight_per_lane and (c.ready or lane.steps):
                        take_step = bool(lane.steps) and (
                            not c.ready or lane.steps[0].arrival <= c.ready[0].arrival)
                        if take_step:
                            self._launch_step(c, lane, lane.steps.popleft(), inflight)
                        else:
                            batch = [c.ready.popleft()]
                            while (c.ready and len(batch) < c.max_batch
                                   and c.ready[0].slot == batch[-1].slot + 1):
                                batch.append(c.ready.popleft())
                            self._launch_aux(c, lane, batch, inflight)
                        lane.inflight += 1
            # completions
            still = []
            for ev, rs, c, lane in inflight:
                if ev.query():
                    t = e0.elapsed_time(ev) * 1e-3
                    for r in rs:
                        r.t_done = t
                        if r.kind == "aux":
                            c.free.append(r.slot)
                        else:
                            self.inflight_of[r.sim] -= 1
                    done += len(rs)
                    lane.inflight -= 1
                else:
                    still.append((ev, rs, c, lane))
            inflight = still
            if not inflight and arriving and arriving[0].arrival > now:
                time.sleep(min(1e-4, arriving[0].arrival - now))
        torch.cuda.synchronize()
        return reqs


def build_requests(sim_n, sim_sigma, sim_is_step, req_sim, req_sigma, req_arrival):
    """Simulations and requests from plain arrays: per simulation its grid size, sigma and
    whether it advances DPM steps; per request its simulation, sigma and arrival time (s).
    A step request takes its simulation's sigma."""
    sims = [Simulation(i, int(sim_n[i]), float(sim_sigma[i]), "step" if sim_is_step[i] else "aux")
            for i in range(len(sim_n))]
    reqs = []
    for k in range(len(req_sim)):
        s = sims[int(req_sim[k])]
        sg = s.sigma if s.kind == "step" else float(req_sigma[k])
        reqs.append(Request(k, s.sid, s.kind, s.n, sg, float(req_arrival[k])))
    return sims, reqs


def summarize(reqs, makespan: float | None = None):
    lat = np.array([r.latency for r in reqs]) * 1e3
    t_end = max(r.t_done for r in reqs)
    t_beg = min(r.arrival for r in reqs)
    span = makespan if makespan is not None else t_end - t_beg
    solves = sum(1 if r.kind == "aux" else 4 for r in reqs)
    per_n = {}
    for n in sorted({r.n for r in reqs}):
        l = np.array([r.latency for r in reqs if r.n == n]) * 1e3
        per_n[str(n)] = {"count": int(l.size), "p50_ms": float(np.percentile(l, 50)),
                         "p99_ms": float(np.percentile(l, 99))}
    return {"requests": len(reqs), "requests_per_s": len(reqs) / span,
            "solves_per_s": solves / span, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_batch": float(np.mean([r.batch for r in reqs])),
            "per_n": per_n}
