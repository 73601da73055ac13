"""Scheduling logic of the continuous-batching servers on the CPU, with the
device library replaced by stand-ins (no GPU): admission order, the memory
budget, slot limits, overlap of requests and retirement."""
import time

import numpy as np

from paper_2601_08552_amd import serve


class _Walker:
    live = 0

    def __init__(self, ctx, lat, par):
        _Walker.live += 1
        self.done = 0

    def measure(self):
        return np.zeros(2)

    def stats(self):
        return {}

    def tracked_weight(self):
        return (0.0, 1)

    def state(self):
        return (None, None, None, self.done)

    def close(self):
        _Walker.live -= 1


class _Ctx:
    def synchronize(self):
        pass


def _sweep_batch(ws, n, measure=False):
    for w in ws:
        w.done += n


def test_admission_budget_slots_and_overlap(monkeypatch):
    monkeypatch.setattr(serve.lecqmc, "Walker", _Walker)
    monkeypatch.setattr(serve.lecqmc, "sweep_batch", _sweep_batch)
    monkeypatch.setattr(serve.lecqmc, "footprint_bytes", lambda lat, par: 1000 + lat.n_sites)
    reqs = serve.poisson_stream(12, rate=100.0, seed=5, lattices=(4, 6, 8), ne_range=(1, 4),
                                beta_range=(0.5, 1.0), sweeps_range=(2, 6))
    budget = int(2.5 * 1064)
    srv = serve.Server(_Ctx(), budget_bytes=budget, max_active=3)
    peak = {"mem": 0, "act": 0}
    step = srv.step

    def watched(now):
        n = step(now)
        peak["mem"] = max(peak["mem"], srv.in_use)
        peak["act"] = max(peak["act"], len(srv.active))
        return n

    srv.step = watched
    rep = srv.run(reqs, clock=lambda: 0.01 * len(srv.step_ms))
    assert rep["requests"] == len(reqs) and _Walker.live == 0 and srv.in_use == 0
    # every request got exactly its sweeps; nothing ran before it arrived
    for r in reqs:
        got = srv.results[r.rid]
        assert got.state[3] == r.sweeps
        assert got.admitted >= r.arrival
    # the budget and the slot limit held, and requests overlapped
    assert peak["mem"] <= budget and peak["act"] <= 3
    assert len(srv.step_ms) < sum(r.sweeps for r in reqs)
    # first come, first served
    adm = sorted(srv.results.values(), key=lambda x: x.rid)
    assert all(a.admitted <= b.admitted for a, b in zip(adm, adm[1:]))


class _LaneCtx:
    """A context whose step takes a set wall time (a stand-in for the GPU)."""

    def __init__(self, step_s):
        self.step_s = step_s
        self.launches = 0

    def synchronize(self):
        time.sleep(self.step_s)


class _LaneWalker(_Walker):
    def __init__(self, ctx, lat, par):
        super().__init__(ctx, lat, par)
        self.ctx = ctx


def _lane_sweep(ws, n, measure=False):
    ctx = ws[0].ctx
    assert all(w.ctx is ctx for w in ws)       # one lane per launch
    ctx.launches += 1
    for w in ws:
        w.done += n


def _lane_stream(seed, lattices, n):
    return serve.poisson_stream(n, rate=2000.0, seed=seed, lattices=lattices, ne_range=(1, 4),
                                beta_range=(0.5, 1.0), sweeps_range=(2, 5))


def test_lanes_route_by_cost_and_step_independently(monkeypatch):
    monkeypatch.setattr(serve.lecqmc, "Walker", _LaneWalker)
    monkeypatch.setattr(serve.lecqmc, "sweep_batch", _lane_sweep)
    monkeypatch.setattr(serve.lecqmc, "footprint_bytes", lambda lat, par: 1000 + lat.n_sites)
    _Walker.live = 0
    reqs = _lane_stream(9, (4, 6, 48), 16)
    # two cost lanes: a step of the expensive lane lasts 0.2 s, of the cheap one 2 ms
    ctxs = [_LaneCtx(0.002), _LaneCtx(0.2)]
    srv = serve.LaneServer(ctxs, budget_bytes=10**9, edges=(1e-3,))
    lanes = {r.rid: srv.lane_of(r) for r in reqs}
    assert set(lanes.values()) == {0, 1}
    rep = srv.run(reqs)
    assert rep["requests"] == len(reqs) and _Walker.live == 0 and srv.in_use == 0
    for r in reqs:
        assert srv.results[r.rid].state[3] == r.sweeps
        assert srv.results[r.rid].admitted >= r.arrival
    # a cheap request never waited for a step of the expensive lane
    for r in reqs:
        if lanes[r.rid] == 0:
            assert srv.results[r.rid].latency < 0.2, (r.rid, srv.results[r.rid].latency)
    assert rep["lanes"][0]["requests"] + rep["lanes"][1]["requests"] == len(reqs)


def test_lanes_keep_the_budget(monkeypatch):
    monkeypatch.setattr(serve.lecqmc, "Walker", _LaneWalker)
    monkeypatch.setattr(serve.lecqmc, "sweep_batch", _lane_sweep)
    monkeypatch.setattr(serve.lecqmc, "footprint_bytes", lambda lat, par: 1000 + lat.n_sites)
    _Walker.live = 0
    reqs = _lane_stream(4, (4, 6, 40), 12)
    budget = 3 * 2600
    srv = serve.LaneServer([_LaneCtx(0.001), _LaneCtx(0.004)], budget_bytes=budget, edges=(1e-3,))
    peak = {"mem": 0}
    admit = srv._admit

    def watched(ln, now):
        admit(ln, now)
        with srv.lock:
            peak["mem"] = max(peak["mem"], srv.in_use)

    srv._admit = watched
    rep = srv.run(reqs)
    assert rep["requests"] == len(reqs) and _Walker.live == 0
    assert 0 < peak["mem"] <= budget


def test_lane_leaving_frees_its_retired_walkers(monkeypatch):
    """A lane whose requests are all done must free its retired walkers when
    its thread leaves: here the cheap request's walker (1000 of a 1500
    budget) would otherwise block the expensive request of the other lane
    for good."""
    import threading
    from paper_2601_08552_amd import workloads as W
    monkeypatch.setattr(serve.lecqmc, "Walker", _LaneWalker)
    monkeypatch.setattr(serve.lecqmc, "sweep_batch", _lane_sweep)
    monkeypatch.setattr(serve.lecqmc, "footprint_bytes", lambda lat, par: 1000)
    _Walker.live = 0
    par = W.Params(U=2.0, beta=0.5, dtau=0.05, n_stab=10, n_up=1, n_dn=1, seed=1)
    cheap = serve.Request(0, W.square_lattice(4), par, 2, 0.0)
    dear = serve.Request(1, W.square_lattice(48), par, 2, 0.2)
    srv = serve.LaneServer([_LaneCtx(0.001), _LaneCtx(0.002)], budget_bytes=1500, edges=(1e-3,))
    assert srv.lane_of(cheap) == 0 and srv.lane_of(dear) == 1
    out = {}
    th = threading.Thread(target=lambda: out.setdefault("rep", srv.run([cheap, dear])), daemon=True)
    th.start()
    th.join(timeout=20.0)
    assert not th.is_alive(), f"server hung: in_use={srv.in_use}, graveyards={[len(l['graveyard']) for l in srv.lanes]}"
    assert out["rep"]["requests"] == 2 and srv.in_use == 0 and _Walker.live == 0


def test_lanes_stop_at_the_deadline(monkeypatch):
    """A serving window: requests still running or queued when the deadline
    passes are cut off, their walkers freed, and the report counts what was
    admitted and done."""
    monkeypatch.setattr(serve.lecqmc, "Walker", _LaneWalker)
    monkeypatch.setattr(serve.lecqmc, "sweep_batch", _lane_sweep)
    monkeypatch.setattr(serve.lecqmc, "footprint_bytes", lambda lat, par: 1000 + lat.n_sites)
    _Walker.live = 0
    reqs = serve.poisson_stream(40, rate=200.0, seed=3, lattices=(4, 6, 48), ne_range=(1, 4),
                                beta_range=(0.5, 1.0), sweeps_range=(200, 400))
    srv = serve.LaneServer([_LaneCtx(0.002), _LaneCtx(0.01)], budget_bytes=10**9, edges=(1e-3,))
    t0 = time.perf_counter()
    rep = srv.run(reqs, deadline=0.5)
    assert time.perf_counter() - t0 < 5.0
    assert _Walker.live == 0 and srv.in_use == 0
    assert 0 < rep["admitted"] <= len(reqs) and rep["requests"] < len(reqs)
    assert rep["sweeps_done"] > 0 and rep["request_sweep_latency_ms"] is not None
