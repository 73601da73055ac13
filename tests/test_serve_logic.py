"""Scheduling logic of the continuous-batching server on the CPU, with the
device library replaced by stand-ins (no GPU): admission order, the memory
budget, slot limits, overlap of requests and retirement."""
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
