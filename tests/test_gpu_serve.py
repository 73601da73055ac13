"""Continuous batching: requests that arrive while others run are admitted as
slots and memory free up, and each result equals the same request run alone
(integer state exactly; weights and estimators to the FP64 parity bar)."""
import numpy as np
import pytest

from paper_2601_08552_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    from paper_2601_08552_amd import lecqmc
    lecqmc.load()
    return lecqmc


def _stream():
    from paper_2601_08552_amd.serve import poisson_stream
    return poisson_stream(10, rate=100.0, seed=3, lattices=(4, 6, 8), ne_range=(1, 6), U_range=(2.0, 6.0),
                          beta_range=(0.5, 1.5), sweeps_range=(2, 6))


def test_results_same_alone_and_in_the_mix(lq):
    from paper_2601_08552_amd.serve import Server
    reqs = _stream()
    big = max(lq.footprint_bytes(r.lattice, r.params) for r in reqs)
    ctx = lq.Context(0)
    srv = Server(ctx, budget_bytes=int(2.5 * big), max_active=4)
    # simulated clock: 10 ms per batched step, so admissions are reproducible
    rep = srv.run(reqs, clock=lambda: 0.01 * len(srv.step_ms))
    assert rep["requests"] == len(reqs)
    # requests did overlap on the device, and some had to wait for memory or a slot
    waited = [r for r in srv.results.values() if r.admitted > r.arrival + 1e-12]
    assert waited and max(len(srv.step_ms), 1) < sum(r.sweeps for r in reqs)
    for r in reqs:
        got = srv.results[r.rid]
        w = lq.Walker(ctx, r.lattice, r.params)
        w.sweep(r.sweeps, measure=True)
        for x, y in zip(got.state, w.state()):
            assert np.array_equal(np.asarray(x), np.asarray(y)), r.rid
        lg, sg = got.tracked_weight
        la, sa = w.tracked_weight()
        assert sg == sa and abs(lg - la) <= 1e-10 * max(1.0, abs(la))
        ma = w.measure()
        assert np.max(np.abs(got.measure - ma)) <= 1e-9 * max(1.0, np.max(np.abs(ma)))
        w.close()
    assert srv.in_use == 0 and ctx.bytes_in_use() == 0
    ctx.close()


def test_lanes_results_same_alone_and_in_the_mix(lq):
    """Two cost lanes (two contexts, two streams) stepping independently:
    every result still equals the request run alone."""
    from paper_2601_08552_amd.serve import LaneServer, sweep_cost
    reqs = _stream()
    costs = sorted(sweep_cost(r.lattice, r.params) for r in reqs)
    edge = costs[len(costs) // 2]
    ctxs = [lq.Context(0), lq.Context(0)]
    srv = LaneServer(ctxs, budget_bytes=1 << 34, edges=(edge,))
    assert {srv.lane_of(r) for r in reqs} == {0, 1}
    rep = srv.run(reqs)
    assert rep["requests"] == len(reqs)
    alone_ctx = lq.Context(0)
    for r in reqs:
        got = srv.results[r.rid]
        w = lq.Walker(alone_ctx, r.lattice, r.params)
        w.sweep(r.sweeps, measure=True)
        for x, y in zip(got.state, w.state()):
            assert np.array_equal(np.asarray(x), np.asarray(y)), r.rid
        lg, sg = got.tracked_weight
        la, sa = w.tracked_weight()
        assert sg == sa and abs(lg - la) <= 1e-10 * max(1.0, abs(la))
        ma = w.measure()
        assert np.max(np.abs(got.measure - ma)) <= 1e-9 * max(1.0, np.max(np.abs(ma)))
        w.close()
    assert srv.in_use == 0 and all(c.bytes_in_use() == 0 for c in ctxs)
    for c in ctxs + [alone_ctx]:
        c.close()
