"""Continuous-batching service over the C ABI.

Independent simulation requests (lattice, particle numbers, U, beta, sweep
count, seed) arrive over time.  The server keeps every admitted request as a
walker resident in device memory and advances all of them together, one
batched sweep per step.  A request is admitted as soon as it has arrived,
a slot is free and its device footprint (``lecqmc_footprint_bytes``) fits the
remaining budget.  Requests that arrive while others run therefore join the
next step, and retired walkers release their memory and slot at once.

Every walker's Markov chain depends only on its own seed, so a request's
result is the same whether it runs alone or in a mix: the integer state
(fields, occupations, counters) is identical and weights and estimators agree
to the FP64 parity bar.  They agree bit for bit when the mix does not change
the walker's register tile or LDS residency.

Reported per run: batched-step latency percentiles (the sweep latency every
resident walker sees), per-request latency percentiles (arrival to
completion) and aggregate HS-field updates per second.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np

from . import lecqmc


@dataclasses.dataclass
class Request:
    rid: int
    lattice: object          # workloads.Lattice
    params: object           # workloads.Params
    sweeps: int
    arrival: float = 0.0     # seconds after the start of the run
    measure: bool = True


@dataclasses.dataclass
class Result:
    rid: int
    measure: np.ndarray
    stats: dict
    tracked_weight: tuple
    state: tuple
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """Admission by footprint, resident walkers, one batched sweep per step."""

    def __init__(self, ctx: "lecqmc.Context", budget_bytes: int, max_active: int = 256):
        self.ctx = ctx
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.pending: deque = deque()
        self.active: list = []          # [request, walker, sweeps done, admitted time]
        self.results: dict = {}
        self.step_ms: list = []
        self.updates = 0
        self.in_use = 0

    def submit(self, req: Request) -> None:
        self.pending.append(req)

    def _admit(self, now: float) -> None:
        while self.pending and self.pending[0].arrival <= now and len(self.active) < self.max_active:
            req = self.pending[0]
            need = lecqmc.footprint_bytes(req.lattice, req.params)
            if need == 0:
                raise ValueError(f"request {req.rid}: invalid lattice or parameters")
            if need > self.budget:
                raise ValueError(f"request {req.rid}: footprint {need} exceeds the whole budget")
            if self.in_use + need > self.budget:
                break                     # first-come first-served: wait for memory
            self.pending.popleft()
            w = lecqmc.Walker(self.ctx, req.lattice, req.params)
            self.in_use += need
            self.active.append([req, w, 0, now, need])

    def _retire(self, now: float) -> None:
        keep = []
        for entry in self.active:
            req, w, done, admitted, need = entry
            if done >= req.sweeps:
                self.results[req.rid] = Result(req.rid, w.measure(), w.stats(), w.tracked_weight(), w.state(),
                                               req.arrival, admitted, now)
                w.close()
                self.in_use -= need
            else:
                keep.append(entry)
        self.active = keep

    def step(self, now: float) -> int:
        """Admit what has arrived, run one batched sweep, retire finished
        requests.  Returns the number of HS-field updates performed."""
        self._admit(now)
        if not self.active:
            return 0
        walkers = [e[1] for e in self.active]
        t0 = time.perf_counter()
        lecqmc.sweep_batch(walkers, 1, measure=any(e[0].measure for e in self.active))
        self.ctx.synchronize()
        self.step_ms.append((time.perf_counter() - t0) * 1e3)
        n = 0
        for e in self.active:
            e[2] += 1
            n += e[0].lattice.n_sites * e[0].params.L_tau
        self.updates += n
        return n

    def run(self, requests, clock=None) -> dict:
        """Serve a list of requests until all have finished.  ``clock`` gives
        the current time in seconds since the start (wall clock by default);
        a request is eligible once ``clock() >= arrival``."""
        for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
            self.submit(r)
        start = time.perf_counter()
        simulated = clock is not None
        clock = clock or (lambda: time.perf_counter() - start)
        while self.pending or self.active:
            now = clock()
            if not self.active and self.pending and self.pending[0].arrival > now:
                if not simulated:
                    time.sleep(min(0.01, self.pending[0].arrival - now))
                    continue
                now = self.pending[0].arrival   # idle under a simulated clock: jump to the next arrival
            self.step(now)
            self._retire(max(now, clock()))
        wall = time.perf_counter() - start
        lat = [r.latency for r in self.results.values()]
        return {
            "requests": len(self.results),
            "wall_s": wall,
            "updates_per_s": self.updates / wall if wall > 0 else 0.0,
            "step_ms": {"p50": float(np.percentile(self.step_ms, 50)), "p99": float(np.percentile(self.step_ms, 99))}
            if self.step_ms else None,
            "request_latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}
            if lat else None,
        }


def poisson_stream(n, rate, seed=0, lattices=(8, 12, 16, 24), ne_range=(2, 16), U_range=(2.0, 8.0),
                   beta_range=(2.0, 4.0), sweeps_range=(5, 20), dtau=0.05, n_stab=10):
    """A seeded stream of requests with exponential gaps (the serving
    workload's structure, at sizes that finish in seconds)."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += float(rng.exponential(1.0 / rate))
        Ls = int(rng.choice(lattices))
        lat = W.square_lattice(Ls)
        ne = int(rng.integers(ne_range[0], ne_range[1] + 1))
        ne = min(ne, lat.n_sites)
        blocks = max(1, int(round(float(rng.uniform(*beta_range)) / (dtau * n_stab))))
        par = W.Params(U=float(np.round(rng.uniform(*U_range), 3)), beta=round(blocks * dtau * n_stab, 9), dtau=dtau,
                       n_stab=n_stab, n_up=ne, n_dn=ne, seed=1000 + rid, walker_id=rid)
        out.append(Request(rid, lat, par, int(rng.integers(sweeps_range[0], sweeps_range[1] + 1)), t))
    return out


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Serve a seeded Poisson stream of simulation requests.")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--rate", type=float, default=50.0, help="arrivals per second")
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    ctx = lecqmc.Context(0)
    srv = Server(ctx, int(args.budget_gb * 2**30))
    rep = srv.run(poisson_stream(args.requests, args.rate, args.seed))
    rep.update({"rate_per_s": args.rate, "budget_gb": args.budget_gb})
    print(json.dumps(rep))
    ctx.close()


if __name__ == "__main__":
    main()
