"""Continuous-batching service over the C ABI.

Independent simulation requests (lattice, particle numbers, U, beta, sweep
count, seed) arrive over time.  A server keeps every admitted request as a
walker resident in device memory and advances the resident walkers in
batched sweeps.  A request is admitted as soon as it has arrived, a slot is
free and its device footprint (``lecqmc_footprint_bytes``) fits the
remaining budget, so requests that arrive while others run join the next
step.  ``Server`` runs one batch (one sweep of every resident walker per
step; retired walkers release their memory at once).  ``LaneServer`` runs
one batch per cost lane, each on its own context, stream and host thread,
so that small requests are not held up by steps of much larger ones.

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
        self.on_finish = None           # optional callback(Result) when a request retires

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
                if self.on_finish:
                    self.on_finish(self.results[req.rid])
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


# Forward-pass cost per site of one walker on MI355X (seconds), by Ne per
# spin, from the chain-shape measurements; used only to route requests.
_SITE_COST = ((8, 2.7e-7), (16, 5.0e-7), (32, 1.3e-6), (64, 1.2e-5), (128, 2.8e-5), (256, 1.0e-4))


def sweep_cost(lattice, params) -> float:
    """Rough seconds per sweep of one request: sites x slices x per-site cost."""
    ne = max(params.n_up, params.n_dn, 1)
    c = _SITE_COST[-1][1]
    for n, v in _SITE_COST:
        if ne <= n:
            c = v
            break
    return lattice.n_sites * params.L_tau * c


class LaneServer:
    """Continuous batching over lanes.  Each lane is a context with its own
    stream, its own resident batch and its own host thread; a request joins
    the lane of its per-sweep cost (``edges`` in seconds), so a lane's
    batched step is not held up by requests a thousand times larger, and the
    lanes' kernels overlap on the device.  A lane thread admits its requests
    first come, first served within the shared memory budget, sweeps its
    batch once, waits for it on its own stream (the library call releases
    the interpreter lock) and retires finished requests.  Walkers are freed
    lazily, when a waiting request needs the memory: freeing device memory
    can wait for the whole device."""

    def __init__(self, ctxs, budget_bytes: int, max_active: int = 256, edges=(0.05, 0.5, 5.0)):
        import threading
        assert len(ctxs) == len(edges) + 1
        self.edges = tuple(edges)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.lanes = [dict(ctx=c, pending=deque(), active=[], graveyard=[], steps=[], step_active=[]) for c in ctxs]
        self.lock = threading.Lock()
        self.results: dict = {}
        self.admitted: dict = {}        # rid -> (arrival, admission time)
        self.sweeps_done: dict = {}     # rid -> sweeps done (also for requests cut off by a deadline)
        self.updates = 0
        self.in_use = 0
        self.n_active = 0
        self.short = False              # a lane waits for memory: the others free their retired walkers
        self.on_finish = None

    def lane_of(self, req) -> int:
        c = sweep_cost(req.lattice, req.params)
        k = 0
        while k < len(self.edges) and c >= self.edges[k]:
            k += 1
        return k

    def _free(self, ln):
        for w, need in ln["graveyard"]:
            w.close()
            with self.lock:
                self.in_use -= need
        ln["graveyard"] = []

    def _admit(self, ln, now):
        while ln["pending"] and ln["pending"][0].arrival <= now:
            req = ln["pending"][0]
            need = lecqmc.footprint_bytes(req.lattice, req.params)
            if need == 0:
                raise ValueError(f"request {req.rid}: invalid lattice or parameters")
            if need > self.budget:
                raise ValueError(f"request {req.rid}: footprint {need} exceeds the whole budget")
            with self.lock:
                ok = self.in_use + need <= self.budget and self.n_active < self.max_active
                if ok:
                    self.in_use += need
                    self.n_active += 1
                elif self.in_use + need > self.budget:
                    self.short = True
            if not ok:
                if ln["graveyard"]:
                    self._free(ln)
                    continue
                break
            ln["pending"].popleft()
            w = lecqmc.Walker(ln["ctx"], req.lattice, req.params)
            ln["active"].append([req, w, 0, now, need])
            with self.lock:
                self.admitted[req.rid] = (req.arrival, now)

    def _retire(self, ln, now):
        keep = []
        for entry in ln["active"]:
            req, w, done, admitted, need = entry
            if done >= req.sweeps:
                res = Result(req.rid, w.measure(), w.stats(), w.tracked_weight(), w.state(), req.arrival, admitted, now)
                ln["graveyard"].append([w, need])
                with self.lock:
                    self.results[req.rid] = res
                    self.n_active -= 1
                if self.on_finish:
                    self.on_finish(res)
            else:
                keep.append(entry)
        ln["active"] = keep

    def _lane(self, ln, clock, errors, deadline=None):
        try:
            while ln["pending"] or ln["active"]:
                if deadline is not None and clock() >= deadline:
                    # the window is over: requests still running are cut off
                    for req, w, done, _, need in ln["active"]:
                        ln["graveyard"].append([w, need])
                        with self.lock:
                            self.sweeps_done[req.rid] = done
                            self.n_active -= 1
                    ln["active"] = []
                    ln["pending"].clear()
                    break
                if self.short and ln["graveyard"]:
                    self._free(ln)
                    self.short = False
                now = clock()
                self._admit(ln, now)
                if not ln["active"]:
                    nxt = ln["pending"][0].arrival if ln["pending"] else now
                    time.sleep(min(0.005, max(nxt - now, 2e-4)))
                    continue
                t0 = time.perf_counter()
                lecqmc.sweep_batch([e[1] for e in ln["active"]], 1, measure=any(e[0].measure for e in ln["active"]))
                ln["ctx"].synchronize()
                ln["steps"].append((time.perf_counter() - t0) * 1e3)
                ln["step_active"].append(len(ln["active"]))
                n = 0
                for e in ln["active"]:
                    e[2] += 1
                    n += e[0].lattice.n_sites * e[0].params.L_tau
                    with self.lock:
                        self.sweeps_done[e[0].rid] = e[2]
                with self.lock:
                    self.updates += n
                self._retire(ln, clock())
            # retired walkers still count against the shared budget, and only
            # this thread may free them (they belong to this lane's context):
            # free them before leaving, or a lane still waiting for memory
            # would wait forever
            self._free(ln)
        except BaseException as exc:    # reported by run() on the caller's thread
            errors.append(exc)

    def run(self, requests, clock=None, deadline=None) -> dict:
        """Serve until every request has finished, or until ``deadline``
        seconds (requests still queued or running then are cut off);
        ``clock`` gives seconds since the start (wall clock by default)."""
        import threading
        lane_of = {}
        for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
            lane_of[r.rid] = self.lane_of(r)
            self.lanes[lane_of[r.rid]]["pending"].append(r)
        start = time.perf_counter()
        clock = clock or (lambda: time.perf_counter() - start)
        errors = []
        threads = [threading.Thread(target=self._lane, args=(ln, clock, errors, deadline), daemon=True)
                   for ln in self.lanes]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        for ln in self.lanes:
            self._free(ln)
        if errors:
            raise errors[0]
        wall = time.perf_counter() - start
        lat = [r.latency for r in self.results.values()]
        steps = [x for ln in self.lanes for x in ln["steps"]]
        # sweep latency as the requests see it: every request resident in a
        # step waits for that whole step
        req_sweeps = [x for ln in self.lanes for x, k in zip(ln["steps"], ln["step_active"]) for _ in range(k)]
        pct = lambda v: {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99))} if v else None
        return {
            "requests": len(self.results),
            "wall_s": wall,
            "updates_per_s": self.updates / wall if wall > 0 else 0.0,
            "lanes": [{"requests": sum(1 for rid in self.results if lane_of[rid] == k), "steps": len(ln["steps"]),
                       "step_ms": pct(ln["steps"]),
                       "request_latency_s": pct([self.results[rid].latency for rid in self.results
                                                 if lane_of[rid] == k])}
                      for k, ln in enumerate(self.lanes)],
            "step_ms": pct(steps),
            "request_sweep_latency_ms": pct(req_sweeps),
            "request_latency_s": pct(lat),
            "admitted": len(self.admitted),
            "queue_wait_s": pct([a - r for r, a in self.admitted.values()]),
            "sweeps_done": int(sum(self.sweeps_done.values())),
        }


_SQUARE = {}


def serving_stream(window, rate=50.0, seed=0, dtau=0.05, n_stab=10, measure=False):
    """The serving workload's requests that arrive within ``window`` seconds:
    Poisson arrivals at ``rate`` per second (seeded exponential gaps), L x L
    periodic square lattices with L uniform over the even numbers 16..128
    (N up to 16384), N_up = N_dn uniform in 4..64, U uniform in [2, 8], beta
    uniform in [4, 32] rounded to a whole number of stabilisation blocks
    (dtau = 0.05, a QR every 10 slices), 100..1000 sweeps, seed = request
    id."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > window:
            return out
        Ls = int(rng.choice(np.arange(16, 129, 2)))
        ne = int(rng.integers(4, 65))
        U = round(float(rng.uniform(2.0, 8.0)), 3)
        blocks = max(1, int(round(float(rng.uniform(4.0, 32.0)) / (dtau * n_stab))))
        rid = len(out)
        par = W.Params(U=U, beta=round(blocks * dtau * n_stab, 9), dtau=dtau, n_stab=n_stab, n_up=ne, n_dn=ne,
                       seed=1000 + rid, walker_id=rid)
        if Ls not in _SQUARE:
            _SQUARE[Ls] = W.square_lattice(Ls)
        out.append(Request(rid, _SQUARE[Ls], par, int(rng.integers(100, 1001)), t, measure=measure))


def serving_window(window, rate=50.0, seed=0, budget_bytes=200 * 2**30, lanes=5, log=None) -> dict:
    """Serve the serving workload's stream for ``window`` seconds on lane
    servers (one context per lane) and report what the window achieved:
    offered, admitted and finished requests, aggregate HS-field updates per
    second, the sweep latency the resident requests saw (p50/p99), the wait
    from arrival to admission, and the highest arrival rate the measured
    throughput sustains (throughput / mean work of a request, the mean taken
    over 20000 draws of the request distribution)."""
    reqs = serving_stream(window, rate, seed)
    draws = serving_stream(20000.0 / rate, rate, seed + 1)
    mean_work = float(np.mean([r.lattice.n_sites * r.params.L_tau * r.sweeps for r in draws]))
    edges = tuple(0.05 * 10.0 ** k for k in range(lanes - 1))
    ctxs = [lecqmc.Context(0) for _ in range(lanes)]
    srv = LaneServer(ctxs, budget_bytes, edges=edges)
    if log:
        srv.on_finish = lambda r: log(f"serving: request {r.rid} finished, latency {r.latency:.1f} s")
    rep = srv.run(reqs, deadline=window)
    for c in ctxs:
        c.close()
    thr = rep["updates_per_s"]
    return {
        "window_s": window, "offered_rate_per_s": rate, "offered": len(reqs), "admitted": rep["admitted"],
        "finished": rep["requests"], "sweeps_done": rep["sweeps_done"],
        "updates_per_s": thr, "unit": "HS-field updates/s",
        "request_sweep_latency_ms": rep["request_sweep_latency_ms"], "queue_wait_s": rep["queue_wait_s"],
        "request_latency_s": rep["request_latency_s"], "lanes": rep["lanes"], "lane_edges_s": list(edges),
        "budget_gib": budget_bytes / 2**30,
        "mean_request_updates": mean_work,
        "sustainable_rate_per_s": thr / mean_work if mean_work > 0 else 0.0,
        "config": "Poisson arrivals at 50/s; L x L periodic square, L even in 16..128; Ne per spin 4..64; U 2..8; "
                  "beta 4..32 (whole QR blocks, dtau=0.05, QR every 10 slices); 100..1000 sweeps; FP64; "
                  "admitted by device footprint; no estimators; requests still queued or running at the end of "
                  "the window are cut off",
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
    import sys
    ap = argparse.ArgumentParser(description="Serve a seeded Poisson stream of simulation requests.")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--rate", type=float, default=50.0, help="arrivals per second")
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--lattices", type=str, default="8,12,16,24", help="L of the L x L lattices, comma separated")
    ap.add_argument("--ne", type=str, default="2,16", help="range of Ne per spin: lo,hi")
    ap.add_argument("--beta", type=str, default="2,4", help="range of beta: lo,hi")
    ap.add_argument("--sweeps", type=str, default="5,20", help="range of sweeps per request: lo,hi")
    ap.add_argument("--lanes", type=int, default=4, help="cost lanes (1: one batch for all requests)")
    args = ap.parse_args()
    two = lambda t, f: tuple(f(x) for x in t.split(","))
    reqs = poisson_stream(args.requests, args.rate, args.seed, lattices=two(args.lattices, int),
                          ne_range=two(args.ne, int), beta_range=two(args.beta, float),
                          sweeps_range=two(args.sweeps, int))
    if args.lanes > 1:
        edges = (0.05, 0.5, 5.0)[: args.lanes - 1] if args.lanes <= 4 else tuple(0.05 * 10 ** (k / 2) for k in range(args.lanes - 1))
        ctxs = [lecqmc.Context(0) for _ in range(len(edges) + 1)]
        srv = LaneServer(ctxs, int(args.budget_gb * 2**30), edges=edges)
    else:
        ctxs = [lecqmc.Context(0)]
        srv = Server(ctxs[0], int(args.budget_gb * 2**30))
    srv.on_finish = lambda r: print(f"[serve] request {r.rid} done: latency {r.latency:.2f} s", file=sys.stderr,
                                    flush=True)
    rep = srv.run(reqs)
    rep.update({"rate_per_s": args.rate, "budget_gb": args.budget_gb, "lattices": args.lattices, "ne": args.ne,
                "beta": args.beta, "sweeps": args.sweeps})
    rep["server"] = f"{len(ctxs)} lane(s)"
    print(json.dumps(rep))
    for c in ctxs:
        c.close()


if __name__ == "__main__":
    main()
