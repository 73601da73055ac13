"""Throughput of the canonical-ensemble DQMC hot path on one MI355X.

Headline workload (value): the batched uneven walkers, 256 independent
chains, L x L periodic square lattices with L uniform in {16, 24, 32, 48, 64}
(N = 256..4096), Ne per spin uniform in [4, 32], U uniform in [2, 6], beta in
{8, 16}, dtau = 0.05, a QR every 10 slices, FP64, chain shapes autotuned.
The walkers are split by cost into four groups with a stream and a HIP graph
each, and the groups' sweeps run concurrently.  It is the largest
fixed configuration that runs on one GPU.  A step is one full sweep of every
walker: left-stack build, forward pass with N * L_tau Ising-flip attempts and
QR stabilisation, and N_sigma particle-hole swaps per spin.

Also measured, as objects of the same JSON line:
- dilute_gas: the 32x32 dilute Fermi gas (N = 1024, 8 + 8, beta = 16,
  320 slices), 64 walkers, FP64 and mixed precision (FP32 propagation);
- flat_band: the 256-cell flat-band chain (N = 512, 128 + 128, beta = 10),
  128 walkers;
- scaling_fig1: seconds per sweep against N on the paper's Fig. 1 workload
  (square Hubbard, beta = 1, 50 + 50 particles, N = 144..16384) and the
  fitted power of N;
- constrained_path: the constrained-path inner walk (256 random walkers) of
  one Fock state of the dilute gas;
- serving: a Poisson stream of simulation requests (50/s, L x L from 16 to
  128, Ne per spin 4..64, U 2..8, beta 4..32, 100..1000 sweeps each)
  admitted by device footprint over a fixed window;
- accuracy: one walker of each workload swept on the GPU and by the FP64
  oracle from the same state, in this run;
- cpu_baseline: the FP64 oracle on the host cores on a stratified sample of
  the headline workload's walkers.

Prints one JSON line; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "HS-field updates/s per GPU at stated err vs FP64 oracle; p50/p99 sweep latency"


def algorithmic_bytes_forward(N, ne_up, ne_dn, L, nstab):
    """Algorithmic HBM bytes of one walker's forward pass (FP64).

    Per slice each spin streams Phi_R and Phi_L (N x Ne) in and out once
    (diagonal factor, flips and checkerboard applied while resident):
    2 sides * 2 (read + write) * N * Ne * 8.  Per stabilisation block the QR
    reads Phi twice and writes Q twice and the fresh Phi_L is read once:
    5 * N * Ne * 8.  Fields: one read and one write byte per site and slice.
    """
    nblk = (L + nstab - 1) // nstab
    b = 0
    for ne in (ne_up, ne_dn):
        b += L * 4 * N * ne * 8 + nblk * 5 * N * ne * 8
    return b + 2 * L * N


def measured_traffic(kernel_src, pmc_json):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counters (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's
    readings), or None when the kernel source changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(pmc_json))
        sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("src_sha256") != sha:
        return None
    kib = rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] + rec["write_kib_per_dispatch"] * rec["write_scale"]
    return kib * 1024.0


def note(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(v):
    return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99))} if len(v) else None


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, one plain process per host core (no process pool,
# so nothing outlives the benchmark)
# ---------------------------------------------------------------------------
def oracle_child(spec_json):
    """Run one walker of the oracle and print its per-sweep seconds (child process)."""
    import oracle
    from paper_2601_08552_amd import workloads as W
    spec = json.loads(spec_json)
    lat = W.square_lattice(spec["L"])
    par = W.Params(**spec["par"])
    w = oracle.Walker(lat, par)
    times = []
    for _ in range(spec["sweeps"]):
        t0 = time.perf_counter()
        w.sweep(1)
        times.append(time.perf_counter() - t0)
    print(json.dumps({"times": times, "updates": lat.n_sites * par.L_tau}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, procs):
    """The FP64 oracle, unmodified, on `procs` host cores: a stratified sample
    of `procs` walkers of the batched workload (sorted by N * L_tau * Ne^2,
    every 256/procs-th), one sweep each, one process per walker.  The rate is
    scaled to the whole workload: the sampled walkers' seconds per update,
    weighted by the updates of the walkers each one stands for, spread over
    the cores."""
    import oracle
    oracle.build()
    order = sorted(range(len(cfg)), key=lambda c: cfg[c][0].n_sites * cfg[c][1].L_tau * cfg[c][1].n_up ** 2)
    stride = max(1, len(cfg) // procs)
    picks = [order[min(len(order) - 1, k * stride + stride // 2)] for k in range(procs)]
    kids = []
    for c in picks:
        lat, par = cfg[c]
        L = int(round(np.sqrt(lat.n_sites)))
        spec = {"L": L, "sweeps": 1, "par": {k: getattr(par, k) for k in ("U", "beta", "dtau", "n_stab", "n_up",
                                                                          "n_dn", "seed", "walker_id")}}
        kids.append(subprocess.Popen([sys.executable, "-c", "import bench; bench.oracle_child(%r)" % json.dumps(spec)],
                                     cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                                     env={**os.environ, "OMP_NUM_THREADS": "1"}))
    t0 = time.perf_counter()
    res = []
    for k in kids:
        out, _ = k.communicate()
        res.append(json.loads(out.decode().strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    # seconds per update of each sample, standing for its stratum of walkers
    spu = [r["times"][0] / r["updates"] for r in res]
    strata = [order[k * stride:(k + 1) * stride] if k < procs - 1 else order[k * stride:] for k in range(procs)]
    upd_total = sum(cfg[c][0].n_sites * cfg[c][1].L_tau for c in range(len(cfg)))
    est_seconds = sum(spu[k] * sum(cfg[c][0].n_sites * cfg[c][1].L_tau for c in strata[k]) for k in range(procs))
    per_sweep = [r["times"][0] for r in res]
    return {"value": upd_total / (est_seconds / procs), "unit": "HS-field updates/s", "cores": procs,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{procs} of the 256 batched walkers (stratified by N*L_tau*Ne^2), one sweep each, one "
                      f"process per core, {wall:.1f} s wall; rate = the whole batch's updates over its estimated "
                      f"oracle time on {procs} cores (per-update cost of each sample times the updates of its "
                      f"stratum)",
            "sec_per_sweep_sampled": pct(per_sweep),
            "us_per_update_sampled": {"min": 1e6 * min(spu), "max": 1e6 * max(spu)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uneven", action="store_true", help="skip the headline batch (profiling of other legs)")
    ap.add_argument("--groups", type=int, default=4, help="concurrent walker groups of the headline batch (1..4)")
    ap.add_argument("--no-dilute", action="store_true", help="skip the 32x32 dilute-gas objects")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-flat", action="store_true", help="skip the 128-walker flat-band batch")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-cp", action="store_true", help="skip the constrained-path walk")
    ap.add_argument("--no-scaling", action="store_true", help="skip the sweep-time-vs-N fit")
    ap.add_argument("--serve-window", type=float, default=60.0, help="seconds of the serving stream")
    ap.add_argument("--cpu-procs", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2601_08552_amd import lecqmc
    from paper_2601_08552_amd import workloads as W

    torch.cuda.set_device(0)

    # ------------------------------------------------------------------
    # headline: the 256-walker uneven batch
    # ------------------------------------------------------------------
    cfg = W.config_batched(256)
    out = headline(args, cfg) if not args.no_uneven else {"metric": METRIC, "value": None, "note": "--no-uneven"}
    run_legs(args, cfg, out)
    print(json.dumps(out), flush=True)


def headline(args, cfg):
    """The 256-walker batch.  Walkers are sorted by cost (N L_tau Ne^2) and
    split into `groups` contiguous groups, each with its own context, stream,
    fixed batch and HIP graph of one sweep.  A step replays every group's
    graph once; the groups' graphs run concurrently on their streams, so the
    cheap walkers' phases overlap the expensive walkers' instead of waiting at
    each phase for the slowest walker of the whole batch.  Every walker
    advances exactly one sweep per step."""
    import torch
    from paper_2601_08552_amd import lecqmc
    G = max(1, min(4, args.groups))
    cost = lambda c: cfg[c][0].n_sites * cfg[c][1].L_tau * max(cfg[c][1].n_up, cfg[c][1].n_dn) ** 2
    order = sorted(range(len(cfg)), key=lambda c: -cost(c))
    groups = [order[k * len(order) // G:(k + 1) * len(order) // G] for k in range(G)]
    note(f"uneven batch: creating 256 walkers in {G} groups")
    streams = [torch.cuda.Stream() for _ in range(G)]
    ctxs = [lecqmc.Context(0, stream=st) for st in streams]
    ws = [None] * len(cfg)
    for g in range(G):
        for c in groups[g]:
            ws[c] = lecqmc.Walker(ctxs[g], *cfg[c])
    note("uneven batch: autotuning (the groups concurrently, one host thread each)")
    import threading
    t_tune = time.perf_counter()
    res = [None] * G

    def tune(g):
        res[g] = lecqmc.autotune([ws[c] for c in groups[g]])

    th = [threading.Thread(target=tune, args=(g,)) for g in range(G)]
    for t_ in th:
        t_.start()
    for t_ in th:
        t_.join()
    tuned = [r for g in range(G) for r in res[g]]
    t_tune = time.perf_counter() - t_tune
    # each group's phases timed alone by its context's events (on the stream
    # its kernels run on)
    note("uneven batch: phase timing")
    ph = []
    for g in range(G):
        wg = [ws[c] for c in groups[g]]
        lecqmc.sweep_batch(wg, 1)
        ctxs[g].synchronize()
        ctxs[g].set_timing(True)
        ctxs[g].phase_times()
        lecqmc.sweep_batch(wg, 2)
        ms, cn = ctxs[g].phase_times()
        ctxs[g].set_timing(False)
        ph.append([ms[k] / max(cn[k], 1) for k in range(3)])
    batches, graphs = [], []
    for g in range(G):
        b = lecqmc.Batch([ws[c] for c in groups[g]])
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=streams[g]):
            b.sweep(1)
        batches.append(b)
        graphs.append(gr)
    torch.cuda.synchronize()
    note(f"uneven batch: {args.warmup} warm-up + {args.steps} timed steps")
    for _ in range(args.warmup):
        for gr in graphs:
            gr.replay()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)] for _ in range(G)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(G):
        ev[g][0].record(streams[g])
    for q in range(args.steps):
        for g in range(G):
            with torch.cuda.stream(streams[g]):
                graphs[g].replay()
            ev[g][q + 1].record(streams[g])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-walker sweep latency: its group's step times
    lat_ms = []
    for g in range(G):
        for q in range(args.steps):
            lat_ms += [ev[g][q].elapsed_time(ev[g][q + 1])] * len(groups[g])
    upd_sweep = sum(lat.n_sites * par.L_tau for lat, par in cfg)
    value = upd_sweep * args.steps / wall
    alg_g = [sum(algorithmic_bytes_forward(cfg[c][0].n_sites, cfg[c][1].n_up, cfg[c][1].n_dn, cfg[c][1].L_tau,
                                           cfg[c][1].n_stab) for c in groups[g]) for g in range(G)]
    fwd_ms = sum(p[1] for p in ph) / G
    alg = sum(alg_g) / G
    achieved = alg / (fwd_ms * 1e-3) / 1e9
    fwd_w = sorted(r[2] for r in tuned)
    st0 = ws[0].stats()
    hbm_gib = sum(cx.bytes_in_use() for cx in ctxs) / 2**30
    for b in batches:
        b.close()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "HS-field updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched uneven walkers: 256 chains, L x L periodic square, L in {16,24,32,48,64}, "
                               "Ne per spin in [4,32], U in [2,6], beta in {8,16}, dtau=0.05, QR every 10 slices, "
                               "FP64, autotuned chain shapes, sweeps replayed from HIP graphs",
                   "walkers": len(ws), "updates_per_sweep": upd_sweep, "hbm_gib": hbm_gib,
                   "groups": G, "note": "walkers sorted by N*L_tau*Ne^2 into contiguous groups, one stream and one "
                                        "graph per group, the groups' sweeps concurrent"},
        "latency_ms": {**pct(lat_ms), "note": "per-walker sweep latency = its group's step time"},
        "phase_ms_per_launch": {"left_stack": [p[0] for p in ph], "forward": [p[1] for p in ph],
                                "fock": [p[2] for p in ph], "note": "per group, each group alone"},
        "autotune": {"seconds": t_tune,
                     "shapes": {f"{t},{c}": sum(1 for r in tuned if r[:2] == (t, c))
                                for (t, c) in sorted({r[:2] for r in tuned})},
                     "forward_ms_per_walker": {"min": fwd_w[0], "median": fwd_w[len(fwd_w) // 2], "max": fwd_w[-1]}},
        "roofline": {"bound": "hbm", "kernel": "k_forward", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg,
                     "note": "one launch = the forward pass of one group's walkers (average over the groups); it "
                             "lasts as long as the group's slowest walker (the dependent flip chain), not as long "
                             "as its bytes take"},
        "stats_walker0": {k: st0[k] for k in ("logw_drift", "max_wrap_err", "qr_shifted")},
        "near_ties": {"count": sum(w.stats()["near_ties"] for w in ws),
                      "decisions": sum(w.stats()["flip_attempts"] + w.stats()["swap_attempts"] for w in ws),
                      "note": "flip and swap decisions of all walkers so far whose uniform lay within 1e-9 of |r| "
                              "(a rounding change of r that size could reverse them)"},
    }
    traffic = measured_traffic(os.path.join(ROOT, "paper_2601_08552_amd", "csrc", "lecqmc_kernels.hip"),
                               os.path.join(ROOT, "profiles", "k_forward_batched256_pmc.json"))
    out["roofline"]["traffic"] = traffic
    for w in ws:
        w.close()
    for cx in ctxs:
        cx.close()
    return out


def run_legs(args, cfg, out):
    import torch
    from paper_2601_08552_amd import lecqmc
    from paper_2601_08552_amd import workloads as W
    ctx = lecqmc.Context(0, stream=torch.cuda.current_stream())
    stream = torch.cuda.current_stream()

    def run_dilute(precision, nw=64, steps=5, warmup=2):
        """Timed batched sweeps of the 32x32 dilute gas at one precision."""
        note(f"dilute gas, precision {precision}: {nw} walkers")
        walkers = [lecqmc.Walker(ctx, *W.config_dilute(seed=s + 1, walker_id=s, precision=precision))
                   for s in range(nw)]
        tuned_d = lecqmc.autotune(walkers)
        for _ in range(warmup):
            lecqmc.sweep_batch(walkers, 1)
        ctx.synchronize()
        ctx.set_timing(True)
        ctx.phase_times()
        evd = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        evd[0].record(stream)
        for k in range(steps):
            lecqmc.sweep_batch(walkers, 1)
            evd[k + 1].record(stream)
        torch.cuda.synchronize()
        wl = time.perf_counter() - t1
        msp, cn = ctx.phase_times()
        ctx.set_timing(False)
        smd = [evd[k].elapsed_time(evd[k + 1]) for k in range(steps)]
        lat, par = W.config_dilute()
        res = {"value": nw * lat.n_sites * par.L_tau * steps / wl, "unit": "HS-field updates/s",
               "walkers": nw, "steps": steps, "ms_per_step": wl * 1e3 / steps, "latency_ms": pct(smd),
               "phase_ms_per_launch": {"left_stack": msp[0] / max(cn[0], 1), "forward": msp[1] / max(cn[1], 1),
                                       "fock": msp[2] / max(cn[2], 1)},
               "chain_shape": {"tile": tuned_d[0][0], "chunk": tuned_d[0][1]}}
        for w in walkers:
            w.close()
        return res

    if not args.no_dilute:
        out["dilute_gas"] = {"config": "32x32 periodic Hubbard, U=4, 8+8 particles, beta=16, dtau=0.05 "
                                       "(320 slices), QR every 10 slices",
                             "fp64": run_dilute(lecqmc.FP64)}
        if not args.no_mixed:
            out["dilute_gas"]["mixed"] = {**run_dilute(lecqmc.MIXED),
                                          "dtype": "f32 propagation / f64 QR, inverses, ratios, weights"}

    if not args.no_flat:
        lat, par = W.config_flat_band(256, imbalance=0, beta=10.0)
        fctx = lecqmc.Context(0, stream=stream)
        mk = lambda s: lecqmc.Walker(fctx, lat, W.Params(**{**par.__dict__, "seed": s + 1, "walker_id": s}))
        note("flat band: autotuning on 8 walkers")
        fw = [mk(s) for s in range(8)]
        tf = lecqmc.autotune(fw)
        note(f"flat band: 120 more walkers (shape {tf[0][:2]})")
        fw += [mk(s) for s in range(8, 128)]
        lecqmc.sweep_batch(fw, 1)
        fctx.synchronize()
        fctx.set_timing(True)
        fctx.phase_times()
        t1 = time.perf_counter()
        lecqmc.sweep_batch(fw, 1)
        fctx.synchronize()
        wl = time.perf_counter() - t1
        msp, cn = fctx.phase_times()
        fctx.set_timing(False)
        out["flat_band"] = {"value": len(fw) * lat.n_sites * par.L_tau / wl, "unit": "HS-field updates/s",
                            "walkers": len(fw), "steps": 1, "ms_per_step": wl * 1e3,
                            "phase_ms_per_launch": {"left_stack": msp[0], "forward": msp[1], "fock": msp[2]},
                            "hbm_gib": fctx.bytes_in_use() / 2**30,
                            "chain_shape": {"tile": fw[-1].shape[0], "chunk": fw[-1].shape[1]},
                            "config": "flat-band chain, 256 cells (N=512), t=t'=1, U=2, 128+128 particles, "
                                      "beta=10, dtau=0.05 (200 slices), QR every 10 slices, FP64"}
        for w in fw:
            w.close()
        fctx.close()

    if not args.no_scaling:
        # sweep time against N on the paper's Fig. 1 workload (square Hubbard,
        # dtau = 0.1, U = 2, T = 1: beta = 1, 10 slices; Ne = 100 as 50 + 50),
        # one walker per lattice size, and the fitted power of N
        pts = []
        for Ls in (12, 16, 24, 32, 48, 64, 96, 128):
            lat = W.square_lattice(Ls)
            par = W.Params(U=2.0, beta=1.0, dtau=0.1, n_stab=10, n_up=50, n_dn=50, seed=Ls, walker_id=0)
            note(f"scaling: {Ls}x{Ls}")
            wk = lecqmc.Walker(ctx, lat, par)
            wk.sweep(1)
            ctx.synchronize()
            t1 = time.perf_counter()
            wk.sweep(3)
            ctx.synchronize()
            pts.append((lat.n_sites, (time.perf_counter() - t1) / 3))
            wk.close()
        Ns = np.array([p[0] for p in pts], float)
        ts = np.array([p[1] for p in pts])
        slope_all = float(np.polyfit(np.log(Ns), np.log(ts), 1)[0])
        big = Ns >= 1024
        slope_big = float(np.polyfit(np.log(Ns[big]), np.log(ts[big]), 1)[0])
        out["scaling_fig1"] = {
            "sec_per_sweep_by_N": {str(int(n)): t for n, t in pts},
            "fitted_power_of_N": slope_all, "fitted_power_of_N_N_ge_1024": slope_big,
            "config": "L x L periodic square Hubbard, dtau=0.1, U=2, T=1 (beta=1, 10 slices), 50+50 particles, "
                      "one walker, FP64, default chain shape; seconds per full sweep (flips, QR, Fock swaps)"}

    if not args.no_cp:
        # constrained-path inner walk: one Fock state of the dilute gas, 256
        # random walkers, importance sampling, a comb every 40 slices
        lat, par = W.config_dilute(seed=1)
        ou, od = W.random_occupation(1024, 8, 21), W.random_occupation(1024, 8, 22)
        nw = 256
        note(f"constrained path: {nw} walkers on the dilute gas")
        cp = lecqmc.CPWalk(ctx, lat, par, ou, od, nw, lecqmc.CP_IMPORTANCE, 40)
        cp.run(0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lr = cp.run(1)
        wl = time.perf_counter() - t1
        st = cp.stats()
        cp.close()
        out["constrained_path"] = {
            "value": nw * lat.n_sites * par.L_tau / wl, "unit": "HS-field draws/s", "walkers": nw,
            "ms_per_walk": wl * 1e3, "log_R_estimate": lr, "cuts": st["cuts"],
            "config": "32x32 periodic Hubbard, U=4, one Fock state of 8+8 particles, beta=16, dtau=0.05 "
                      "(320 slices), QR every 10 slices, 256 walkers, importance sampling, comb every 40 "
                      "slices, FP64"}

    if not args.no_serving:
        from paper_2601_08552_amd import serve
        note(f"serving: {args.serve_window:.0f} s window of the 50/s request stream")
        out["serving"] = serve.serving_window(args.serve_window, rate=50.0, seed=0,
                                              budget_bytes=int(200 * 2**30), log=note)

    if not args.no_accuracy:
        import oracle
        acc = {}
        for name, (lat, par) in (("batched_walker0", cfg[min(range(len(cfg)), key=lambda c: cfg[c][0].n_sites
                                                                              * cfg[c][1].L_tau)]),
                                 ("dilute_gas", W.config_dilute(seed=1))):
            note(f"accuracy: {name} vs the oracle, one sweep")
            g = lecqmc.Walker(ctx, lat, par)
            o = oracle.Walker(lat, par)
            lf, lo = g.log_weight()[0], o.log_weight()[0]
            g.sweep(1)
            o.sweep(1)
            sg, so = g.state(), o.state()
            same = all(np.array_equal(np.asarray(a), np.asarray(b)) for a, b in zip(sg, so))
            lt, lto = g.tracked_weight()[0], o.tracked_weight()[0]
            acc[name] = {"N": lat.n_sites, "ne": [par.n_up, par.n_dn], "L_tau": par.L_tau,
                         "fresh_logw_rel_err": abs(lf - lo) / max(1.0, abs(lo)),
                         "chain_identical_after_sweep": bool(same),
                         "tracked_logw_rel_err_after_sweep": abs(lt - lto) / max(1.0, abs(lto)),
                         "near_ties": {"gpu": g.stats()["near_ties"], "oracle": o.stats()["near_ties"]}}
            g.close()
        out["accuracy"] = acc
    ctx.close()

    if not args.no_cpu_baseline:
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        note(f"cpu baseline: the oracle on {procs} host cores")
        out["cpu_baseline"] = cpu_baseline(cfg, procs)


if __name__ == "__main__":
    main()
