"""Physics sweeps of the main text, run on the gfx950 path.

- average_sign: the average sign against the linear size L at fixed particle
  number and temperature on the square-lattice Hubbard model (main text,
  "Sign problem in the dilute limit", Fig. 2);
- flat_band_order: S_par(q=0) and S_zz(q=0) of the flat-band chain against
  temperature (main text Fig. 4 and its definitions).

The paper states only some of these runs' parameters (Fig. 2 fixes neither
N_e, U nor T in the text); the defaults below are a reading and are printed
with every result.  Each walker is one independent chain and one jackknife
bin.

    python -m paper_2601_08552_amd.physics sign --L 4 6 8 12 16 --ne 4 4 --U 4 --beta 4
    python -m paper_2601_08552_amd.physics flat --cells 32 --T 1 0.5 0.25 --U 2
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import lecqmc
from . import workloads as W


def jackknife_ratio(num, den):
    """Ratio of sums and its jackknife error over bins (one bin per walker)."""
    num, den = np.asarray(num, float), np.asarray(den, float)
    n = len(num)
    est = num.sum() / den.sum()
    if n < 2:
        return float(est), float("nan")
    loo = (num.sum() - num) / (den.sum() - den)
    err = np.sqrt((n - 1) / n * np.sum((loo - loo.mean()) ** 2))
    return float(est), float(err)


def _run(ctx, lat, par, walkers, warm, sweeps, seed):
    ws = [lecqmc.Walker(ctx, lat, W.Params(**{**par.__dict__, "seed": seed + k, "walker_id": k}))
          for k in range(walkers)]
    lecqmc.autotune(ws)
    lecqmc.sweep_batch(ws, warm)
    for w in ws:
        w.reset_measure()
    lecqmc.sweep_batch(ws, sweeps, measure=True)
    bins = np.array([w.measure() for w in ws])
    for w in ws:
        w.close()
    return bins


def average_sign(ctx, Ls, n_up, n_dn, U, beta, dtau=0.05, n_stab=10, walkers=32, warm=20, sweeps=100, seed=1):
    """<sign> = sum of signs / number of measurements, for each L (N = L^2)."""
    out = []
    for L in Ls:
        lat = W.square_lattice(L)
        par = W.Params(U=U, beta=beta, dtau=dtau, n_stab=n_stab, n_up=n_up, n_dn=n_dn, seed=seed)
        bins = _run(ctx, lat, par, walkers, warm, sweeps, seed)
        s, e = jackknife_ratio(bins[:, 0], bins[:, 1])
        out.append({"L": L, "N": L * L, "density": (n_up + n_dn) / (L * L), "sign": s, "err": e})
    return out


def flat_band_order(ctx, temperatures, n_cells, U, t1=-0.2, t2=1.0, dtau=0.05, n_stab=10, walkers=32, warm=20,
                    sweeps=100, seed=1, imbalance=0):
    """S_par(q=0) and S_zz(q=0) per cell of the flat-band chain at half
    filling of the flat band (N_up + N_dn = n_cells), per temperature."""
    out = []
    lat = W.flat_band_chain(n_cells, t1, t2, t2, t1)
    ne = n_cells
    n_up, n_dn = (ne + imbalance) // 2, (ne - imbalance) // 2
    for T in temperatures:
        beta = round(1.0 / T / dtau) * dtau
        par = W.Params(U=U, beta=beta, dtau=dtau, n_stab=n_stab, n_up=n_up, n_dn=n_dn, seed=seed)
        bins = _run(ctx, lat, par, walkers, warm, sweeps, seed)
        sp, spe = jackknife_ratio(bins[:, 4], bins[:, 0])
        sz, sze = jackknife_ratio(bins[:, 5], bins[:, 0])
        sg, sge = jackknife_ratio(bins[:, 0], bins[:, 1])
        out.append({"T": T, "beta": beta, "S_par_q0": sp, "S_par_err": spe, "S_zz_q0": sz, "S_zz_err": sze,
                    "sign": sg, "sign_err": sge})
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("sign")
    a.add_argument("--L", type=int, nargs="+", default=[4, 6, 8, 12, 16, 24])
    a.add_argument("--ne", type=int, nargs=2, default=[4, 4])
    a.add_argument("--U", type=float, default=4.0)
    a.add_argument("--beta", type=float, default=4.0)
    b = sub.add_parser("flat")
    b.add_argument("--cells", type=int, default=32)
    b.add_argument("--T", type=float, nargs="+", default=[1.0, 0.5, 0.25, 0.125])
    b.add_argument("--U", type=float, default=2.0)
    for p in (a, b):
        p.add_argument("--walkers", type=int, default=32)
        p.add_argument("--warm", type=int, default=20)
        p.add_argument("--sweeps", type=int, default=100)
    args = ap.parse_args()
    ctx = lecqmc.Context(0)
    if args.cmd == "sign":
        res = average_sign(ctx, args.L, args.ne[0], args.ne[1], args.U, args.beta, walkers=args.walkers,
                           warm=args.warm, sweeps=args.sweeps)
        params = {"ne": args.ne, "U": args.U, "beta": args.beta}
    else:
        res = flat_band_order(ctx, args.T, args.cells, args.U, walkers=args.walkers, warm=args.warm,
                              sweeps=args.sweeps)
        params = {"cells": args.cells, "U": args.U, "t1": -0.2, "t2": 1.0}
    print(json.dumps({"run": args.cmd, "params": {**params, "walkers": args.walkers, "warm": args.warm,
                                                 "sweeps": args.sweeps}, "results": res}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
