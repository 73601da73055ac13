"""The physics sweeps (paper_2601_08552_amd/physics.py: average sign against
L, main text Fig. 2; flat-band S_par(q=0) and S_zz(q=0) against T, Fig. 4)
on the GPU path: at U = 0 every canonical weight is a diagonal element of a
positive operator, so the sign is exactly 1; at U > 0 the drivers' ratios
equal those of the oracle's chains from the same seeds (the chains are the
same, so the sums agree to rounding)."""
import numpy as np
import pytest

import oracle
from paper_2601_08552_amd import physics
from paper_2601_08552_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2601_08552_amd import lecqmc
    lecqmc.load()
    c = lecqmc.Context(0)
    yield c
    c.close()


def _oracle_bins(lat, par, walkers, warm, sweeps, seed):
    bins = []
    for k in range(walkers):
        o = oracle.Walker(lat, W.Params(**{**par.__dict__, "seed": seed + k, "walker_id": k}))
        o.sweep(warm)
        o.reset_measure()
        o.sweep(sweeps, measure=True)
        bins.append(o.measure())
    return np.array(bins)


def test_average_sign_is_one_at_u0(ctx):
    res = physics.average_sign(ctx, [4, 6], 3, 3, U=0.0, beta=2.0, walkers=4, warm=2, sweeps=4)
    for r in res:
        assert r["sign"] == 1.0 and r["err"] == 0.0


def test_average_sign_matches_the_oracle_chains(ctx):
    res = physics.average_sign(ctx, [4], 3, 3, U=6.0, beta=2.0, walkers=4, warm=2, sweeps=6, seed=9)
    lat = W.square_lattice(4)
    par = W.Params(U=6.0, beta=2.0, dtau=0.05, n_stab=10, n_up=3, n_dn=3, seed=9)
    bins = _oracle_bins(lat, par, 4, 2, 6, 9)
    s, e = physics.jackknife_ratio(bins[:, 0], bins[:, 1])
    print(f"<sign> gpu {res[0]['sign']:.12f} oracle {s:.12f}", flush=True)
    assert abs(res[0]["sign"] - s) < 1e-12 and -1.0 <= s <= 1.0


def test_flat_band_order_matches_the_oracle_chains(ctx):
    res = physics.flat_band_order(ctx, [1.0], 4, U=2.0, walkers=4, warm=2, sweeps=6, seed=3)
    lat = W.flat_band_chain(4, -0.2, 1.0, 1.0, -0.2)
    par = W.Params(U=2.0, beta=1.0, dtau=0.05, n_stab=10, n_up=2, n_dn=2, seed=3)
    bins = _oracle_bins(lat, par, 4, 2, 6, 3)
    sp, _ = physics.jackknife_ratio(bins[:, 4], bins[:, 0])
    sz, _ = physics.jackknife_ratio(bins[:, 5], bins[:, 0])
    print(f"S_par gpu {res[0]['S_par_q0']:.10f} oracle {sp:.10f}; S_zz gpu {res[0]['S_zz_q0']:.10f} "
          f"oracle {sz:.10f}", flush=True)
    assert abs(res[0]["S_par_q0"] - sp) < 1e-9 * max(1.0, abs(sp))
    assert abs(res[0]["S_zz_q0"] - sz) < 1e-9 * max(1.0, abs(sz))
