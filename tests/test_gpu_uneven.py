"""The batched uneven-walker workload at full size: 256 independent chains,
L x L square lattices with L in {16, 24, 32, 48, 64} (N up to 4096), Ne per
spin in [4, 32], U in [2, 6], beta in {8, 16} (up to 320 slices), dtau =
0.05, a QR every 10 slices.  The walkers are autotuned, held in one fixed
batch (one launch per phase for all 256), and the sweep is recorded into a
HIP graph and replayed.  Sampled walkers -- the smallest and largest
lattices and Ne at both ends -- must follow the oracle's chain.
"""
import numpy as np
import pytest

import oracle
from paper_2601_08552_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.fixture(scope="module")
def lq():
    from paper_2601_08552_amd import lecqmc
    lecqmc.load()
    return lecqmc


def _samples(cfg):
    """Indices covering both ends of N and Ne, and the costliest walker."""
    idx = sorted(range(len(cfg)), key=lambda c: (cfg[c][0].n_sites, cfg[c][1].n_up, cfg[c][1].L_tau))
    pick = [idx[0], idx[-1]]
    for N in (256, 1024, 4096):
        of_n = [c for c in idx if cfg[c][0].n_sites == N]
        pick += [of_n[0], of_n[-1]]
    return sorted(set(pick))


def test_uneven_batch_full_size_graph_and_oracle(lq):
    import torch
    cfg = W.config_batched(256)
    s = torch.cuda.Stream()
    ctx = lq.Context(0, stream=s)
    ws = [lq.Walker(ctx, lat, par) for lat, par in cfg]
    print("created", len(ws), "walkers,", ctx.bytes_in_use() / 2**30, "GiB", flush=True)
    res = lq.autotune(ws)
    keys = {}
    for (tile, chunk, ms), (lat, par) in zip(res, cfg):
        assert tile in (0, 9) or max(par.n_up, par.n_dn) <= 8 * tile
        assert chunk in (4, 8, 16, 32) and ms > 0
        keys.setdefault((lat.n_sites, par.n_up, par.n_dn), set()).add((tile, chunk))
    assert all(len(v) == 1 for v in keys.values())    # one shape per key
    print("tuned shapes:", sorted({r[:2] for r in res}), flush=True)
    b = lq.Batch(ws)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.sweep(1)
    torch.cuda.synchronize()
    assert all(w.stats()["sweeps"] == 0 for w in ws)   # capture ran nothing
    g.replay()
    torch.cuda.synchronize()
    print("replayed one sweep", flush=True)
    for w in ws:
        st = w.stats()
        assert st["sweeps"] == 1
        assert st["flip_attempts"] == w.N * w.L
        assert st["logw_drift"] < 1e-6
    for c in _samples(cfg):
        lat, par = cfg[c]
        print(f"oracle walker {c}: N={lat.n_sites} Ne={par.n_up} L_tau={par.L_tau}", flush=True)
        o = oracle.Walker(lat, par)
        o.sweep(1)
        fg, ug, dg, sg = ws[c].state()
        fo, uo, do, so = o.state()
        assert sg == so
        assert np.array_equal(ug, uo) and np.array_equal(dg, do)
        assert np.array_equal(fg, fo)
        lg, sgg = ws[c].tracked_weight()
        lo, soo = o.tracked_weight()
        assert sgg == soo and abs(lg - lo) <= RTOL * max(1.0, abs(lo))
    b.close()
    ctx.close()
