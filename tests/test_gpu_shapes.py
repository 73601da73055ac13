"""Flip-chain shapes (register tile, chunk) and the autotuner.

Every shape must sample the oracle's chain: identical fields, occupations
and counters, log-weights within 1e-10 relative and estimators within 1e-9.
The chunk (sites staged per step) must not change a single bit; the tile
changes only the rounding order of the ratio sums.  The autotuner must leave
every walker's chain where it was and hand its choice to later walkers of
the same shape key.  A batch whose walkers have different shapes runs them
in one launch (each walker dispatches its own shape) and must reproduce the
walkers swept alone bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2601_08552_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-10
TILES = (1, 2, 4, 0, 9, 10)
CHUNKS = (4, 8, 16, 32)


@pytest.fixture(scope="module")
def lq():
    from paper_2601_08552_amd import lecqmc
    lecqmc.load()
    return lecqmc


def _close(a, b, rtol=RTOL):
    return abs(a - b) <= rtol * max(1.0, abs(b))


def _case(ne_up, ne_dn, Ls=6, U=4.0, beta=1.5, seed=5, n_stab=5):
    lat = W.square_lattice(Ls)
    par = W.Params(U=U, beta=beta, dtau=0.05, n_stab=n_stab, n_up=ne_up, n_dn=ne_dn, seed=seed, walker_id=1)
    return lat, par


def _same(a, b):
    for x, y in zip(a.state(), b.state()):
        if not np.array_equal(np.asarray(x), np.asarray(y)):
            return False
    return a.tracked_weight() == b.tracked_weight() and np.array_equal(a.measure(), b.measure())


def _matches_oracle(g, o):
    fg, ug, dg, sg = g.state()
    fo, uo, do, so = o.state()
    assert sg == so
    assert np.array_equal(fg, fo) and np.array_equal(ug, uo) and np.array_equal(dg, do)
    lg, sgg = g.tracked_weight()
    lo, soo = o.tracked_weight()
    assert sgg == soo and _close(lg, lo)
    stg, sto = g.stats(), o.stats()
    for k in ("flip_attempts", "flip_accepts", "swap_attempts", "swap_accepts", "near_ties"):
        assert stg[k] == sto[k], k
    assert stg["logw_drift"] < 1e-8
    mg, mo = g.measure(), o.measure()
    assert np.max(np.abs(mg - mo)) < 1e-9 * max(1.0, np.max(np.abs(mo)))


def test_every_shape_follows_the_oracle(lq):
    """All 20 valid (tile, chunk) shapes on one walker (Ne = 5 + 3, ragged last
    chunk: N = 36) against the oracle's sweep."""
    lat, par = _case(5, 3)
    o = oracle.Walker(lat, par)
    o.sweep(2, measure=True)
    ctx = lq.Context(0)
    for t in TILES:
        for c in CHUNKS:
            print(f"shape tile={t} chunk={c}", flush=True)
            g = lq.Walker(ctx, lat, par)
            if (t == 9 and c > 16) or (t == 10 and c != 16):
                # the delayed chain takes at most 16 sites per chunk, the
                # matrix-core chain exactly one 16-wide tile
                with pytest.raises(lq.LecqmcError) as e:
                    g.set_shape(t, c)
                assert e.value.code == lq.EINVAL
                g.close()
                continue
            g.set_shape(t, c)
            assert g.shape == (t, c)
            g.sweep(2, measure=True)
            _matches_oracle(g, o)
            g.close()
    ctx.close()


def test_chunk_changes_no_bit(lq):
    """The same walker with chunks 4 and 32 (tile fixed): identical state,
    weights, estimators and drift statistics."""
    lat, par = _case(12, 9, Ls=8, beta=1.0)
    ctx = lq.Context(0)
    a = lq.Walker(ctx, lat, par)
    b = lq.Walker(ctx, lat, par)
    a.set_shape(2, 4)
    b.set_shape(2, 32)
    a.sweep(2, measure=True)
    b.sweep(2, measure=True)
    assert _same(a, b)
    assert a.stats()["logw_drift"] == b.stats()["logw_drift"]
    ctx.close()


def test_shape_validation(lq):
    """Shapes the walker's Ne cannot use are refused; a walker of a live
    batch keeps its shape."""
    lat, par = _case(12, 3, Ls=6)
    ctx = lq.Context(0)
    w = lq.Walker(ctx, lat, par)
    assert w.shape == (2, 32)               # default for 8 < Ne <= 16
    for bad in ((1, 16), (3, 16), (16, 16), (2, 12), (2, 64), (-1, 8)):
        with pytest.raises(lq.LecqmcError) as e:
            w.set_shape(*bad)
        assert e.value.code == lq.EINVAL
    b = lq.Batch([w])
    with pytest.raises(lq.LecqmcError) as e:
        w.set_shape(4, 8)
    assert e.value.code == lq.ESTATE
    with pytest.raises(lq.LecqmcError) as e:
        lq.autotune([w])
    assert e.value.code == lq.ESTATE
    b.close()
    w.set_shape(4, 8)
    assert w.shape == (4, 8)
    ctx.close()


def test_autotune_keeps_the_chain(lq):
    """Tuning runs whole forward passes but restores every walker: state,
    weights and counters are unchanged, and the next sweep is the oracle's.
    A walker created later with a tuned key starts with the tuned shape."""
    specs = [(3, 2, 6), (11, 7, 6), (20, 18, 6), (36, 4, 8)]
    ctx = lq.Context(0)
    made = []
    for (nu, nd, Ls) in specs:
        lat, par = _case(nu, nd, Ls=Ls, beta=1.0, seed=7 + nu)
        made.append((lat, par, lq.Walker(ctx, lat, par)))
    ws = [m[2] for m in made]
    lq.sweep_batch(ws, 1, measure=True)
    before = [(w.state(), w.tracked_weight(), w.stats(), w.measure()) for w in ws]
    res = lq.autotune(ws)
    assert len(res) == len(ws)
    for (tile, chunk, ms), w, (nu, nd, _) in zip(res, ws, specs):
        assert (tile, chunk) == w.shape
        assert tile in TILES and chunk in CHUNKS and ms > 0
        assert tile in (0, 9, 10) or max(nu, nd) <= 8 * tile
    for w, (st, tw, stats, meas) in zip(ws, before):
        for x, y in zip(w.state(), st):
            assert np.array_equal(np.asarray(x), np.asarray(y))
        assert w.tracked_weight() == tw
        assert w.stats() == stats
        assert np.array_equal(w.measure(), meas)
    # the chains continue as the oracle's (two sweeps from the seeded start)
    lq.sweep_batch(ws, 1, measure=True)
    for (lat, par, g) in made:
        o = oracle.Walker(lat, par)
        o.sweep(2, measure=True)
        _matches_oracle(g, o)
    # later walkers of a tuned key inherit the shape
    for (lat, par, g) in made:
        assert lq.Walker(ctx, lat, par).shape == g.shape
    ctx.close()


def test_mixed_shape_batch_equals_alone(lq):
    """Walkers with tiles 1, 2, 4, 0, 9 (delayed) and 10 (matrix cores) and different chunks in one batch
    (one launch that dispatches each walker's shape) against the same
    walkers swept alone."""
    specs = [(3, 2, 6, (1, 32)), (11, 7, 6, (2, 8)), (20, 18, 6, (4, 16)), (36, 4, 8, (0, 4)), (6, 6, 8, (4, 32)),
             (13, 9, 6, (0, 8)), (27, 30, 6, (4, 8)), (12, 5, 6, (9, 16)), (40, 33, 8, (9, 8)),
             (21, 19, 6, (10, 16)), (5, 3, 6, (10, 16)), (44, 37, 8, (10, 16))]
    ctx = lq.Context(0)
    alone, batch = [], []
    for (nu, nd, Ls, shp) in specs:
        lat, par = _case(nu, nd, Ls=Ls, beta=1.0, seed=30 + nu)
        a, b = lq.Walker(ctx, lat, par), lq.Walker(ctx, lat, par)
        a.set_shape(*shp)
        b.set_shape(*shp)
        alone.append(a)
        batch.append(b)
    for a in alone:
        a.sweep(2, measure=True)
    bt = lq.Batch(batch)
    bt.sweep(2, measure=True)
    ctx.synchronize()
    for a, b in zip(alone, batch):
        assert _same(a, b)
        assert a.stats()["logw_drift"] == b.stats()["logw_drift"]
    bt.close()
    ctx.close()


@pytest.mark.parametrize("big_shape", [(0, 4), (9, 16), (10, 16)])
def test_large_ne_in_a_batch(lq, big_shape):
    """A walker with Ne > 64 (work matrices in device memory for the whole
    launch) batched with walkers that alone keep them in LDS: every walker
    matches itself swept alone, and the large one matches the oracle."""
    specs = [(3, 2, 6), (40, 12, 8), (90, 66, 12)]
    ctx = lq.Context(0)
    alone, batch, cfg = [], [], []
    for (nu, nd, Ls) in specs:
        lat, par = _case(nu, nd, Ls=Ls, beta=0.5, seed=50 + nu)
        cfg.append((lat, par))
        alone.append(lq.Walker(ctx, lat, par))
        batch.append(lq.Walker(ctx, lat, par))
    for w in (alone[-1], batch[-1]):
        w.set_shape(*big_shape)
    for a in alone:
        a.sweep(2, measure=True)
    lq.sweep_batch(batch, 2, measure=True)
    for a, b in zip(alone, batch):
        assert _same(a, b)
    lat, par = cfg[-1]
    o = oracle.Walker(lat, par)
    o.sweep(2, measure=True)
    _matches_oracle(batch[-1], o)
    ctx.close()


def test_batch_moves_matrices_out_of_lds(lq):
    """Two walkers that each fit LDS alone but not together (Ne = 64 with the
    inverse in memory, and Ne = 32 with a 32-site chunk): the launch moves its
    Ne x Ne work matrices to device memory, and both walkers still match
    themselves swept alone."""
    specs = [((64, 40), 8, (0, 4)), ((32, 30), 8, (4, 32))]
    ctx = lq.Context(0)
    alone, batch = [], []
    for (ne, Ls, shp) in specs:
        lat, par = _case(ne[0], ne[1], Ls=Ls, beta=0.5, seed=70 + ne[0])
        a, b = lq.Walker(ctx, lat, par), lq.Walker(ctx, lat, par)
        a.set_shape(*shp)
        b.set_shape(*shp)
        alone.append(a)
        batch.append(b)
    for a in alone:
        a.sweep(2, measure=True)
    lq.sweep_batch(batch, 2, measure=True)
    for a, b in zip(alone, batch):
        assert _same(a, b)
    ctx.close()


@pytest.mark.parametrize("ne", [(1, 1), (8, 8), (16, 15), (17, 2), (32, 32), (33, 31), (48, 0), (64, 64)])
def test_matrix_core_chain_follows_the_oracle(lq, ne):
    """The matrix-core chain (tile 10) on tile edges of Ne (1, 15/16/17,
    32/33, 48 with an empty spin, 64) and a ragged last chunk (N = 36 or 100):
    the oracle's chain, weights and estimators."""
    Ls = 6 if max(ne) <= 20 else 10
    lat, par = _case(ne[0], ne[1], Ls=Ls, beta=1.0, seed=90 + ne[0])
    o = oracle.Walker(lat, par)
    o.sweep(2, measure=True)
    ctx = lq.Context(0)
    g = lq.Walker(ctx, lat, par)
    g.set_shape(10, 16)
    print(f"tile 10, Ne = {ne}", flush=True)
    g.sweep(2, measure=True)
    _matches_oracle(g, o)
    ctx.close()
