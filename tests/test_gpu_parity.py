"""Parity of the gfx950 path (through the C ABI) with the FP64 CPU oracle.

Tolerance: 1e-10 relative for log-weights, Green's functions and ratios
(FP64 on both sides; the two differ only in summation order and in the QR
algorithm, Householder vs Cholesky-QR2, which agree to a few ulps times the
condition number of a stabilisation block).  Integer state (fields,
occupations, sweep counters, move counts) must match exactly: both sides draw
the same Philox4x32-10 numbers and take every decision in FP64.
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


@pytest.fixture(scope="module")
def ctx(lq):
    c = lq.Context(0)
    yield c
    c.close()


def _close(a, b, rtol=RTOL):
    return abs(a - b) <= rtol * max(1.0, abs(b))


CASES = {
    "square4_u4": (lambda: W.square_lattice(4), dict(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=2)),
    "pchain6_ragged": (lambda: W.periodic_chain(6), dict(U=2.0, beta=1.3, dtau=0.1, n_stab=5, n_up=3, n_dn=1)),
    "chain5_open": (lambda: W.open_chain(5), dict(U=3.0, beta=0.8, dtau=0.05, n_stab=7, n_up=2, n_dn=2)),
    "flat4": (lambda: W.flat_band_chain(4), dict(U=2.0, beta=1.0, dtau=0.05, n_stab=6, n_up=2, n_dn=2)),
    "square6_ne5": (lambda: W.square_lattice(6), dict(U=4.0, beta=1.0, dtau=0.1, n_stab=3, n_up=5, n_dn=4)),
    "square4_empty_dn": (lambda: W.square_lattice(4), dict(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=3, n_dn=0)),
    "chain4_full_up": (lambda: W.open_chain(4), dict(U=4.0, beta=0.5, dtau=0.1, n_stab=2, n_up=4, n_dn=1)),
    "square4_one_each": (lambda: W.square_lattice(4), dict(U=2.0, beta=2.0, dtau=0.05, n_stab=10, n_up=1, n_dn=1)),
    "square4_U0": (lambda: W.square_lattice(4), dict(U=0.0, beta=1.0, dtau=0.1, n_stab=5, n_up=2, n_dn=3)),
    "square4_nstab1": (lambda: W.square_lattice(4), dict(U=4.0, beta=0.4, dtau=0.1, n_stab=1, n_up=2, n_dn=2)),
    "square8_ne12": (lambda: W.square_lattice(8), dict(U=4.0, beta=1.0, dtau=0.1, n_stab=10, n_up=12, n_dn=12)),
    # 16 < Ne <= 32 (widest register tile) and Ne > 32 (inverse kept in LDS)
    "square6_ne20": (lambda: W.square_lattice(6), dict(U=4.0, beta=0.6, dtau=0.1, n_stab=3, n_up=20, n_dn=17)),
    "chain40_ne34": (lambda: W.periodic_chain(40), dict(U=2.0, beta=0.4, dtau=0.1, n_stab=2, n_up=34, n_dn=5)),
    # Ne > 64: the Ne x Ne work matrices move from LDS to device memory
    "square12_ne80": (lambda: W.square_lattice(12), dict(U=4.0, beta=0.4, dtau=0.1, n_stab=2, n_up=80, n_dn=70)),
    "flat48_ne72": (lambda: W.flat_band_chain(48), dict(U=2.0, beta=0.5, dtau=0.05, n_stab=4, n_up=72, n_dn=24)),
}


def _pair(lq, ctx, name, seed=3, given=True):
    mk, kw = CASES[name]
    lat = mk()
    par = W.Params(seed=seed, walker_id=seed % 5, **kw)
    if given:
        f = W.random_fields(par.L_tau, lat.n_sites, seed + 100)
        ou = W.random_occupation(lat.n_sites, par.n_up, seed + 200)
        od = W.random_occupation(lat.n_sites, par.n_dn, seed + 300)
        g = lq.Walker(ctx, lat, par, f, ou, od)
        o = oracle.Walker(lat, par, f, ou, od)
    else:
        g = lq.Walker(ctx, lat, par)
        o = oracle.Walker(lat, par)
    return lat, par, g, o


@pytest.mark.parametrize("name", sorted(CASES))
def test_seeded_initial_state_matches(lq, ctx, name):
    """Fields and occupations drawn on the device equal the oracle's draws."""
    _, _, g, o = _pair(lq, ctx, name, seed=11, given=False)
    fg, ug, dg, sg = g.state()
    fo, uo, do, so = o.state()
    assert np.array_equal(fg, fo) and np.array_equal(ug, uo) and np.array_equal(dg, do) and sg == so == 0


@pytest.mark.parametrize("name", sorted(CASES))
def test_log_weight(lq, ctx, name):
    _, _, g, o = _pair(lq, ctx, name)
    lg, sg = g.log_weight()
    lo, so = o.log_weight()
    assert sg == so and _close(lg, lo), (lg, lo)
    assert g.tracked_weight()[1] == so


@pytest.mark.parametrize("name", ["square4_u4", "pchain6_ragged", "flat4", "square6_ne5", "square4_empty_dn",
                                  "chain4_full_up", "square8_ne12", "square6_ne20", "chain40_ne34", "flat48_ne72"])
def test_green(lq, ctx, name):
    lat, par, g, o = _pair(lq, ctx, name)
    for b in sorted({0, 1, par.n_stab, min(par.n_stab + 3, par.L_tau), par.L_tau}):
        for sp in (0, 1):
            Gg, Go = g.green(b, sp), o.green(b, sp)
            assert np.max(np.abs(Gg - Go)) < RTOL, (b, sp)


@pytest.mark.parametrize("name", ["square4_u4", "pchain6_ragged", "chain5_open", "flat4", "square6_ne5",
                                  "square4_empty_dn", "square8_ne12", "square6_ne20", "chain40_ne34",
                                  "square12_ne80", "flat48_ne72"])
def test_flip_ratio(lq, ctx, name):
    lat, par, g, o = _pair(lq, ctx, name)
    rng = np.random.default_rng(7)
    for _ in range(5):
        l, i = int(rng.integers(par.L_tau)), int(rng.integers(lat.n_sites))
        rg, ro = g.flip_ratio(l, i), o.flip_ratio(l, i)
        assert _close(rg, ro), (l, i, rg, ro)


@pytest.mark.parametrize("name", ["square4_u4", "pchain6_ragged", "chain5_open", "flat4", "square6_ne5",
                                  "square4_one_each", "square8_ne12", "square12_ne80", "flat48_ne72"])
def test_swap_ratio(lq, ctx, name):
    lat, par, g, o = _pair(lq, ctx, name)
    _, ou, od, _ = o.state()
    rng = np.random.default_rng(9)
    for sp, occ in ((0, ou), (1, od)):
        if len(occ) in (0, lat.n_sites):
            continue
        for _ in range(3):
            k = int(rng.integers(len(occ)))
            j = int(rng.choice([s for s in range(lat.n_sites) if s not in occ]))
            rg, ro = g.swap_ratio(sp, k, j), o.swap_ratio(sp, k, j)
            assert _close(rg, ro), (sp, k, j, rg, ro)


@pytest.mark.parametrize("name", sorted(CASES))
def test_sweep_trajectory(lq, ctx, name):
    """Whole sweeps: identical Markov chains (fields, occupations, counters),
    weights and sign-weighted estimators."""
    lat, par, g, o = _pair(lq, ctx, name, seed=5, given=False)
    for rep in range(3):
        g.sweep(2, measure=True)
        o.sweep(2, measure=True)
        fg, ug, dg, sg = g.state()
        fo, uo, do, so = o.state()
        assert sg == so
        assert np.array_equal(fg, fo), f"fields differ after {2 * (rep + 1)} sweeps"
        assert np.array_equal(ug, uo) and np.array_equal(dg, do)
        lg, sgg = g.tracked_weight()
        lo, soo = o.tracked_weight()
        assert sgg == soo and _close(lg, lo)
    stg, sto = g.stats(), o.stats()
    for k in ("flip_attempts", "flip_accepts", "swap_attempts", "swap_accepts", "near_ties"):
        assert stg[k] == sto[k], k
    assert stg["max_wrap_err"] < 1e-8 and stg["logw_drift"] < 1e-8
    mg, mo = g.measure(), o.measure()
    assert mg.shape == mo.shape
    assert np.max(np.abs(mg - mo)) < 1e-9 * max(1.0, np.max(np.abs(mo)))


def test_batch_matches_single(lq, ctx):
    """Walkers of different shapes advanced in one batched launch reproduce
    the same walkers advanced alone, bit for bit."""
    names = ["square4_u4", "pchain6_ragged", "flat4", "square6_ne5", "square4_empty_dn", "square8_ne12"]
    alone, batch = [], []
    for t, nm in enumerate(names):
        mk, kw = CASES[nm]
        lat = mk()
        par = W.Params(seed=20 + t, walker_id=t, **kw)
        alone.append(lq.Walker(ctx, lat, par))
        batch.append(lq.Walker(ctx, lat, par))
    for w in alone:
        w.sweep(3, measure=True)
    lq.sweep_batch(batch, 3, measure=True)
    for a, b in zip(alone, batch):
        sa, sb = a.state(), b.state()
        for x, y in zip(sa, sb):
            assert np.array_equal(np.asarray(x), np.asarray(y))
        assert a.tracked_weight() == b.tracked_weight()
        assert np.array_equal(a.measure(), b.measure())


def test_dilute_gas_full_size_first_sweep(lq, ctx):
    """The 32x32 dilute workload (N=1024, 8+8 particles, 320 slices): weights,
    sampled flip ratios and one whole sweep against the oracle."""
    lat, par = W.config_dilute(seed=1, walker_id=0)
    g = lq.Walker(ctx, lat, par)
    o = oracle.Walker(lat, par)
    assert np.array_equal(g.state()[0], o.state()[0])
    lg, sg = g.log_weight()
    lo, so = o.log_weight()
    assert sg == so and _close(lg, lo)
    for (l, i) in ((0, 0), (157, 513), (319, 1023)):
        assert _close(g.flip_ratio(l, i), o.flip_ratio(l, i))
    g.sweep(1)
    o.sweep(1)
    fg, ug, dg, _ = g.state()
    fo, uo, do, _ = o.state()
    assert np.array_equal(ug, uo) and np.array_equal(dg, do)
    assert np.array_equal(fg, fo)
    assert _close(g.tracked_weight()[0], o.tracked_weight()[0])


def test_errors_are_reported(lq, ctx):
    lat = W.square_lattice(4)
    with pytest.raises(lq.LecqmcError) as e:
        lq.Walker(ctx, lat, W.Params(U=4.0, beta=1.0, dtau=0.3, n_stab=4, n_up=2, n_dn=2))
    assert e.value.code == lq.EINVAL
    with pytest.raises(lq.LecqmcError):
        lq.Walker(ctx, lat, W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=0, n_up=2, n_dn=2))
    with pytest.raises(lq.LecqmcError):
        lq.Walker(ctx, lat, W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=17, n_dn=2))
    small = lq.Context(0, hbm_budget_bytes=1000)
    with pytest.raises(lq.LecqmcError) as e:
        lq.Walker(small, lat, W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=2))
    assert e.value.code == lq.ENOMEM
    g = lq.Walker(ctx, lat, W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=2))
    _, ou, _, _ = g.state()
    with pytest.raises(lq.LecqmcError):
        g.swap_ratio(0, 0, int(ou[1]))
