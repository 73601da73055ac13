"""Constrained-path inner walk (SM Sec. VI) on the gfx950 path through the C
ABI (lecqmc_cp_*), against the oracle's walk from the same seed: the same
field paths (bit for bit), the same cut walkers, and per-walker log weights,
log draw probabilities and the estimate of R(eta) within 1e-9 (small) or 1e-8
(full size) absolute, for both sampling modes, with and without the comb.
The walks share nothing but their inputs and the counter-based generator's
published definition (walker slot a, stream 7, sweep = tag)."""
import numpy as np
import pytest

import oracle
from paper_2601_08552_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _compare(lq, ctx, lat, par, ou, od, nw, mode, pc, tag, tol):
    g = lq.CPWalk(ctx, lat, par, ou, od, nw, mode, pc)
    o = oracle.CPWalk(lat, par, ou, od, nw, mode, pc)
    lg, lo = g.run(tag), o.run(tag)
    sg, so = g.stats(), o.stats()
    print(f"N={lat.n_sites} ne={par.n_up}+{par.n_dn} L={par.L_tau} nw={nw} mode={mode} pc={pc}: "
          f"log R gpu {lg:.12f} oracle {lo:.12f}, cuts {sg['cuts']}/{so['cuts']}", flush=True)
    assert sg["cuts"] == so["cuts"] and sg["alive"] == so["alive"]
    assert abs(sg["log_pc"] - so["log_pc"]) <= tol * max(1.0, abs(so["log_pc"]))
    if lo == -np.inf:
        assert lg == -np.inf
    else:
        assert abs(lg - lo) <= tol * max(1.0, abs(lo))
    for a in range(nw):
        wg, qg, fg = g.walker(a)
        wo, qo, fo = o.walker(a)
        assert np.array_equal(fg, fo), f"walker {a}: field paths differ"
        if wo == -np.inf:
            assert wg == -np.inf
        else:
            assert abs(wg - wo) <= tol * max(1.0, abs(wo)), (a, wg, wo)
        assert abs(qg - qo) <= tol * max(1.0, abs(qo)), (a, qg, qo)
    g.close()
    return sg


@pytest.mark.parametrize("mode", ["importance", "free"])
@pytest.mark.parametrize("pc", [0, 3])
@pytest.mark.parametrize("case", ["ring6", "sq6"])
def test_cp_walk_matches_oracle(lq, ctx, mode, pc, case):
    if case == "ring6":
        lat = W.periodic_chain(6)
        par = W.Params(U=2.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=1, seed=11)
        ou, od = [0, 3], [2]
    else:
        lat = W.square_lattice(6)
        par = W.Params(U=4.0, beta=1.2, dtau=0.1, n_stab=5, n_up=7, n_dn=5, seed=12)
        ou, od = W.random_occupation(36, 7, 3), W.random_occupation(36, 5, 4)
    m = lq.CP_IMPORTANCE if mode == "importance" else lq.CP_FREE
    _compare(lq, ctx, lat, par, ou, od, 24, m, pc, tag=5, tol=1e-9)


@pytest.mark.parametrize("pc", [0, 1])
def test_cp_cut_walkers_match_oracle(lq, ctx, pc):
    """Strong coupling, free sampling: the phaseless cut kills walkers; the
    same ones die at the same site, and a comb after every slice never
    copies a dead walker."""
    lat = W.periodic_chain(4)
    par = W.Params(U=8.0, beta=4.0, dtau=0.1, n_stab=5, n_up=2, n_dn=2, seed=5)
    st = _compare(lq, ctx, lat, par, [0, 1], [1, 2], 64, lq.CP_FREE, pc, tag=pc, tol=1e-9)
    assert st["cuts"] > 0


def test_cp_is_exactly_one_at_u0(lq, ctx):
    lat = W.square_lattice(4)
    par = W.Params(U=0.0, beta=1.0, dtau=0.1, n_stab=4, n_up=3, n_dn=2, seed=1)
    g = lq.CPWalk(ctx, lat, par, [0, 5, 9], [3, 12], 8, lq.CP_IMPORTANCE, 4)
    assert g.run(0) == 0.0
    assert g.stats() == {"log_pc": 0.0, "cuts": 0, "alive": 8}
    g.close()


def test_cp_refuses_what_it_does_not_handle(lq, ctx):
    lat = W.square_lattice(10)
    par = W.Params(U=2.0, beta=1.0, dtau=0.1, n_stab=5, n_up=65, n_dn=2, seed=1)
    with pytest.raises(lq.LecqmcError) as e:
        lq.CPWalk(ctx, lat, par, list(range(65)), [0, 1], 4)
    assert e.value.code == lq.EINVAL
    par = W.Params(U=2.0, beta=1.0, dtau=0.1, n_stab=5, n_up=2, n_dn=2, seed=1, precision=lq.MIXED)
    with pytest.raises(lq.LecqmcError) as e:
        lq.CPWalk(ctx, lat, par, [0, 1], [0, 1], 4)
    assert e.value.code == lq.EINVAL
    par = W.Params(U=2.0, beta=1.0, dtau=0.1, n_stab=5, n_up=2, n_dn=2, seed=1)
    with pytest.raises(lq.LecqmcError):
        lq.CPWalk(ctx, lat, par, [0, 1], [0, 1], 0)
    with pytest.raises(lq.LecqmcError):
        lq.CPWalk(ctx, lat, par, [0, 0], [0, 1], 4)


def test_cp_dilute_gas_full_size(lq, ctx):
    """The 32 x 32 dilute gas (8 + 8 particles, beta = 16: 320 slices, a QR
    every 10) as the Fock state of the walk: 8 walkers, importance sampling,
    a comb every 40 slices."""
    lat, par = W.config_dilute(seed=1)
    ou, od = W.random_occupation(1024, 8, 21), W.random_occupation(1024, 8, 22)
    _compare(lq, ctx, lat, par, ou, od, 8, lq.CP_IMPORTANCE, 40, tag=2, tol=1e-8)
