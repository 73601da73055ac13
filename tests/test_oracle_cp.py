"""Pins of the oracle's constrained-path (phaseless) inner walk (SM Sec. VI)
against what the mathematics fixes, independently of the oracle's own
arithmetic:

- H = H_0 (U = 0): every overlap ratio is 1, so R(eta) = 1 exactly, with and
  without population control;
- telescoping: a walker's final weight is the product of its site-by-site
  overlap ratios, which must equal the ratio of determinants of the dense
  propagator products (tests/exact.py) for the field path it drew:
  free sampling      log w = log det(P^T B(s) P) - log W_T(eta),
  importance sampling log w + sum log p(s) = -N L log 2 + the same;
  this pins the trial state, the walker propagation, the Sherman-Morrison
  updates, the QR stabilisation and the sign conventions of the fields;
- unbiasedness where the constraint never cuts (small U): the mean of the
  estimates of R(eta) agrees within 4 sigma with the Trotter-exact many-body
  value e^{beta U N_e / 2} <eta|T^L|eta> / <eta|T_0^L|eta> from sector ED,
  for both sampling modes, with and without the comb;
- two-stage sampling: the outer U = 0 LEC-QMC chain draws eta from
  W_T(eta) / Z_0, so the mean of R over its samples estimates Z / Z_0, which
  sector ED fixes as e^{beta U N_e / 2} Tr T^L / Tr T_0^L;
- the constraint: at strong coupling, free sampling cuts walkers; a cut walker
  has weight 0, draws nothing more, and a comb never copies it.
"""
import dataclasses

import numpy as np
import pytest

import exact
import oracle
from paper_2601_08552_amd import workloads as W


def _case(U=2.0, beta=1.0, n_stab=4, seed=11):
    lat = W.periodic_chain(6)
    par = W.Params(U=U, beta=beta, dtau=0.1, n_stab=n_stab, n_up=2, n_dn=1, seed=seed)
    return lat, par, np.array([0, 3]), np.array([2])


def _exact_R(lat, par, ou, od):
    ed = exact.SectorED(lat, par)
    ed0 = exact.SectorED(lat, dataclasses.replace(par, U=0.0))
    idx = ed.bu.index(tuple(int(x) for x in ou)) * len(ed.bd) + ed.bd.index(tuple(int(x) for x in od))
    ne = par.n_up + par.n_dn
    return np.exp(par.beta * par.U * ne / 2) * ed.TL[idx, idx] / ed0.TL[idx, idx]


@pytest.mark.parametrize("pc", [0, 3])
def test_cp_is_exactly_one_at_u0(pc):
    lat, par, ou, od = _case(U=0.0)
    c = oracle.CPWalk(lat, par, ou, od, 8, oracle.CP_IMPORTANCE, pc)
    assert c.run(0) == 0.0
    st = c.stats()
    assert st["cuts"] == 0 and st["alive"] == 8 and st["log_pc"] == 0.0


@pytest.mark.parametrize("mode", [oracle.CP_FREE, oracle.CP_IMPORTANCE])
@pytest.mark.parametrize("n_stab", [1, 4, 10])
def test_cp_walker_weight_telescopes_to_determinant_ratio(mode, n_stab):
    lat, par, ou, od = _case(n_stab=n_stab)
    p0 = dataclasses.replace(par, U=0.0)
    log_wt, s_wt = exact.log_weight_direct(lat, p0, np.ones((par.L_tau, lat.n_sites), np.int8), ou, od)
    assert s_wt == 1
    c = oracle.CPWalk(lat, par, ou, od, 12, mode)
    c.run(7)
    assert c.stats()["cuts"] == 0
    for a in range(12):
        lw, lq, f = c.walker(a)
        assert set(np.unique(f)) <= {-1, 1}
        ld, sg = exact.log_weight_direct(lat, par, f, ou, od)
        assert sg == 1
        if mode == oracle.CP_FREE:
            assert abs(lw - (ld - log_wt)) < 1e-11
        else:
            assert abs(lw + lq - (-lat.n_sites * par.L_tau * np.log(2.0) + ld - log_wt)) < 1e-11


@pytest.mark.parametrize("mode,pc,n_runs", [(oracle.CP_IMPORTANCE, 0, 30), (oracle.CP_IMPORTANCE, 3, 30),
                                            (oracle.CP_FREE, 0, 60), (oracle.CP_FREE, 3, 60)])
def test_cp_unbiased_against_sector_ed(mode, pc, n_runs):
    lat, par, ou, od = _case()
    R = _exact_R(lat, par, ou, od)
    ests = []
    for t in range(n_runs):
        c = oracle.CPWalk(lat, par, ou, od, 64, mode, pc)
        ests.append(np.exp(c.run(t)))
        assert c.stats()["cuts"] == 0
    m, e = np.mean(ests), np.std(ests, ddof=1) / np.sqrt(n_runs)
    assert abs(m - R) <= 4 * e, (m, e, R)
    assert e < 0.1 * R


def test_cp_two_stage_partition_ratio_against_sector_ed():
    lat, par, _, _ = _case(U=1.0, beta=0.8)
    ed = exact.SectorED(lat, par)
    ed0 = exact.SectorED(lat, dataclasses.replace(par, U=0.0))
    ne = par.n_up + par.n_dn
    ref = np.exp(par.beta * par.U * ne / 2) * np.trace(ed.TL) / np.trace(ed0.TL)
    rs = oracle.cp_partition_ratio(lat, par, n_eta=400, sweeps_between=2, n_walkers=16)
    bins = rs.reshape(20, -1).mean(axis=1)
    m, e = bins.mean(), bins.std(ddof=1) / np.sqrt(len(bins))
    assert abs(m - ref) <= 4 * e, (m, e, ref)
    assert e < 0.05 * ref


def test_cp_constraint_cuts_and_comb_never_copies_a_cut_walker():
    lat = W.periodic_chain(4)
    par = W.Params(U=8.0, beta=4.0, dtau=0.1, n_stab=5, n_up=2, n_dn=2, seed=5)
    ou, od = np.array([0, 1]), np.array([1, 2])
    c = oracle.CPWalk(lat, par, ou, od, 64, oracle.CP_FREE, 0)
    c.run(0)
    st = c.stats()
    assert st["cuts"] > 0 and st["alive"] == 64 - st["cuts"]
    for a in range(64):
        lw, _, f = c.walker(a)
        if lw == -np.inf:
            # drew nothing after the cut: its path ends in unset fields
            assert (f.ravel() == 0).any() and f.ravel()[-1] == 0
        else:
            assert (f != 0).all()
    # a comb after every slice: a walker can only be dead if it died in the
    # last slice, and every path is complete up to that slice
    c = oracle.CPWalk(lat, par, ou, od, 64, oracle.CP_FREE, 1)
    c.run(1)
    assert c.stats()["cuts"] > 0
    for a in range(64):
        _, _, f = c.walker(a)
        assert (f[:-1] != 0).all()
