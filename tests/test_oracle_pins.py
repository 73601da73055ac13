"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, dense brute-force determinants and Green's functions,
exact diagonalisation, free-fermion closed forms and exact identities.
"""
import os

import mpmath
import numpy as np
import pytest

import exact
import oracle
from paper_2601_08552_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert list(oracle.philox4x32_10(ctr, key)) == out


def test_uniform_in_unit_interval_and_flat():
    u = np.array([oracle.uniform(7, 3, oracle.S_FLIP, 1, a, b) for a in range(40) for b in range(50)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    # different streams / walkers / seeds decorrelate
    v = np.array([oracle.uniform(7, 4, oracle.S_FLIP, 1, a, b) for a in range(40) for b in range(50)])
    assert abs(np.corrcoef(u, v)[0, 1]) < 0.1


def _lattices():
    return [
        ("square4", W.square_lattice(4)),
        ("pchain6", W.periodic_chain(6)),
        ("chain5", W.open_chain(5)),
        ("flat4", W.flat_band_chain(4)),
    ]


@pytest.mark.parametrize("name,lat", _lattices())
@pytest.mark.parametrize("U,beta,dtau,nstab,nu,nd", [
    (4.0, 1.0, 0.1, 3, 2, 1),     # 10 slices, last block shorter
    (2.0, 0.6, 0.05, 4, 1, 2),
    (0.0, 1.0, 0.1, 5, 2, 2),     # U = 0: fields inert
])
def test_log_weight_matches_dense_product(name, lat, U, beta, dtau, nstab, nu, nd):
    N = lat.n_sites
    par = W.Params(U=U, beta=beta, dtau=dtau, n_stab=nstab, n_up=min(nu, N), n_dn=min(nd, N), seed=3)
    f = W.random_fields(par.L_tau, N, 11)
    ou, od = W.random_occupation(N, par.n_up, 5), W.random_occupation(N, par.n_dn, 6)
    w = oracle.Walker(lat, par, f, ou, od)
    la, sg = w.log_weight()
    la0, sg0 = exact.log_weight_direct(lat, par, f, ou, od)
    assert sg == sg0
    assert abs(la - la0) <= 1e-11 * max(1.0, abs(la0))


def test_log_weight_low_temperature_mpmath():
    """beta = 8 on 4x4: the dense FP64 product is ill-conditioned, so the
    reference determinant is taken in 60-digit arithmetic."""
    lat = W.square_lattice(4)
    par = W.Params(U=4.0, beta=8.0, dtau=0.1, n_stab=10, n_up=3, n_dn=2, seed=1)
    f = W.random_fields(par.L_tau, 16, 2)
    ou, od = W.random_occupation(16, 3, 3), W.random_occupation(16, 2, 4)
    w = oracle.Walker(lat, par, f, ou, od)
    la, sg = w.log_weight()
    mpmath.mp.dps = 60
    E = mpmath.matrix(exact.ek_matrix(lat, par.dtau).tolist())
    lam = exact.hs_lambda(par.U, par.dtau)
    tot, sgn = mpmath.mpf(0), 1
    for sigma, occ in ((1, ou), (-1, od)):
        B = mpmath.eye(16)
        for l in range(par.L_tau):
            D = mpmath.diag([mpmath.e ** (sigma * lam * int(f[l, i])) for i in range(16)])
            B = E * D * B
        sub = mpmath.matrix([[B[int(a), int(b)] for b in occ] for a in occ])
        d = mpmath.det(sub)
        tot += mpmath.log(abs(d))
        sgn *= 1 if d > 0 else -1
    assert sg == sgn
    assert abs(la - float(tot)) < 1e-10 * abs(float(tot))


@pytest.mark.parametrize("name,lat", _lattices())
def test_green_matches_direct_formula(name, lat):
    N = lat.n_sites
    par = W.Params(U=3.0, beta=1.2, dtau=0.1, n_stab=5, n_up=min(3, N - 1), n_dn=2, seed=9)
    f = W.random_fields(par.L_tau, N, 21)
    ou, od = W.random_occupation(N, par.n_up, 22), W.random_occupation(N, par.n_dn, 23)
    w = oracle.Walker(lat, par, f, ou, od)
    for b in (0, 3, 5, 7, par.L_tau):
        for sp, sigma, occ in ((0, 1, ou), (1, -1, od)):
            G = w.green(b, sp)
            G0 = exact.green_direct(lat, par, f, occ, sigma, b)
            assert np.max(np.abs(G - G0)) < 1e-11
            # A = I - G is an idempotent projector of trace Ne
            A = np.eye(N) - G
            assert np.max(np.abs(A @ A - A)) < 1e-10
            assert abs(np.trace(A) - len(occ)) < 1e-10


@pytest.mark.parametrize("name,lat", _lattices())
def test_flip_ratio_matches_weight_ratio(name, lat):
    N = lat.n_sites
    par = W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=min(2, N), seed=5)
    f = W.random_fields(par.L_tau, N, 31)
    ou, od = W.random_occupation(N, 2, 32), W.random_occupation(N, par.n_dn, 33)
    w = oracle.Walker(lat, par, f, ou, od)
    la0, sg0 = exact.log_weight_direct(lat, par, f, ou, od)
    rng = np.random.default_rng(0)
    for _ in range(6):
        l, i = int(rng.integers(par.L_tau)), int(rng.integers(N))
        f2 = f.copy()
        f2[l, i] = -f2[l, i]
        la1, sg1 = exact.log_weight_direct(lat, par, f2, ou, od)
        r0 = sg0 * sg1 * np.exp(la1 - la0)
        r = w.flip_ratio(l, i)
        assert abs(r - r0) < 1e-11 * max(1.0, abs(r0))


def _swap_cases():
    return [
        (W.square_lattice(4), W.Params(U=4.0, beta=2.0, dtau=0.1, n_stab=5, n_up=3, n_dn=2, seed=1)),
        (W.periodic_chain(8), W.Params(U=2.0, beta=1.5, dtau=0.05, n_stab=7, n_up=4, n_dn=1, seed=2)),
        (W.flat_band_chain(4), W.Params(U=2.0, beta=1.0, dtau=0.05, n_stab=6, n_up=3, n_dn=3, seed=3)),
    ]


@pytest.mark.parametrize("case", range(3))
def test_swap_ratio_matches_determinant_ratio(case):
    """Removal by permutation + Givens, addition by layer-wise CGS2 (SM Sec. I):
    the ratio equals det[P'^T B P'] / det[P^T B P] computed densely."""
    lat, par = _swap_cases()[case]
    N = lat.n_sites
    f = W.random_fields(par.L_tau, N, 40 + case)
    ou, od = W.random_occupation(N, par.n_up, 50 + case), W.random_occupation(N, par.n_dn, 60 + case)
    w = oracle.Walker(lat, par, f, ou, od)
    la0, sg0 = exact.log_weight_direct(lat, par, f, ou, od)
    rng = np.random.default_rng(case)
    for sp, occ in ((0, ou), (1, od)):
        for _ in range(4):
            k = int(rng.integers(len(occ)))
            empty = [s for s in range(N) if s not in occ]
            j = int(rng.choice(empty))
            new = np.array([o for t, o in enumerate(occ) if t != k] + [j], dtype=np.int32)
            args = (f, new, od) if sp == 0 else (f, ou, new)
            la1, sg1 = exact.log_weight_direct(lat, par, *args)
            r0 = sg0 * sg1 * np.exp(la1 - la0)
            r = w.swap_ratio(sp, k, j)
            assert abs(r - r0) < 1e-10 * max(1.0, abs(r0)), (sp, k, j, r, r0)


@pytest.mark.parametrize("case", range(3))
def test_swap_commit_keeps_stack_exact(case):
    """After committed swaps the stack still satisfies B_i Q_{i-1} = Q_i V_i with
    Q^T Q = I, V upper triangular with non-negative diagonal, and the stored
    inverse equals (P^T Q_n)^{-1}; the tracked weight equals the fresh one."""
    lat, par = _swap_cases()[case]
    N = lat.n_sites
    f = W.random_fields(par.L_tau, N, 70 + case)
    w = oracle.Walker(lat, par, f)
    rng = np.random.default_rng(10 + case)
    for step in range(5):
        _, ou, od, _ = w.state()
        sp = step % 2
        occ = ou if sp == 0 else od
        k = int(rng.integers(len(occ)))
        j = int(rng.choice([s for s in range(N) if s not in occ]))
        w.swap_commit(sp, k, j)
    _, ou, od, _ = w.state()
    nb = w.n_blocks()
    for sp, sigma, occ in ((0, 1, ou), (1, -1, od)):
        m = len(occ)
        Qprev = np.zeros((N, m))
        Qprev[occ, np.arange(m)] = 1.0
        for i in range(nb):
            Q, V = w.right_stack(sp, i)
            l0, l1 = i * par.n_stab, min((i + 1) * par.n_stab, par.L_tau)
            Bi = exact.b_product(lat, par, f, sigma, l0, l1)
            lhs = Bi @ Qprev
            assert np.max(np.abs(lhs - Q @ V)) < 1e-11 * max(1.0, np.abs(lhs).max())
            assert np.max(np.abs(Q.T @ Q - np.eye(m))) < 1e-12
            assert np.max(np.abs(np.tril(V, -1))) == 0.0
            assert np.all(np.diag(V) >= 0.0)
            Qprev = Q
        Mi = w.inverse(sp)
        assert np.max(np.abs(Mi @ Qprev[occ, :] - np.eye(m))) < 1e-10
    la_t, sg_t = w.tracked_weight()
    la_f, sg_f = exact.log_weight_direct(lat, par, f, ou, od)
    assert sg_t == sg_f and abs(la_t - la_f) < 1e-9 * max(1, abs(la_f))


def test_sweep_bookkeeping_matches_fresh_recompute():
    """Sherman-Morrison bookkeeping over whole sweeps: the tracked log-weight
    equals the fresh one and the wrapped A agrees with the recomputed one."""
    lat, par = W.config_small(U=4.0, seed=4)
    w = oracle.Walker(lat, par)
    w.sweep(10)
    st = w.stats()
    assert st["flip_attempts"] == 10 * 16 * 40
    assert st["logw_drift"] < 1e-8
    assert st["max_wrap_err"] < 1e-8
    f, ou, od, sc = w.state()
    assert sc == 10
    la, sg = w.tracked_weight()
    la0, sg0 = exact.log_weight_direct(lat, par, f, ou, od)
    assert sg == sg0 and abs(la - la0) < 1e-8 * max(1, abs(la0))
    # occupation lists remain valid sets
    assert len(set(ou)) == 2 and len(set(od)) == 2


def test_exhaustive_sum_equals_trotter_trace():
    """Sum over all (eta, s) of det[P^T B P] (main text Eq. (1)) equals the
    Trotter-exact canonical trace times the Ising constant 2^{N L} e^{beta U Ne / 2}."""
    lat = W.open_chain(2)
    par = W.Params(U=3.0, beta=0.8, dtau=0.1, n_stab=4, n_up=1, n_dn=1)
    N, L = 2, par.L_tau
    tot = 0.0
    import itertools
    for bits in itertools.product((1, -1), repeat=N * L):
        f = np.array(bits, dtype=np.int8).reshape(L, N)
        Bu = exact.b_product(lat, par, f, 1)
        Bd = exact.b_product(lat, par, f, -1)
        tot += np.trace(Bu) * np.trace(Bd)        # sum over eta of 1x1 minors
    ed = exact.SectorED(lat, par)
    ref = ed.Z * 2.0 ** (N * L) * np.exp(par.beta * par.U * 2 / 2)
    assert abs(tot - ref) < 1e-10 * ref
    # and the oracle's weight of a few of those configurations
    rng = np.random.default_rng(1)
    for _ in range(5):
        f = np.where(rng.random((L, N)) < 0.5, 1, -1).astype(np.int8)
        occ_u, occ_d = [int(rng.integers(2))], [int(rng.integers(2))]
        w = oracle.Walker(lat, par, f, occ_u, occ_d)
        la, sg = w.log_weight()
        la0, sg0 = exact.log_weight_direct(lat, par, f, occ_u, occ_d)
        assert sg == sg0 and abs(la - la0) < 1e-12 * max(1, abs(la0))


def test_free_fermion_canonical_sum():
    """U = 0: sum over eta of det[P^T B P] = e_Ne(eigenvalues of B) (sum of principal minors)."""
    lat = W.square_lattice(4)
    par = W.Params(U=0.0, beta=2.0, dtau=0.1, n_stab=5, n_up=2, n_dn=0)
    f = np.ones((par.L_tau, 16), dtype=np.int8)
    B = exact.b_product(lat, par, f, 1)
    ev = np.linalg.eigvals(B).real
    e2 = exact.elementary_symmetric(ev, 2)
    import itertools
    tot = 0.0
    for occ in itertools.combinations(range(16), 2):
        w = oracle.Walker(lat, par, f, list(occ), [])
        la, sg = w.log_weight()
        tot += sg * np.exp(la)
    assert abs(tot - e2) < 1e-10 * e2


def _run_bins(w, nbins, per_bin, warm):
    w.sweep(warm)
    w.reset_measure()
    bins = []
    for _ in range(nbins):
        w.sweep(per_bin, measure=True)
        bins.append(w.measure())
        w.reset_measure()
    return np.array(bins)


def _check(bins, idx, ref, nsig=4.0, abs_floor=1e-12):
    est, err = exact.jackknife_ratio(bins[:, idx], bins[:, 0])
    assert abs(est - ref) <= nsig * err + abs_floor, (idx, est, err, ref)
    return est, err


def test_mc_free_fermions_against_closed_form():
    """U = 0 on the 4x4 torus, 2 up + 1 down: the Fock-state moves alone
    sample eta; energies and correlations match the canonical ED."""
    lat = W.square_lattice(4)
    par = W.Params(U=0.0, beta=2.0, dtau=0.1, n_stab=5, n_up=2, n_dn=1, seed=12)
    w = oracle.Walker(lat, par)
    bins = _run_bins(w, 30, 40, 20)
    ed = exact.SectorED(lat, par)
    _check(bins, 3, ed.ekin_per_site())
    _check(bins, 2, ed.docc_per_site())
    assert w.stats()["swap_accepts"] > 0


def test_mc_hubbard_against_trotter_ed():
    """U = 4 on a 6-site ring, 2 up + 2 down: estimators vs Trotter-exact ED."""
    lat = W.periodic_chain(6)
    par = W.Params(U=4.0, beta=2.0, dtau=0.1, n_stab=5, n_up=2, n_dn=2, seed=8)
    w = oracle.Walker(lat, par)
    bins = _run_bins(w, 30, 60, 30)
    ed = exact.SectorED(lat, par)
    _check(bins, 3, ed.ekin_per_site())
    _check(bins, 2, ed.docc_per_site())
    N = 6
    off_ss = 8 + 2 * 1 * 1
    for (i, j) in ((0, 0), (0, 1), (0, 3)):
        ref = ed.szz(i, j) + ed.spsm(i, j)
        _check(bins, off_ss + i * N + j, ref)
        _check(bins, off_ss + N * N + i * N + j, ed.nn(i, j))
    # S_par(q=0) = (1/L) sum_ij <SxSx + SySy> (main text, definition beside
    # Fig. 4(a)): the total [4] and its one-sublattice block [8 + ns^2]
    spar = ed.transverse_sum(range(N), range(N)) / N
    assert spar > 0.05   # far from zero, so a wrong normalisation shows
    _check(bins, 4, spar)
    _check(bins, 8 + 1, spar)


def test_mc_ed_benchmark_point_short():
    """The SM's ED benchmark geometry (4x4, 1 up + 1 down, U = 2) at a
    shortened beta = 2 so that the CPU suite stays fast."""
    lat = W.square_lattice(4)
    par = W.Params(U=2.0, beta=2.0, dtau=0.05, n_stab=10, n_up=1, n_dn=1, seed=2)
    w = oracle.Walker(lat, par)
    bins = _run_bins(w, 24, 40, 20)
    ed = exact.SectorED(lat, par)
    _check(bins, 3, ed.ekin_per_site())
    N = 16
    off_ss = 8 + 2 * 2 * 2
    for j in (0, 1, 5):
        _check(bins, off_ss + j, ed.szz(0, j) + ed.spsm(0, j))
        _check(bins, off_ss + N * N + j, ed.nn(0, j))


# ---------------------------------------------------------------------------
# flat-band chain (SM Secs. III-V)
# ---------------------------------------------------------------------------

def test_flat_band_spectrum():
    """H_eff(k) = S S^dag has a flat zero band and lambda_2 = |S1|^2 + |S2|^2."""
    t1, t2, t3, t4 = -0.2, 1.0, 1.0, -0.2
    Lc = 8
    lat = W.flat_band_chain(Lc, t1, t2, t3, t4)
    ev = np.sort(np.linalg.eigvalsh(exact.hopping_matrix(lat)))
    k = 2 * np.pi * np.arange(Lc) / Lc
    lam2 = np.abs(t1 + t2 * np.exp(-1j * k)) ** 2 + np.abs(t3 + t4 * np.exp(-1j * k)) ** 2
    assert np.max(np.abs(ev[:Lc])) < 1e-12
    assert np.max(np.abs(ev[Lc:] - np.sort(lam2))) < 1e-12
    # Wannier overlap <W_R|W_{R+1}> = t1 t2 + t3 t4 (connectivity condition)
    assert abs((t1 * t2 + t3 * t4) - (-0.4)) < 1e-15


def _flat_gs_sz(Lc, t1, t2, t3, t4, nup, ndn):
    import itertools
    lat = W.flat_band_chain(Lc, t1, t2, t3, t4)
    H1 = exact.hopping_matrix(lat)
    N = lat.n_sites
    bu, bd = exact.sector_basis(N, nup), exact.sector_basis(N, ndn)
    # many-body H in the sector from one-body hopping + U n n
    U = 2.0
    par = W.Params(U=U, beta=1.0, dtau=1.0, n_stab=1, n_up=nup, n_dn=ndn)
    ed = exact.SectorED.__new__(exact.SectorED)
    ed.N, ed.lat, ed.bu, ed.bd = N, lat, bu, bd
    D = len(bu) * len(bd)
    H = np.zeros((D, D))
    for i in range(N):
        for j in range(N):
            if H1[i, j] != 0.0:
                H += H1[i, j] * (ed.hop_matrix_element(0, i, j) + ed.hop_matrix_element(1, i, j))
    nu = np.repeat(np.array([[1.0 if s in b else 0.0 for s in range(N)] for b in bu]), len(bd), axis=0)
    nd = np.tile(np.array([[1.0 if s in b else 0.0 for s in range(N)] for b in bd]), (len(bu), 1))
    H += np.diag(U * (nu * nd).sum(axis=1))
    e, v = np.linalg.eigh(H)
    g = v[:, 0]
    sz = 0.5 * (nu - nd)
    szA = sz[:, 0::2].sum(axis=1)
    szB = sz[:, 1::2].sum(axis=1)
    return e, float(g @ (szA ** 2 * g)), float(g @ (szB ** 2 * g)), float(g @ (szA * szB * g))


def test_flat_band_sublattice_fluctuation_one_sixteenth():
    """Unique ferromagnetic ground state at nu = 1, S^z_tot = 0:
    <(S^z_A1)^2>/L = 1/16 and S11 = S22 = -S12 (eq. SzA with p(k) = 1/2)."""
    Lc = 4
    e, a, b, ab = _flat_gs_sz(Lc, -0.2, 1.0, 1.0, -0.2, 2, 2)
    assert abs(e[0]) < 1e-10 and e[1] - e[0] > 1e-6   # unique ground state at E = 0
    assert abs(a / Lc - 1 / 16) < 1e-10
    assert abs(b / Lc - 1 / 16) < 1e-10
    assert abs(ab / Lc + 1 / 16) < 1e-10


def test_flat_band_general_formula_eq_SzA():
    """eq. SzA for generic hoppings (p(k) not constant) against ED."""
    t1, t2, t3, t4 = 0.3, 1.0, 0.8, -0.5
    Lc = 4
    e, a, _, _ = _flat_gs_sz(Lc, t1, t2, t3, t4, 2, 2)
    k = 2 * np.pi * np.arange(Lc) / Lc
    S1 = t1 + t2 * np.exp(-1j * k)
    S2 = t3 + t4 * np.exp(-1j * k)
    # weight of the flat-band state on A1 is |S2|^2 / (|S1|^2 + |S2|^2) (psi_A1 = S2*)
    p = np.abs(S2) ** 2 / (np.abs(S1) ** 2 + np.abs(S2) ** 2)
    Ne = Lc
    P1, P2 = p.sum(), (p ** 2).sum()
    ref = ((Ne - 1) * P1 - P1 ** 2 + P2) / (4 * (Ne - 1))
    assert abs(a - ref) < 1e-9


def test_mc_flat_band_against_trotter_ed():
    """Oracle sampler on the 4-cell flat-band chain (five colours, onsite
    energies in D) against the Trotter-exact sublattice spin correlations."""
    lat = W.flat_band_chain(4, -0.2, 1.0, 1.0, -0.2)
    par = W.Params(U=2.0, beta=2.0, dtau=0.1, n_stab=5, n_up=2, n_dn=2, seed=4)
    w = oracle.Walker(lat, par)
    bins = _run_bins(w, 24, 50, 20)
    ed = exact.SectorED(lat, par)
    sz = 0.5 * (ed.n_up_site - ed.n_dn_site)
    szA, szB = sz[:, 0::2].sum(axis=1), sz[:, 1::2].sum(axis=1)
    ref11 = ed.avg_diag(szA * szA) / 4
    ref12 = ed.avg_diag(szA * szB) / 4
    _check(bins, 8 + 0, ref11)
    _check(bins, 8 + 1, ref12)
    _check(bins, 3, ed.ekin_per_site())
    # sublattice-resolved S_par(q=0)_ab = (1/L_c) sum_{i in a, j in b}
    # <SxSx + SySy> and its total (L_c = 4 cells)
    sub = [list(range(0, 8, 2)), list(range(1, 8, 2))]
    for a in range(2):
        for b in range(2):
            _check(bins, 8 + 4 + 2 * a + b, ed.transverse_sum(sub[a], sub[b]) / 4)
    _check(bins, 4, ed.transverse_sum(range(8), range(8)) / 4)
    # S^z_tot = 0 sector: sum_ab S^zz_ab(q=0) vanishes configuration by configuration
    tot = bins[:, 8:12].sum(axis=1)
    assert np.max(np.abs(tot)) < 1e-9


def test_ed_transverse_sum_one_electron():
    """The ED transverse sum itself: one up electron has S = S^z = 1/2, so
    <S_x^2 + S_y^2> = S(S+1) - (S^z)^2 = 1/2 at any temperature."""
    lat = W.periodic_chain(6)
    par = W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=5, n_up=1, n_dn=0)
    ed = exact.SectorED(lat, par)
    assert abs(ed.transverse_sum(range(6), range(6)) - 0.5) < 1e-12


def test_szz_total_sum_rule_with_imbalance():
    """S^z_tot = (N_up - N_dn)/2 = M in every configuration, so the total
    S^zz(q=0) = (1/L_c) <(S^z_tot)^2> and the sum of its sublattice blocks are
    M^2 / L_c per sample (Fig. 4 caption, sum rule); S_par(q=0) against ED."""
    lat = W.flat_band_chain(4, -0.2, 1.0, 1.0, -0.2)
    par = W.Params(U=2.0, beta=1.0, dtau=0.1, n_stab=5, n_up=3, n_dn=1, seed=6)
    w = oracle.Walker(lat, par)
    bins = _run_bins(w, 16, 30, 10)
    M, Lc = 1.0, 4
    for b in bins:
        assert abs(b[5] - b[0] * M * M / Lc) < 1e-9 * max(1.0, abs(b[0]))
        assert abs(b[8:12].sum() - b[0] * M * M / Lc) < 1e-9 * max(1.0, abs(b[0]))
    ed = exact.SectorED(lat, par)
    _check(bins, 4, ed.transverse_sum(range(8), range(8)) / Lc)
