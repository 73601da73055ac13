"""Exact references for the tests: dense single-particle propagators, exact
diagonalisation in a fixed (N_up, N_dn) sector, and free-fermion closed forms.

Everything here is written from the definitions (main text Eq. (1) and the
Hubbard Hamiltonian), independently of the oracle and of the HIP path:

* single-particle propagator of one colour: scipy expm of -dtau K_c built
  bond by bond (not the 2x2 cosh/sinh form the oracle uses);
* many-body transfer matrix of one slice after summing the Ising field:
  T = E_K(many-body) . exp(-dtau U sum_i n_iu n_id) . exp(-dtau sum_i eps_i n_i);
  a one-body exponential acts on the n-particle sector through its n-th
  compound matrix (all n x n minors), which is exact;
* Trotter-exact expectation values <O> = Tr[O T^L] / Tr[T^L].
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sl


def colour_matrices(lat):
    N = lat.n_sites
    Ks = []
    for c in range(lat.n_colors):
        K = np.zeros((N, N))
        for b in range(lat.n_bonds):
            if lat.bond_color[b] == c:
                i, j, h = int(lat.bond_i[b]), int(lat.bond_j[b]), float(lat.bond_h[b])
                K[i, j] += h
                K[j, i] += h
        Ks.append(K)
    return Ks


def hopping_matrix(lat):
    K = sum(colour_matrices(lat)) if lat.n_colors else np.zeros((lat.n_sites, lat.n_sites))
    if lat.onsite is not None:
        K = K + np.diag(lat.onsite)
    return K


def ek_matrix(lat, dtau):
    """E_K = e^{-dtau K_0} e^{-dtau K_1} ... e^{-dtau K_{C-1}} (dense)."""
    E = np.eye(lat.n_sites)
    for K in colour_matrices(lat):
        E = E @ sl.expm(-dtau * K)
    return E


def hs_lambda(U, dtau):
    return np.arccosh(np.exp(dtau * U / 2.0))


def slice_matrix(lat, par, fields_l, sigma):
    """B_l = E_K D_l for spin sigma = +1/-1 and one slice of Ising fields."""
    lam = hs_lambda(par.U, par.dtau)
    eps = lat.onsite if lat.onsite is not None else np.zeros(lat.n_sites)
    d = np.exp(sigma * lam * fields_l.astype(float) - par.dtau * eps)
    return ek_matrix(lat, par.dtau) @ np.diag(d)


def b_product(lat, par, fields, sigma, l_from=0, l_to=None):
    """B_{l_to} ... B_{l_from+1} (slices numbered from 1), dense FP64."""
    if l_to is None:
        l_to = fields.shape[0]
    E = ek_matrix(lat, par.dtau)
    lam = hs_lambda(par.U, par.dtau)
    eps = lat.onsite if lat.onsite is not None else np.zeros(lat.n_sites)
    B = np.eye(lat.n_sites)
    for l in range(l_from, l_to):
        d = np.exp(sigma * lam * fields[l].astype(float) - par.dtau * eps)
        B = E @ (d[:, None] * B)
    return B


def log_weight_direct(lat, par, fields, occ_up, occ_dn):
    """log|W| and sign of W = prod_sigma det(P^T B P) from the dense product."""
    la, sg = 0.0, 1
    for sigma, occ in ((1, occ_up), (-1, occ_dn)):
        if len(occ) == 0:
            continue
        B = b_product(lat, par, fields, sigma)
        s, l = np.linalg.slogdet(B[np.ix_(occ, occ)])
        la += l
        sg *= int(np.sign(s))
    return la, sg


def green_direct(lat, par, fields, occ, sigma, boundary):
    """G = I - B1 P (P^T B2 B1 P)^{-1} P^T B2, B1 = B_b..B_1, B2 = B_L..B_{b+1}."""
    N = lat.n_sites
    B1 = b_product(lat, par, fields, sigma, 0, boundary)
    B2 = b_product(lat, par, fields, sigma, boundary, fields.shape[0])
    P = np.zeros((N, len(occ)))
    P[np.asarray(occ), np.arange(len(occ))] = 1.0
    R = B1 @ P
    Lm = P.T @ B2
    A = R @ np.linalg.solve(Lm @ R, Lm)
    return np.eye(N) - A


# ----------------------------------------------------------------------------
# exact diagonalisation in a particle-number sector
# ----------------------------------------------------------------------------

def sector_basis(N, n):
    return [tuple(c) for c in itertools.combinations(range(N), n)]


def compound(E, basis):
    """n-th compound matrix: <eta'|Gamma(E)|eta> = det E[eta', eta]."""
    n = len(basis[0]) if basis else 0
    D = len(basis)
    C = np.empty((D, D))
    if n == 0:
        return np.ones((1, 1))
    idx = np.array(basis)
    for a in range(D):
        rows = idx[a]
        sub = E[rows][:, idx]              # (n, D, n)
        sub = np.transpose(sub, (1, 0, 2))  # (D, n, n)
        C[a, :] = np.linalg.det(sub)
    return C


class SectorED:
    """Trotter-exact thermal averages in the (n_up, n_dn) sector."""

    def __init__(self, lat, par):
        N = lat.n_sites
        self.N = N
        self.lat = lat
        self.bu = sector_basis(N, par.n_up)
        self.bd = sector_basis(N, par.n_dn)
        E = ek_matrix(lat, par.dtau)
        Cu, Cd = compound(E, self.bu), compound(E, self.bd)
        self.nu = np.array([[1.0 if i in s else 0.0 for i in range(N)] for s in self.bu]).reshape(len(self.bu), N)
        self.nd = np.array([[1.0 if i in s else 0.0 for i in range(N)] for s in self.bd]).reshape(len(self.bd), N)
        eps = lat.onsite if lat.onsite is not None else np.zeros(N)
        nu_full = np.repeat(self.nu, len(self.bd), axis=0)
        nd_full = np.tile(self.nd, (len(self.bu), 1))
        self.n_up_site, self.n_dn_site = nu_full, nd_full   # (D, N)
        dbl = (nu_full * nd_full).sum(axis=1)
        onsite = ((nu_full + nd_full) * eps[None, :]).sum(axis=1)
        diag = np.exp(-par.dtau * par.U * dbl - par.dtau * onsite)
        T = np.kron(Cu, Cd) * diag[None, :]
        self.T = T
        self.TL = np.linalg.matrix_power(T, par.L_tau)
        self.Z = np.trace(self.TL)

    def avg_diag(self, values):
        """<O> for O diagonal in the Fock basis (values per basis state)."""
        return float(np.dot(np.diag(self.TL), values) / self.Z)

    def avg(self, O):
        return float(np.trace(O @ self.TL) / self.Z)

    # --- observables -----------------------------------------------------
    def docc_per_site(self):
        return self.avg_diag((self.n_up_site * self.n_dn_site).sum(axis=1)) / self.N

    def szz(self, i, j):
        sz = 0.5 * (self.n_up_site - self.n_dn_site)
        return self.avg_diag(sz[:, i] * sz[:, j])

    def nn(self, i, j):
        n = self.n_up_site + self.n_dn_site
        return self.avg_diag(n[:, i] * n[:, j])

    def hop_single(self, spin, i, j):
        """c_i^dag c_j of one spin species on that species' own sector basis."""
        basis = self.bu if spin == 0 else self.bd
        D = len(basis)
        index = {s: a for a, s in enumerate(basis)}
        M = np.zeros((D, D))
        for a, s in enumerate(basis):
            if j in s and (i not in s or i == j):
                lst = list(s)
                pj = lst.index(j)
                sgn = (-1) ** pj
                lst.pop(pj)
                if i in lst:
                    continue
                # insert i in order
                pos = sum(1 for x in lst if x < i)
                sgn *= (-1) ** pos
                new = tuple(sorted(lst + [i]))
                M[index[new], a] += sgn
        return M

    def hop_matrix_element(self, spin, i, j):
        """<c_i^dag c_j> for spin 0 (up) / 1 (down) as a Fock-space matrix."""
        M = self.hop_single(spin, i, j)
        if spin == 0:
            return np.kron(M, np.eye(len(self.bd)))
        return np.kron(np.eye(len(self.bu)), M)

    def avg_kron(self, Pu, Qd):
        """<O> for O = Pu (x) Qd (up factor, down factor) without forming O."""
        Du, Dd = len(self.bu), len(self.bd)
        TL4 = self.TL.reshape(Du, Dd, Du, Dd)
        return float(np.einsum("ac,bd,cdab->", Pu, Qd, TL4) / self.Z)

    def transverse_sum(self, rows, cols):
        """sum over i in rows, j in cols of <S^x_i S^x_j + S^y_i S^y_j>
        = (1/2) <S+_i S-_j + S-_i S+_j>, with the spin-flip products written
        per species: S+_i S-_j = (c_iu^dag c_ju) (x) (delta_ij - c_jd^dag c_id)
        and S-_i S+_j = (delta_ij - c_ju^dag c_iu) (x) (c_id^dag c_jd)."""
        Iu, Id = np.eye(len(self.bu)), np.eye(len(self.bd))
        tot = 0.0
        for i in rows:
            for j in cols:
                d = 1.0 if i == j else 0.0
                pm = self.avg_kron(self.hop_single(0, i, j), d * Id - self.hop_single(1, j, i))
                mp = self.avg_kron(d * Iu - self.hop_single(0, j, i), self.hop_single(1, i, j))
                tot += 0.5 * (pm + mp)
        return tot

    def ekin_per_site(self):
        tot = 0.0
        lat = self.lat
        for b in range(lat.n_bonds):
            i, j, h = int(lat.bond_i[b]), int(lat.bond_j[b]), float(lat.bond_h[b])
            for sp in (0, 1):
                tot += h * (self.avg(self.hop_matrix_element(sp, i, j)) + self.avg(self.hop_matrix_element(sp, j, i)))
        return tot / self.N

    def spsm(self, i, j):
        """<S+_i S-_j + S-_i S+_j>/2 via the transverse correlation."""
        # S+_i S-_j = c_iu^dag c_id c_jd^dag c_ju ; build from one-body pieces
        upij = self.hop_matrix_element(0, i, j)   # c_iu^dag c_ju
        dnji = self.hop_matrix_element(1, j, i)   # c_jd^dag c_id
        # c_iu^dag c_id c_jd^dag c_ju = c_iu^dag c_ju c_id c_jd^dag (spin operators anticommute: two swaps)
        # and c_id c_jd^dag = delta_ij - c_jd^dag c_id
        Dd = len(self.bd)
        Du = len(self.bu)
        I = np.eye(Du * Dd)
        pm = upij @ ((1.0 if i == j else 0.0) * I - dnji)
        dnij = self.hop_matrix_element(1, i, j)
        upji = self.hop_matrix_element(0, j, i)
        mp = dnij @ ((1.0 if i == j else 0.0) * I - upji)
        return 0.5 * (self.avg(pm) + self.avg(mp))


def elementary_symmetric(vals, n):
    """e_n of the values (recursive product expansion)."""
    e = np.zeros(n + 1)
    e[0] = 1.0
    for v in vals:
        for k in range(n, 0, -1):
            e[k] += v * e[k - 1]
    return e[n]


def jackknife_ratio(num_bins, den_bins):
    """Mean and error of sum(num)/sum(den) by jackknife over bins."""
    num_bins = np.asarray(num_bins, float)
    den_bins = np.asarray(den_bins, float)
    nb = len(num_bins)
    tot_n, tot_d = num_bins.sum(axis=0), den_bins.sum()
    est = tot_n / tot_d
    jk = np.array([(tot_n - num_bins[b]) / (tot_d - den_bins[b]) for b in range(nb)])
    err = np.sqrt((nb - 1) / nb * ((jk - jk.mean(axis=0)) ** 2).sum(axis=0))
    return est, err
