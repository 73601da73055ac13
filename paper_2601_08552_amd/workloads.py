"""Seeded synthetic inputs for the canonical-ensemble DQMC hot path.

This module builds lattices (bond lists with a checkerboard colouring) and
run parameters.  It holds none of the method's arithmetic: no exponentials,
no propagators, no determinants.  Both the HIP path and the CPU oracle take
its outputs as plain arrays, so neither depends on the other.

Lattices follow the models of the paper:
  * the 2D square-lattice Hubbard model with nearest-neighbour hopping t
    (main text, "Time scaling" section, Hubbard Hamiltonian);
  * the 1D flat-band effective chain H_eff(k) = S(k) S(k)^dagger with
    S1 = t1 + t2 e^{-ik}, S2 = t3 + t4 e^{-ik} (SM Sec. III, chiral limit).

Conventions (shared interface, restated on each side):
  H = sum_b h_b (c_i^dag c_j + h.c.) + sum_i eps_i n_i + U sum_i n_iu n_id,
  so the usual "-t" hopping has h_b = -t.  Bonds of one colour never share a
  site.  Colours are numbered 0..C-1 in the order of the product
  e^{-dtau K_0} e^{-dtau K_1} ... e^{-dtau K_{C-1}}.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Lattice:
    n_sites: int
    bond_i: np.ndarray       # int32 [n_bonds]
    bond_j: np.ndarray       # int32 [n_bonds]
    bond_color: np.ndarray   # int32 [n_bonds]
    bond_h: np.ndarray       # float64 [n_bonds], hopping matrix element h_ij
    n_colors: int
    onsite: Optional[np.ndarray] = None      # float64 [n_sites] or None
    sublattice: Optional[np.ndarray] = None  # int32 [n_sites] or None
    n_sublattices: int = 1
    n_cells: int = 0
    name: str = ""

    @property
    def n_bonds(self) -> int:
        return int(self.bond_i.shape[0])

    def check(self) -> None:
        """Validate that every colour is a set of site-disjoint bonds."""
        for c in range(self.n_colors):
            sel = self.bond_color == c
            sites = np.concatenate([self.bond_i[sel], self.bond_j[sel]])
            if len(np.unique(sites)) != len(sites):
                raise ValueError(f"colour {c} has a shared site")
        if np.any(self.bond_i == self.bond_j):
            raise ValueError("self bond")


@dataclasses.dataclass
class Params:
    U: float
    beta: float
    dtau: float
    n_stab: int
    n_up: int
    n_dn: int
    seed: int = 1
    walker_id: int = 0
    precision: int = 0      # 0 = all FP64, 1 = mixed (FP32 propagation)
    flags: int = 0
    wrap_tol: float = 0.0   # <= 0: the library's default (1e-8 FP64, 1e-4 mixed)

    @property
    def L_tau(self) -> int:
        return int(round(self.beta / self.dtau))


def _mk(n, bi, bj, bc, bh, ncol, **kw) -> Lattice:
    lat = Lattice(n_sites=n,
                  bond_i=np.ascontiguousarray(bi, dtype=np.int32),
                  bond_j=np.ascontiguousarray(bj, dtype=np.int32),
                  bond_color=np.ascontiguousarray(bc, dtype=np.int32),
                  bond_h=np.ascontiguousarray(bh, dtype=np.float64),
                  n_colors=ncol, **kw)
    lat.check()
    return lat


def square_lattice(L: int, t: float = 1.0) -> Lattice:
    """Periodic L x L square lattice, site index x + L*y.

    Four colours: x-bonds from even x, x-bonds from odd x, y-bonds from even
    y, y-bonds from odd y.  L must be even (and >= 4, so that the periodic
    wrap does not double a bond).  Sublattice = (x + y) mod 2.
    """
    if L % 2 or L < 4:
        raise ValueError("square lattice needs even L >= 4")
    bi, bj, bc = [], [], []
    for y in range(L):
        for x in range(L):
            s = x + L * y
            bi.append(s); bj.append(((x + 1) % L) + L * y); bc.append(0 if x % 2 == 0 else 1)
    for y in range(L):
        for x in range(L):
            s = x + L * y
            bi.append(s); bj.append(x + L * ((y + 1) % L)); bc.append(2 if y % 2 == 0 else 3)
    n = L * L
    sub = np.array([(s % L + s // L) % 2 for s in range(n)], dtype=np.int32)
    return _mk(n, bi, bj, bc, np.full(len(bi), -t), 4,
               sublattice=sub, n_sublattices=2, n_cells=n // 2, name=f"square{L}x{L}")


def open_chain(n: int, t: float = 1.0) -> Lattice:
    """Open chain of n sites: colour 0 = bonds (2m, 2m+1), colour 1 = (2m+1, 2m+2)."""
    bi = list(range(n - 1))
    bj = [i + 1 for i in bi]
    bc = [i % 2 for i in bi]
    return _mk(n, bi, bj, bc, np.full(len(bi), -t), 2 if n > 2 else 1,
               n_cells=n, name=f"chain{n}")


def periodic_chain(n: int, t: float = 1.0) -> Lattice:
    """Periodic chain, n even >= 4; colour 0 = (2m, 2m+1), colour 1 = (2m+1, 2m+2 mod n)."""
    if n % 2 or n < 4:
        raise ValueError("periodic chain needs even n >= 4")
    bi = list(range(n))
    bj = [(i + 1) % n for i in bi]
    bc = [i % 2 for i in bi]
    return _mk(n, bi, bj, bc, np.full(n, -t), 2, n_cells=n, name=f"pchain{n}")


def flat_band_chain(n_cells: int, t1: float = -0.2, t2: float = 1.0,
                    t3: float = 1.0, t4: float = -0.2) -> Lattice:
    """Effective flat-band chain of the chiral-limit BCL model (SM Sec. III).

    Real-space matrix elements of H_eff(k) = S S^dag with S1 = t1 + t2 e^{-ik},
    S2 = t3 + t4 e^{-ik}:
      onsite A1: t1^2 + t2^2, onsite A2: t3^2 + t4^2,
      A1_R - A1_{R+1}: t1 t2,  A2_R - A2_{R+1}: t3 t4,
      A1_R - A2_R (rung): t1 t3 + t2 t4,
      A1_R - A2_{R+1}: t1 t4,  A2_R - A1_{R+1}: t2 t3.
    Site index: A1_R = 2R, A2_R = 2R + 1; periodic, n_cells even >= 4.
    Five colours: legs from even R, legs from odd R, rungs, diagonals from
    even R, diagonals from odd R.
    """
    Lc = n_cells
    if Lc % 2 or Lc < 4:
        raise ValueError("flat-band chain needs even n_cells >= 4")
    A1 = lambda R: 2 * (R % Lc)
    A2 = lambda R: 2 * (R % Lc) + 1
    bi, bj, bc, bh = [], [], [], []
    for R in range(Lc):
        col = 0 if R % 2 == 0 else 1
        bi += [A1(R), A2(R)]; bj += [A1(R + 1), A2(R + 1)]
        bc += [col, col]; bh += [t1 * t2, t3 * t4]
    for R in range(Lc):
        bi.append(A1(R)); bj.append(A2(R)); bc.append(2); bh.append(t1 * t3 + t2 * t4)
    for R in range(Lc):
        col = 3 if R % 2 == 0 else 4
        bi += [A1(R), A2(R)]; bj += [A2(R + 1), A1(R + 1)]
        bc += [col, col]; bh += [t1 * t4, t2 * t3]
    n = 2 * Lc
    onsite = np.array([t1 * t1 + t2 * t2, t3 * t3 + t4 * t4] * Lc, dtype=np.float64)
    sub = np.array([0, 1] * Lc, dtype=np.int32)
    return _mk(n, bi, bj, bc, bh, 5, onsite=onsite, sublattice=sub,
               n_sublattices=2, n_cells=Lc, name=f"flatband{Lc}")


def drop_uniform_onsite(lat: Lattice) -> Lattice:
    """Return a copy without onsite energies when they are uniform.

    A uniform onsite energy only multiplies every canonical weight by the same
    constant, so it may be dropped without changing any expectation value.
    """
    if lat.onsite is None:
        return lat
    if np.ptp(lat.onsite) > 1e-15:
        raise ValueError("onsite energies are not uniform")
    return dataclasses.replace(lat, onsite=None)


# ---------------------------------------------------------------------------
# Configurations of the workloads (synthetic, seeded)
# ---------------------------------------------------------------------------

def config_small(U: float = 4.0, seed: int = 1):
    """4x4 periodic Hubbard, t=1, 2 up + 2 down, beta=4, dtau=0.1 (40 slices), QR every 10."""
    return square_lattice(4), Params(U=U, beta=4.0, dtau=0.1, n_stab=10,
                                     n_up=2, n_dn=2, seed=seed)


def config_dilute(seed: int = 1, walker_id: int = 0, precision: int = 0):
    """32x32 periodic Hubbard (N=1024), U=4, 8 up + 8 down, beta=16, dtau=0.05 (320 slices), QR every 10."""
    return square_lattice(32), Params(U=4.0, beta=16.0, dtau=0.05, n_stab=10,
                                      n_up=8, n_dn=8, seed=seed,
                                      walker_id=walker_id, precision=precision)


def config_ed_benchmark(seed: int = 1):
    """4x4 Hubbard, 1 up + 1 down, U=2, dtau=0.05, T=0.05 (beta=20, 400 slices)."""
    return square_lattice(4), Params(U=2.0, beta=20.0, dtau=0.05, n_stab=10,
                                     n_up=1, n_dn=1, seed=seed)


def config_batched(n_walkers: int = 256, seed: int = 1):
    """Uneven batch: L in {16,24,32,48,64}, Ne per spin in [4,32], U in [2,6], beta in {8,16}."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_walkers):
        L = int(rng.choice([16, 24, 32, 48, 64]))
        ne = int(rng.integers(4, 33))
        U = float(rng.uniform(2.0, 6.0))
        beta = float(rng.choice([8.0, 16.0]))
        out.append((square_lattice(L), Params(U=U, beta=beta, dtau=0.05, n_stab=10,
                                              n_up=ne, n_dn=ne, seed=seed + c, walker_id=c)))
    return out


def config_flat_band(n_cells: int = 256, imbalance: int = 0, beta: float = 10.0,
                     tprime: float = 1.0, seed: int = 1):
    """Flat-band chain with t2=t3=1, t1=t4=tprime, U=2, N_up+N_dn = n_cells (flat band half filled)."""
    lat = drop_uniform_onsite(flat_band_chain(n_cells, t1=tprime, t2=1.0, t3=1.0, t4=tprime))
    ntot = n_cells
    nup = (ntot + imbalance) // 2
    ndn = ntot - nup
    return lat, Params(U=2.0, beta=beta, dtau=0.05, n_stab=10, n_up=nup, n_dn=ndn, seed=seed)


def random_fields(L_tau: int, n: int, seed: int) -> np.ndarray:
    """Seeded +-1 Ising field, int8 [L_tau][n] (numpy PCG64, independent of the method's RNG)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L_tau, n)) < 0.5, 1, -1).astype(np.int8)


def random_occupation(n: int, ne: int, seed: int) -> np.ndarray:
    """Seeded occupied-site list (int32, length ne), in random order."""
    rng = np.random.default_rng(seed)
    return rng.permutation(n)[:ne].astype(np.int32)
