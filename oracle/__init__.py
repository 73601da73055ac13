"""Python access to the FP64 CPU oracle (ctypes).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark may use this module; the product path never
does.  It shares no code with the HIP implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblecqmc_oracle.so")
_SRC = os.path.join(_HERE, "lecqmc_oracle.c")

NO_FOCK = 1
NO_FLIPS = 2
S_FLIP, S_SWAP_K, S_SWAP_J, S_SWAP_ACC, S_INIT_FIELD, S_INIT_OCC = 1, 2, 3, 4, 5, 6
S_CP_FIELD, S_CP_COMB = 7, 8
CP_IMPORTANCE, CP_FREE = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no BLAS, no OpenMP, single thread)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               _SRC, "-o", _SO + ".tmp", "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Lat(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("n_bonds", C.c_int32), ("n_colors", C.c_int32),
                ("bond_i", C.POINTER(C.c_int32)), ("bond_j", C.POINTER(C.c_int32)),
                ("bond_color", C.POINTER(C.c_int32)), ("bond_h", C.POINTER(C.c_double)),
                ("onsite", C.POINTER(C.c_double)), ("sublattice", C.POINTER(C.c_int32)),
                ("n_sublattices", C.c_int32), ("n_cells", C.c_int32)]


class _Par(C.Structure):
    _fields_ = [("U", C.c_double), ("beta", C.c_double), ("dtau", C.c_double),
                ("n_stab", C.c_int32), ("n_up", C.c_int32), ("n_dn", C.c_int32),
                ("seed", C.c_uint64), ("walker_id", C.c_uint64), ("flags", C.c_int32),
                ("wrap_tol", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("flip_attempts", C.c_int64), ("flip_accepts", C.c_int64),
                ("swap_attempts", C.c_int64), ("swap_accepts", C.c_int64),
                ("max_wrap_err", C.c_double), ("logw_drift", C.c_double), ("near_ties", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp = C.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(_Lat), C.POINTER(_Par), vp, vp, vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_last_error.restype = C.c_char_p
        L.orc_sweep.argtypes = [vp, C.c_int32, C.c_int32]
        L.orc_log_weight.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.orc_tracked_weight.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.orc_get_state.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_uint64)]
        L.orc_set_state.argtypes = [vp, vp, vp, vp, C.c_uint64]
        L.orc_green.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.orc_flip_ratio.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
        L.orc_swap_ratio.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
        L.orc_swap_commit.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
        L.orc_right_stack.argtypes = [vp, C.c_int32, C.c_int32, vp, vp]
        L.orc_inverse.argtypes = [vp, C.c_int32, vp]
        L.orc_n_blocks.argtypes = [vp]
        L.orc_obs_size.restype = C.c_int64
        L.orc_obs_size.argtypes = [vp]
        L.orc_measure.argtypes = [vp, vp]
        L.orc_reset_measure.argtypes = [vp]
        L.orc_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_cp_create.restype = vp
        L.orc_cp_create.argtypes = [C.POINTER(_Lat), C.POINTER(_Par), vp, vp, C.c_int32, C.c_int32, C.c_int32]
        L.orc_cp_destroy.argtypes = [vp]
        L.orc_cp_run.argtypes = [vp, C.c_uint32, C.POINTER(C.c_double)]
        L.orc_cp_walker.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
        L.orc_cp_stats.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        _lib = L
    return _lib


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def uniform(seed, walker_id, stream, sweep, a, b) -> float:
    return lib().orc_uniform(seed, walker_id, stream, sweep, a, b)


def _ptr(a):
    return None if a is None else a.ctypes.data


class Walker:
    """One Markov chain of the oracle."""

    def __init__(self, lat, par, fields=None, occ_up=None, occ_dn=None):
        self._keep = []

        def arr(x, dt):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return a

        bi, bj, bc = arr(lat.bond_i, np.int32), arr(lat.bond_j, np.int32), arr(lat.bond_color, np.int32)
        bh, on, sub = arr(lat.bond_h, np.float64), arr(lat.onsite, np.float64), arr(lat.sublattice, np.int32)
        P = lambda a, t: C.cast(a.ctypes.data, C.POINTER(t)) if a is not None else C.POINTER(t)()
        self._lat = _Lat(lat.n_sites, lat.n_bonds, lat.n_colors, P(bi, C.c_int32), P(bj, C.c_int32),
                         P(bc, C.c_int32), P(bh, C.c_double), P(on, C.c_double), P(sub, C.c_int32),
                         lat.n_sublattices if sub is not None else 1, lat.n_cells)
        self._par = _Par(par.U, par.beta, par.dtau, par.n_stab, par.n_up, par.n_dn, par.seed,
                         par.walker_id, par.flags, par.wrap_tol)
        f = arr(fields, np.int8)
        ou = arr(occ_up, np.int32)
        od = arr(occ_dn, np.int32)
        self.N = lat.n_sites
        self.L = par.L_tau
        self.ne = (par.n_up, par.n_dn)
        h = lib().orc_create(C.byref(self._lat), C.byref(self._par), _ptr(f), _ptr(ou), _ptr(od))
        if not h:
            raise ValueError(lib().orc_last_error().decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def _chk(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}: {lib().orc_last_error().decode()}")

    def sweep(self, n=1, measure=False, flags=None):
        if flags is not None:
            raise ValueError("flags are fixed at creation")
        self._chk(lib().orc_sweep(self.h, n, 1 if measure else 0))

    def log_weight(self):
        la, sg = C.c_double(), C.c_int32()
        self._chk(lib().orc_log_weight(self.h, C.byref(la), C.byref(sg)))
        return la.value, sg.value

    def tracked_weight(self):
        la, sg = C.c_double(), C.c_int32()
        self._chk(lib().orc_tracked_weight(self.h, C.byref(la), C.byref(sg)))
        return la.value, sg.value

    def state(self):
        f = np.zeros((self.L, self.N), dtype=np.int8)
        ou = np.zeros(max(self.ne[0], 1), dtype=np.int32)
        od = np.zeros(max(self.ne[1], 1), dtype=np.int32)
        sc = C.c_uint64()
        self._chk(lib().orc_get_state(self.h, f.ctypes.data, ou.ctypes.data, od.ctypes.data, C.byref(sc)))
        return f, ou[:self.ne[0]].copy(), od[:self.ne[1]].copy(), sc.value

    def set_state(self, fields=None, occ_up=None, occ_dn=None, sweep_counter=0):
        f = None if fields is None else np.ascontiguousarray(fields, dtype=np.int8)
        ou = None if occ_up is None else np.ascontiguousarray(occ_up, dtype=np.int32)
        od = None if occ_dn is None else np.ascontiguousarray(occ_dn, dtype=np.int32)
        self._chk(lib().orc_set_state(self.h, _ptr(f), _ptr(ou), _ptr(od), sweep_counter))

    def green(self, boundary, spin):
        G = np.zeros((self.N, self.N))
        self._chk(lib().orc_green(self.h, boundary, spin, G.ctypes.data))
        return G

    def flip_ratio(self, slice_, site):
        r = C.c_double()
        self._chk(lib().orc_flip_ratio(self.h, slice_, site, C.byref(r)))
        return r.value

    def swap_ratio(self, spin, k, j):
        r = C.c_double()
        self._chk(lib().orc_swap_ratio(self.h, spin, k, j, C.byref(r)))
        return r.value

    def swap_commit(self, spin, k, j):
        r = C.c_double()
        rc = lib().orc_swap_commit(self.h, spin, k, j, C.byref(r))
        if rc not in (0, -3):
            self._chk(rc)
        return r.value

    def n_blocks(self):
        return lib().orc_n_blocks(self.h)

    def right_stack(self, spin, level):
        m = self.ne[spin]
        Q = np.zeros((self.N, max(m, 1)))
        V = np.zeros((max(m, 1), max(m, 1)))
        self._chk(lib().orc_right_stack(self.h, spin, level, Q.ctypes.data, V.ctypes.data))
        return Q.ravel()[: self.N * m].reshape(self.N, m).copy(), V.ravel()[: m * m].reshape(m, m).copy()

    def inverse(self, spin):
        m = self.ne[spin]
        Mi = np.zeros(max(m * m, 1))
        self._chk(lib().orc_inverse(self.h, spin, Mi.ctypes.data))
        return Mi[: m * m].reshape(m, m).copy()

    def measure(self):
        n = lib().orc_obs_size(self.h)
        o = np.zeros(n)
        self._chk(lib().orc_measure(self.h, o.ctypes.data))
        return o

    def reset_measure(self):
        self._chk(lib().orc_reset_measure(self.h))

    def stats(self):
        st = Stats()
        self._chk(lib().orc_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}


class CPWalk:
    """Constrained-path inner walk of one Fock state (SM Sec. VI): a
    population of random walkers whose weights estimate R(eta) =
    E_s[prod_sigma det(P^T B(s) P)] / W_T(eta) under the phaseless cut."""

    def __init__(self, lat, par, occ_up, occ_dn, n_walkers, mode=CP_IMPORTANCE, pc_every=0):
        self._w = Walker.__new__(Walker)   # reuse Walker's marshalling of lattice and parameters
        self._keep = []

        def arr(x, dt):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return a

        bi, bj, bc = arr(lat.bond_i, np.int32), arr(lat.bond_j, np.int32), arr(lat.bond_color, np.int32)
        bh, on, sub = arr(lat.bond_h, np.float64), arr(lat.onsite, np.float64), arr(lat.sublattice, np.int32)
        P = lambda a, t: C.cast(a.ctypes.data, C.POINTER(t)) if a is not None else C.POINTER(t)()
        self._lat = _Lat(lat.n_sites, lat.n_bonds, lat.n_colors, P(bi, C.c_int32), P(bj, C.c_int32),
                         P(bc, C.c_int32), P(bh, C.c_double), P(on, C.c_double), P(sub, C.c_int32),
                         lat.n_sublattices if sub is not None else 1, lat.n_cells)
        self._par = _Par(par.U, par.beta, par.dtau, par.n_stab, par.n_up, par.n_dn, par.seed,
                         par.walker_id, par.flags, par.wrap_tol)
        ou, od = arr(occ_up, np.int32), arr(occ_dn, np.int32)
        self.N, self.L, self.nw = lat.n_sites, par.L_tau, n_walkers
        h = lib().orc_cp_create(C.byref(self._lat), C.byref(self._par), _ptr(ou), _ptr(od), n_walkers, mode,
                                pc_every)
        if not h:
            raise ValueError(lib().orc_last_error().decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_cp_destroy(self.h)
            self.h = None

    def run(self, tag=0):
        """One inner walk from Phi = P_eta; returns log of the estimate of R(eta)."""
        lr = C.c_double()
        if lib().orc_cp_run(self.h, tag, C.byref(lr)) != 0:
            raise RuntimeError(lib().orc_last_error().decode())
        return lr.value

    def walker(self, a):
        """(log weight, sum of log p of its draws, field path [L][N]) of slot a."""
        lw, lq = C.c_double(), C.c_double()
        f = np.zeros((self.L, self.N), dtype=np.int8)
        if lib().orc_cp_walker(self.h, a, C.byref(lw), C.byref(lq), f.ctypes.data) != 0:
            raise RuntimeError(lib().orc_last_error().decode())
        return lw.value, lq.value, f

    def stats(self):
        lp, cuts, alive = C.c_double(), C.c_int64(), C.c_int32()
        lib().orc_cp_stats(self.h, C.byref(lp), C.byref(cuts), C.byref(alive))
        return {"log_pc": lp.value, "cuts": cuts.value, "alive": alive.value}


def cp_partition_ratio(lat, par, n_eta, sweeps_between, n_walkers, mode=CP_IMPORTANCE, pc_every=0, burn=5):
    """Two-stage estimate of Z / Z_0 = sum_eta W_T(eta) R(eta) / sum_eta W_T(eta)
    (SM Sec. VI): the outer chain is the LEC-QMC chain at U = 0, whose Fock
    moves sample eta with probability W_T(eta) / Z_0; each sampled eta gets
    one inner walk.  Returns the per-eta estimates of R(eta)."""
    import dataclasses
    p0 = dataclasses.replace(par, U=0.0, flags=NO_FLIPS)
    outer = Walker(lat, p0)
    outer.sweep(burn)
    rs = []
    for t in range(n_eta):
        _, ou, od, _ = outer.state()
        walk = CPWalk(lat, par, ou, od, n_walkers, mode, pc_every)
        rs.append(np.exp(walk.run(tag=t)))
        outer.sweep(sweeps_between)
    return np.array(rs)
