"""Thin ctypes binding of the C ABI in include/lecqmc.h.

Argument marshalling only: every step of the method runs in the gfx950
kernels of liblecqmc.so.  There is no CPU fallback; loading fails loudly when
the library has not been built.  torch is used (optionally) only to hand the
library a HIP stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblecqmc.so")

OK, EINVAL, ENOMEM, EUNSTABLE, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
FP64 = 0
MIXED = 1
NO_FOCK = 1
NO_FLIPS = 2
MAX_NE = 256

EXPORTED = [
    "lecqmc_ctx_create", "lecqmc_ctx_destroy", "lecqmc_ctx_synchronize", "lecqmc_ctx_bytes_in_use",
    "lecqmc_ctx_set_timing", "lecqmc_ctx_phase_times",
    "lecqmc_footprint_bytes", "lecqmc_create_walker", "lecqmc_destroy_walker", "lecqmc_sweep",
    "lecqmc_sweep_batch", "lecqmc_log_weight", "lecqmc_tracked_weight", "lecqmc_obs_size",
    "lecqmc_measure", "lecqmc_reset_measure", "lecqmc_get_stats", "lecqmc_get_state",
    "lecqmc_set_state", "lecqmc_green", "lecqmc_flip_ratio", "lecqmc_swap_ratio", "lecqmc_last_error",
    "lecqmc_batch_create", "lecqmc_batch_sweep", "lecqmc_batch_destroy",
    "lecqmc_get_shape", "lecqmc_set_shape", "lecqmc_autotune", "lecqmc_ctx_query",
    "lecqmc_sweep_batch_static",
    "lecqmc_cp_create", "lecqmc_cp_run", "lecqmc_cp_walker", "lecqmc_cp_stats", "lecqmc_cp_destroy",
]
CP_IMPORTANCE = 0
CP_FREE = 1
STATIC_MAX_WALKERS = 1024


class LecqmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lecqmc error {code}: {msg}")
        self.code = code


class _Lattice(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("n_bonds", C.c_int32), ("n_colors", C.c_int32),
                ("bond_i", C.c_void_p), ("bond_j", C.c_void_p), ("bond_color", C.c_void_p),
                ("bond_h", C.c_void_p), ("onsite", C.c_void_p), ("sublattice", C.c_void_p),
                ("n_sublattices", C.c_int32), ("n_cells", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("U", C.c_double), ("beta", C.c_double), ("dtau", C.c_double),
                ("n_stab", C.c_int32), ("n_up", C.c_int32), ("n_dn", C.c_int32),
                ("seed", C.c_uint64), ("walker_id", C.c_uint64), ("precision", C.c_int32),
                ("flags", C.c_int32), ("wrap_tol", C.c_double)]


class SweepStats(C.Structure):
    _fields_ = [("flip_attempts", C.c_int64), ("flip_accepts", C.c_int64),
                ("swap_attempts", C.c_int64), ("swap_accepts", C.c_int64),
                ("max_wrap_err", C.c_double), ("logw_drift", C.c_double),
                ("qr_shifted", C.c_int64), ("sweeps", C.c_uint64), ("near_ties", C.c_int64)]


_lib = None
_live_walkers: "weakref.WeakSet" = weakref.WeakSet()
_live_batches: "weakref.WeakSet" = weakref.WeakSet()
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()
_live_cps: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _release_all():
    """Free device state while the HIP runtime is still up (batches, then
    walkers, then contexts)."""
    for b in list(_live_batches):
        b.close()
    for cp in list(_live_cps):
        cp.close()
    for w in list(_live_walkers):
        w.close()
    for c in list(_live_contexts):
        c.close()


def load():
    """Load liblecqmc.so (built by __graft_entry__.build()); raise if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built; run __graft_entry__.build()")
        # One HIP runtime per process: torch ships its own libamdhip64 (soname
        # libamdhip64.so.7, loaded by torch as libamdhip64.so).  Loading torch
        # first lets the dynamic linker bind this library to that copy; the
        # other order would map a second runtime that torch cannot share.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "lecqmc_ctx_create": (C.c_int, [C.c_int, vp, C.c_size_t, C.POINTER(vp)]),
            "lecqmc_ctx_destroy": (C.c_int, [vp]),
            "lecqmc_ctx_synchronize": (C.c_int, [vp]),
            "lecqmc_ctx_query": (C.c_int, [vp]),
            "lecqmc_ctx_bytes_in_use": (C.c_size_t, [vp]),
            "lecqmc_ctx_set_timing": (C.c_int, [vp, i32]),
            "lecqmc_ctx_phase_times": (C.c_int, [vp, vp, vp]),
            "lecqmc_footprint_bytes": (C.c_size_t, [C.POINTER(_Lattice), C.POINTER(_Params)]),
            "lecqmc_create_walker": (C.c_int, [vp, C.POINTER(_Lattice), C.POINTER(_Params), vp, vp, vp, C.POINTER(vp)]),
            "lecqmc_destroy_walker": (C.c_int, [vp]),
            "lecqmc_sweep": (C.c_int, [vp, i32, i32]),
            "lecqmc_sweep_batch": (C.c_int, [C.POINTER(vp), i32, i32, i32]),
            "lecqmc_sweep_batch_static": (C.c_int, [C.POINTER(vp), i32, i32, i32]),
            "lecqmc_log_weight": (C.c_int, [vp, C.POINTER(dbl), C.POINTER(i32)]),
            "lecqmc_tracked_weight": (C.c_int, [vp, C.POINTER(dbl), C.POINTER(i32)]),
            "lecqmc_obs_size": (i64, [vp]),
            "lecqmc_measure": (C.c_int, [vp, vp, i64]),
            "lecqmc_reset_measure": (C.c_int, [vp]),
            "lecqmc_get_stats": (C.c_int, [vp, C.POINTER(SweepStats)]),
            "lecqmc_get_state": (C.c_int, [vp, vp, vp, vp, C.POINTER(C.c_uint64)]),
            "lecqmc_set_state": (C.c_int, [vp, vp, vp, vp, C.c_uint64]),
            "lecqmc_green": (C.c_int, [vp, i32, i32, vp]),
            "lecqmc_flip_ratio": (C.c_int, [vp, i32, i32, C.POINTER(dbl)]),
            "lecqmc_swap_ratio": (C.c_int, [vp, i32, i32, i32, C.POINTER(dbl)]),
            "lecqmc_last_error": (C.c_char_p, []),
            "lecqmc_batch_create": (C.c_int, [C.POINTER(vp), i32, C.POINTER(vp)]),
            "lecqmc_batch_sweep": (C.c_int, [vp, i32, i32]),
            "lecqmc_batch_destroy": (C.c_int, [vp]),
            "lecqmc_get_shape": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32)]),
            "lecqmc_set_shape": (C.c_int, [vp, i32, i32]),
            "lecqmc_autotune": (C.c_int, [C.POINTER(vp), i32, C.POINTER(i32), C.POINTER(i32),
                                          C.POINTER(C.c_double)]),
            "lecqmc_cp_create": (C.c_int, [vp, C.POINTER(_Lattice), C.POINTER(_Params), vp, vp, i32, i32, i32,
                                           C.POINTER(vp)]),
            "lecqmc_cp_run": (C.c_int, [vp, C.c_uint32, C.POINTER(dbl)]),
            "lecqmc_cp_walker": (C.c_int, [vp, i32, C.POINTER(dbl), C.POINTER(dbl), vp]),
            "lecqmc_cp_stats": (C.c_int, [vp, C.POINTER(dbl), C.POINTER(i64), C.POINTER(i32)]),
            "lecqmc_cp_destroy": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise LecqmcError(rc, load().lecqmc_last_error().decode())


def _marshal(lat, par, keep):
    def arr(x, dt):
        if x is None:
            return None
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    sub = arr(lat.sublattice, np.int32)
    L = _Lattice(lat.n_sites, lat.n_bonds, lat.n_colors, arr(lat.bond_i, np.int32),
                 arr(lat.bond_j, np.int32), arr(lat.bond_color, np.int32),
                 arr(lat.bond_h, np.float64), arr(lat.onsite, np.float64), sub,
                 lat.n_sublattices if sub is not None else 1, lat.n_cells)
    P = _Params(par.U, par.beta, par.dtau, par.n_stab, par.n_up, par.n_dn, par.seed,
                par.walker_id, par.precision, par.flags, par.wrap_tol)
    return L, P


def footprint_bytes(lat, par) -> int:
    keep = []
    L, P = _marshal(lat, par, keep)
    return int(load().lecqmc_footprint_bytes(C.byref(L), C.byref(P)))


class Context:
    """Device, HIP stream (borrowed from torch when given) and memory budget."""

    def __init__(self, device=0, stream=None, hbm_budget_bytes=0):
        lib = load()
        h = C.c_void_p()
        s = None
        if stream is not None:
            s = C.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))
        _check(lib.lecqmc_ctx_create(device, s, hbm_budget_bytes, C.byref(h)))
        self.h = h
        self.device = device
        self._walkers = weakref.WeakSet()
        self._batches = weakref.WeakSet()
        self._cps = weakref.WeakSet()
        _live_contexts.add(self)

    def synchronize(self):
        _check(load().lecqmc_ctx_synchronize(self.h))

    def query(self) -> bool:
        """True when the context's stream has no work left (does not block)."""
        rc = load().lecqmc_ctx_query(self.h)
        _check(min(rc, 0))
        return rc == 1

    def set_timing(self, enable=True):
        _check(load().lecqmc_ctx_set_timing(self.h, 1 if enable else 0))

    def phase_times(self):
        """(ms[3], counts[3]) for (left stack, forward pass, Fock phase) since the last call."""
        ms = np.zeros(3)
        cnt = np.zeros(3, dtype=np.int64)
        _check(load().lecqmc_ctx_phase_times(self.h, ms.ctypes.data, cnt.ctypes.data))
        return ms, cnt

    def bytes_in_use(self) -> int:
        return int(load().lecqmc_ctx_bytes_in_use(self.h))

    def close(self):
        """Destroy the context and every walker it still owns."""
        if getattr(self, "h", None):
            for b in list(self._batches):
                b.close()
            for cp in list(self._cps):
                cp.close()
            for w in list(self._walkers):
                w.close()
            _check(load().lecqmc_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Walker:
    """One Markov chain resident on the GPU."""

    def __init__(self, ctx: Context, lat, par, fields=None, occ_up=None, occ_dn=None):
        lib = load()
        keep = []
        self._lat, self._par = _marshal(lat, par, keep)
        f = None if fields is None else np.ascontiguousarray(fields, dtype=np.int8)
        ou = None if occ_up is None else np.ascontiguousarray(occ_up, dtype=np.int32)
        od = None if occ_dn is None else np.ascontiguousarray(occ_dn, dtype=np.int32)
        h = C.c_void_p()
        _check(lib.lecqmc_create_walker(ctx.h, C.byref(self._lat), C.byref(self._par),
                                        None if f is None else f.ctypes.data,
                                        None if ou is None else ou.ctypes.data,
                                        None if od is None else od.ctypes.data, C.byref(h)))
        self.h = h
        self.ctx = ctx
        ctx._walkers.add(self)
        _live_walkers.add(self)
        self.N = lat.n_sites
        self.L = par.L_tau
        self.ne = (par.n_up, par.n_dn)

    def close(self):
        if getattr(self, "h", None):
            if load().lecqmc_destroy_walker(self.h) == 0:
                self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1, measure=False):
        _check(load().lecqmc_sweep(self.h, n, 1 if measure else 0))

    def log_weight(self):
        la, sg = C.c_double(), C.c_int32()
        _check(load().lecqmc_log_weight(self.h, C.byref(la), C.byref(sg)))
        return la.value, sg.value

    def tracked_weight(self):
        la, sg = C.c_double(), C.c_int32()
        _check(load().lecqmc_tracked_weight(self.h, C.byref(la), C.byref(sg)))
        return la.value, sg.value

    def measure(self):
        n = load().lecqmc_obs_size(self.h)
        o = np.zeros(n)
        _check(load().lecqmc_measure(self.h, o.ctypes.data, n))
        return o

    def reset_measure(self):
        _check(load().lecqmc_reset_measure(self.h))

    def stats(self):
        st = SweepStats()
        _check(load().lecqmc_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in SweepStats._fields_}

    def state(self):
        f = np.zeros((self.L, self.N), dtype=np.int8)
        ou = np.zeros(max(self.ne[0], 1), dtype=np.int32)
        od = np.zeros(max(self.ne[1], 1), dtype=np.int32)
        sc = C.c_uint64()
        _check(load().lecqmc_get_state(self.h, f.ctypes.data, ou.ctypes.data, od.ctypes.data, C.byref(sc)))
        return f, ou[: self.ne[0]].copy(), od[: self.ne[1]].copy(), sc.value

    def set_state(self, fields=None, occ_up=None, occ_dn=None, sweep_counter=0):
        f = None if fields is None else np.ascontiguousarray(fields, dtype=np.int8)
        ou = None if occ_up is None else np.ascontiguousarray(occ_up, dtype=np.int32)
        od = None if occ_dn is None else np.ascontiguousarray(occ_dn, dtype=np.int32)
        _check(load().lecqmc_set_state(self.h, None if f is None else f.ctypes.data,
                                       None if ou is None else ou.ctypes.data,
                                       None if od is None else od.ctypes.data, sweep_counter))

    @property
    def shape(self):
        """(tile, chunk) of the flip chain: register tile T (Ne <= 8T) or 0
        for the inverse in LDS, and the sites per staged chunk."""
        t, c = C.c_int32(), C.c_int32()
        _check(load().lecqmc_get_shape(self.h, C.byref(t), C.byref(c)))
        return int(t.value), int(c.value)

    def set_shape(self, tile, chunk):
        _check(load().lecqmc_set_shape(self.h, tile, chunk))

    def green(self, boundary, spin):
        G = np.zeros((self.N, self.N))
        _check(load().lecqmc_green(self.h, boundary, spin, G.ctypes.data))
        return G

    def flip_ratio(self, slice_, site):
        r = C.c_double()
        _check(load().lecqmc_flip_ratio(self.h, slice_, site, C.byref(r)))
        return r.value

    def swap_ratio(self, spin, k, j):
        r = C.c_double()
        _check(load().lecqmc_swap_ratio(self.h, spin, k, j, C.byref(r)))
        return r.value


def autotune(walkers):
    """Time every valid flip-chain shape on these walkers (their chains are
    not advanced); walkers of one (N, Ne_up, Ne_dn, precision) key get the
    shape with the least total time.  Returns [(tile, chunk, ms)] per walker."""
    n = len(walkers)
    arr = (C.c_void_p * n)(*[w.h for w in walkers])
    tl, ch, ms = (C.c_int32 * n)(), (C.c_int32 * n)(), (C.c_double * n)()
    _check(load().lecqmc_autotune(arr, n, tl, ch, ms))
    return [(int(tl[t]), int(ch[t]), float(ms[t])) for t in range(n)]


def sweep_batch(walkers, n_sweeps=1, measure=False):
    arr = (C.c_void_p * len(walkers))(*[w.h for w in walkers])
    _check(load().lecqmc_sweep_batch(arr, len(walkers), n_sweeps, 1 if measure else 0))


def sweep_batch_static(walkers, n_sweeps=1, measure=False):
    """sweep_batch through the entry point that allocates no device memory
    (descriptors staged in the library's fixed per-device array)."""
    arr = (C.c_void_p * len(walkers))(*[w.h for w in walkers])
    _check(load().lecqmc_sweep_batch_static(arr, len(walkers), n_sweeps, 1 if measure else 0))


class Batch:
    """A fixed set of walkers whose sweeps only launch kernels on the
    context's stream (so they may be captured into a HIP graph)."""

    def __init__(self, walkers):
        self.walkers = list(walkers)
        arr = (C.c_void_p * len(self.walkers))(*[w.h for w in self.walkers])
        h = C.c_void_p()
        _check(load().lecqmc_batch_create(arr, len(self.walkers), C.byref(h)))
        self.h = h
        if self.walkers:
            self.walkers[0].ctx._batches.add(self)
        _live_batches.add(self)

    def sweep(self, n_sweeps=1, measure=False):
        _check(load().lecqmc_batch_sweep(self.h, n_sweeps, 1 if measure else 0))

    def close(self):
        if getattr(self, "h", None):
            load().lecqmc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CPWalk:
    """Constrained-path inner walk of one Fock state (lecqmc_cp_*): a
    population of random walkers on the GPU whose weights estimate
    R(eta) = E_s[prod_sigma det(P^T B(s) P)] / W_T(eta) under the phaseless cut."""

    def __init__(self, ctx: Context, lat, par, occ_up, occ_dn, n_walkers, mode=CP_IMPORTANCE, pc_every=0):
        lib = load()
        keep = []
        self._lat, self._par = _marshal(lat, par, keep)
        ou = np.ascontiguousarray(occ_up, dtype=np.int32)
        od = np.ascontiguousarray(occ_dn, dtype=np.int32)
        h = C.c_void_p()
        _check(lib.lecqmc_cp_create(ctx.h, C.byref(self._lat), C.byref(self._par), ou.ctypes.data, od.ctypes.data,
                                    n_walkers, mode, pc_every, C.byref(h)))
        self.h = h
        self.N, self.L, self.nw = lat.n_sites, par.L_tau, n_walkers
        ctx._cps.add(self)
        _live_cps.add(self)

    def run(self, tag=0):
        """One inner walk from Phi = P_eta; returns log of the estimate of R(eta)."""
        lr = C.c_double()
        _check(load().lecqmc_cp_run(self.h, tag, C.byref(lr)))
        return lr.value

    def walker(self, a):
        """(log weight, sum of log p of its draws, field path [L][N]) of slot a."""
        lw, lq = C.c_double(), C.c_double()
        f = np.zeros((self.L, self.N), dtype=np.int8)
        _check(load().lecqmc_cp_walker(self.h, a, C.byref(lw), C.byref(lq), f.ctypes.data))
        return lw.value, lq.value, f

    def stats(self):
        lp, cuts, alive = C.c_double(), C.c_int64(), C.c_int32()
        _check(load().lecqmc_cp_stats(self.h, C.byref(lp), C.byref(cuts), C.byref(alive)))
        return {"log_pc": lp.value, "cuts": cuts.value, "alive": alive.value}

    def close(self):
        if getattr(self, "h", None):
            load().lecqmc_cp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
