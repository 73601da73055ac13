"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every entry point declared in include/lecqmc.h, and its host-only logic
(input validation, device-footprint plan) behaves as documented."""
import os
import re

import numpy as np
import pytest

from paper_2601_08552_amd import lecqmc
from paper_2601_08552_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lecqmc.h")).read()
    return sorted(set(re.findall(r"\b(lecqmc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = lecqmc.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(lecqmc.EXPORTED) == names


def test_footprint_plan_scales_with_stacks():
    lat, par = W.config_dilute()
    fb = lecqmc.footprint_bytes(lat, par)
    nblk, L = 32, 320
    # per spin: left states at boundaries (n+1) and at every slice (L), right stack (n)
    stacks = 2 * (2 * nblk + 1 + L) * 1024 * 8 * 8
    assert stacks < fb < stacks * 1.3


def test_mixed_footprint_halves_the_stored_left_states():
    """Mixed precision stores the per-slice left states in FP32: the plan
    shrinks by L_tau * N * Ne * 4 bytes per spin and nothing else."""
    lat, par = W.config_dilute()
    mix = W.config_dilute(precision=lecqmc.MIXED)[1]
    fb, fm = lecqmc.footprint_bytes(lat, par), lecqmc.footprint_bytes(lat, mix)
    saved = 2 * 320 * 1024 * 8 * 4
    assert abs((fb - fm) - saved) <= 2 * 256


@pytest.mark.parametrize("bad", [
    dict(dtau=0.35),          # beta / dtau not integral
    dict(n_stab=0),
    dict(n_up=17),            # more particles than sites
    dict(n_up=-1),
    dict(U=-1.0),
    dict(precision=3),
])
def test_footprint_rejects_invalid_input(bad):
    lat = W.square_lattice(4)
    kw = dict(U=4.0, beta=1.2, dtau=0.1, n_stab=4, n_up=2, n_dn=2)
    kw.update(bad)
    assert lecqmc.footprint_bytes(lat, W.Params(**kw)) == 0
    assert lecqmc.footprint_bytes(lat, W.Params(U=4.0, beta=1.2, dtau=0.1, n_stab=4, n_up=2, n_dn=2)) > 0


def test_footprint_rejects_overlapping_colour():
    lat = W.square_lattice(4)
    lat.bond_color = lat.bond_color.copy()
    lat.bond_color[1] = lat.bond_color[0]     # (0,1) and (1,2) share site 1
    assert lecqmc.footprint_bytes(lat, W.Params(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=2)) == 0
