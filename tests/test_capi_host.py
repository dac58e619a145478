"""Host-side checks of the C ABI that need no GPU.

The shared library must load, export every entry point that include/ssrpa.h
declares, and reject bad descriptions on the host (validation, the
alias-free grid bound, footprint and valence-block planning) without
touching a device.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from synth import systems as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2405_20258_amd import ssrpa
    return ssrpa


def declared_symbols():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"SSRPA_API[^;(]*?\b(ssrpa_\w+)\s*\(", text,
                                re.S)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert len(names) >= 20
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), f"{n} declared but not exported"
        assert n in lib.EXPORTED, f"{n} has no binding"


def test_status_strings(lib):
    for s in range(7):
        assert len(lib.ssrpa_status_string(s)) > 0
    assert lib.ssrpa_version().decode().endswith("gfx950")


def test_frequency_grid_matches_legendre(lib):
    for n in (1, 2, 16, 20, 64):
        om, wt = lib.frequency_grid(n, 1.0)
        ref_om, ref_wt = sy.frequency_grid(n)
        # near x -> 1 the map amplifies the rounding of the nodes
        assert np.allclose(om, ref_om, rtol=1e-12, atol=0)
        assert np.allclose(wt, ref_wt, rtol=1e-11, atol=0)
    om, wt = lib.frequency_grid(64, 2.0)
    assert abs(np.dot(wt, 1.0 / (4.0 + om ** 2)) - math.pi / 4) < 1e-12


def _desc(lib, s, fft=None, keep=None):
    keep = [] if keep is None else keep
    return lib.make_desc(s.a, fft or s.fft, s.miller, s.coeff, s.energy,
                         s.n_v, s.ecut_chi, keep), keep


def test_footprint_and_alias_bound(lib):
    s = sy.make_system(sy.TINY, 1000)
    d, keep = _desc(lib, s)
    b = ctypes.c_size_t()
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 0,
                               ctypes.byref(b)) == lib.OK
    full = b.value
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 4,
                               ctypes.byref(b)) == lib.OK
    assert b.value < full
    # one below the alias-free bound 2*7 + 4 + 1 = 19 (18 = 2 * 3^2)
    d2, keep2 = _desc(lib, s, fft=(18, 18, 18))
    assert lib.ssrpa_footprint(ctypes.byref(d2), 75, 16, lib.FP64, 0,
                               ctypes.byref(b)) == lib.ERR_ALIAS
    # grid size that is not 2^i 3^j
    d3, keep3 = _desc(lib, s, fft=(25, 24, 24))
    assert lib.ssrpa_footprint(ctypes.byref(d3), 75, 16, lib.FP64, 0,
                               ctypes.byref(b)) == lib.ERR_ARG


def test_plan_valence_block(lib):
    s = sy.make_system(sy.TINY, 1000)
    d, keep = _desc(lib, s)
    vb = ctypes.c_int()
    assert lib.ssrpa_plan_valence_block(ctypes.byref(d), 75, 16, lib.FP64,
                                        1 << 40, ctypes.byref(vb)) == lib.OK
    assert vb.value == s.n_v
    b = ctypes.c_size_t()
    lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 3, ctypes.byref(b))
    assert lib.ssrpa_plan_valence_block(ctypes.byref(d), 75, 16, lib.FP64,
                                        b.value, ctypes.byref(vb)) == lib.OK
    assert vb.value == 3
    assert lib.ssrpa_plan_valence_block(ctypes.byref(d), 75, 16, lib.FP64,
                                        1000, ctypes.byref(vb)) == lib.ERR_NOMEM


def test_invalid_descriptions(lib):
    s = sy.make_system(sy.TINY, 1000)
    b = ctypes.c_size_t()
    d, keep = _desc(lib, s)
    d.n_v = 0
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, 0, 0,
                               ctypes.byref(b)) == lib.ERR_ARG
    d, keep = _desc(lib, s)
    d.ecut_chi = -1.0
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, 0, 0,
                               ctypes.byref(b)) == lib.ERR_ARG
    d, keep = _desc(lib, s)
    for i in range(9):
        d.lattice[i] = 0.0
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, 0, 0,
                               ctypes.byref(b)) == lib.ERR_ARG
    assert lib.ssrpa_footprint(None, 75, 16, 0, 0, ctypes.byref(b)) \
        == lib.ERR_ARG
    assert lib.ssrpa_frequency_grid(0, 1.0, None, None) == lib.ERR_ARG


def test_null_handles_are_rejected(lib):
    assert lib.ssrpa_context_destroy(None) == lib.ERR_ARG
    assert lib.ssrpa_system_destroy(None) == lib.ERR_ARG
    assert lib.ssrpa_chi0_static(None, 0, 0, None, 1, None) == lib.ERR_ARG
    assert lib.ssrpa_ticket_query(None, None) == lib.ERR_ARG


def test_occupation_validation_on_the_host(lib):
    """Partial occupations (Eqs. 4-6) are validated before any device work:
    f in [0, 1], non-increasing along the bands, ascending energies with
    equal f at equal energies, and n_v = the count of f > 0."""
    s = sy.make_system(sy.TINY, 1000)
    occ = sy.fermi_dirac_occupations(s.energy, 0.05, 0.01)
    sp = sy.with_occupations(s, occ)
    b = ctypes.c_size_t()

    def fp(occ_, n_v=sp.n_v, energy=sp.energy):
        keep = []
        d = lib.make_desc(sp.a, sp.fft, sp.miller, sp.coeff, energy, n_v,
                          sp.ecut_chi, keep, occ_)
        return lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 0,
                                   ctypes.byref(b))
    assert fp(occ) == lib.OK
    with_occ = b.value
    assert fp(None, n_v=s.n_v) == lib.OK
    assert with_occ > b.value          # more pairs: V x C grows
    bad = occ.copy()
    bad[3] = 1.5
    assert fp(bad) == lib.ERR_ARG      # outside [0, 1]
    bad = occ.copy()
    k = int(np.nonzero((occ > 0) & (occ < 1))[0][0])
    bad[k], bad[k + 1] = bad[k + 1], bad[k]
    assert fp(bad) == lib.ERR_ARG      # increasing along the bands
    assert fp(occ, n_v=sp.n_v - 1) == lib.ERR_ARG
    e2 = sp.energy.copy()
    e2[k + 1] = e2[k]                   # equal energies, different f
    assert fp(occ, energy=e2) == lib.ERR_ARG


def test_slab_truncation_needs_a_normal_third_axis(lib):
    s = sy.make_system(sy.TINY, 1000)
    b = ctypes.c_size_t()
    keep = []
    d = lib.make_desc(s.a, s.fft, s.miller, s.coeff, s.energy, s.n_v,
                      s.ecut_chi, keep, None, "slab")
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 0,
                               ctypes.byref(b)) == lib.OK
    lat = np.eye(3) * s.a
    lat[2, 0] = 0.5                      # a3 tilted: not normal to a1
    d = lib.make_desc(lat, s.fft, s.miller, s.coeff, s.energy, s.n_v,
                      s.ecut_chi, keep, None, "slab")
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 0,
                               ctypes.byref(b)) == lib.ERR_ARG
    d.coulomb_truncation = 7
    assert lib.ssrpa_footprint(ctypes.byref(d), 75, 16, lib.FP64, 0,
                               ctypes.byref(b)) == lib.ERR_ARG
