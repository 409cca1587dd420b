"""The C-ABI library loads, exports every symbol declared in include/ezeta.h,
and rejects bad arguments on the host before any launch (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2504_11989_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libezeta.so not built")
    return _native


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ezeta.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|ez_status|uint64_t)\s*(ez_\w+)\s*\(", src, re.M)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for s in ["ez_epstein_zeta", "ez_nbody_lattice_sum", "ez_atm_energy", "ez_lattice_sums",
              "ez_last_error", "ez_finalize", "ez_version"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    nat = _lib()
    L = ctypes.CDLL(nat.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(nat.EXPORTED) == set(declared_symbols())


def test_struct_layout_matches_header():
    nat = _lib()
    assert ctypes.sizeof(nat.QuadSpec) == 48


def _spec(nat, **kw):
    s = dict(n_q=6, n_panels=3, n_g=8, ell=4, eps=1e-2, lam=1.0, a_cut=36.0)
    s.update(kw)
    return nat.QuadSpec.from_dict(s)


def test_host_validation_errors():
    nat = _lib()
    L = nat.lib()
    dummy = ctypes.c_void_p(16)          # never dereferenced: validation fails first
    nu = (ctypes.c_double * 3)(3.0, 3.0, 3.0)
    # d out of range
    assert L.ez_nbody_lattice_sum(1, 4, dummy, 3, nu, ctypes.byref(_spec(nat)), dummy, None, None) == 1
    # null A
    assert L.ez_nbody_lattice_sum(1, 3, None, 3, nu, ctypes.byref(_spec(nat)), dummy, None, None) == 1
    # bad specs
    for bad in [dict(n_q=0), dict(ell=7), dict(ell=9), dict(eps=0.7), dict(eps=0.0), dict(lam=-1.0), dict(a_cut=500.0)]:
        assert L.ez_nbody_lattice_sum(1, 3, dummy, 3, nu, ctypes.byref(_spec(nat, **bad)), dummy, None, None) == 1
    # mixed precision: derivatives refuse it, unknown precision and a_mix < 8 are invalid
    assert L.ez_atm_energy(1, 3, dummy, ctypes.byref(_spec(nat, precision=1)), dummy, dummy, None, None) == 4
    assert b"FP64 only" in L.ez_last_error()
    assert L.ez_atm_energy(1, 3, dummy, ctypes.byref(_spec(nat, precision=2)), dummy, None, None, None) == 1
    assert L.ez_atm_energy(1, 3, dummy, ctypes.byref(_spec(nat, precision=1, flags=nat.spec_mix_a(4))),
                           dummy, None, None, None) == 1
    # non-finite exponents in the quadrature; an exponent nu = d + 2m with its logarithmic
    # singular part cannot share a call with non-integer exponents
    nu2 = (ctypes.c_double * 2)(2.5, float("nan"))
    assert L.ez_nbody_lattice_sum(1, 3, dummy, 2, nu2, ctypes.byref(_spec(nat)), dummy, None, None) == 1
    nu3 = (ctypes.c_double * 2)(2.5, 5.0)
    assert L.ez_nbody_lattice_sum(1, 3, dummy, 2, nu3, ctypes.byref(_spec(nat)), dummy, None, None) == 4
    assert b"logarithmic" in L.ez_last_error()
    # derivatives need integer exponents
    nu4 = (ctypes.c_double * 1)(2.5)
    t1 = (ctypes.c_int * 1)(0)
    c1 = (ctypes.c_double * 1)(1.0)
    n1 = (ctypes.c_int * 1)(1)
    f1 = (ctypes.c_int * 4)(0, 0, 0, 0)
    m1 = (ctypes.c_int * 4)(2, 0, 0, 0)
    sp1 = (nat.QuadSpec * 1)(_spec(nat))
    assert L.ez_lattice_sums_grad(1, 3, dummy, 1, nu4, 1, t1, c1, n1, f1, m1, 1, sp1, 1, dummy, dummy,
                                  None, None) == 4
    assert b"integer" in L.ez_last_error()
    # a Hadamard exponent mu = d + (nu - d) = 0: nu = 0 alone (paper, Sec. 3, mu + 2k = 0)
    nu0 = (ctypes.c_double * 1)(0.0)
    assert L.ez_nbody_lattice_sum(1, 3, dummy, 1, nu0, ctypes.byref(_spec(nat)), dummy, None, None) == 4
    # Epstein: bad n_nu, non-finite nu
    nu_inf = (ctypes.c_double * 1)(float("inf"))
    assert L.ez_epstein_zeta(3, dummy, 0, nu, 1, dummy, dummy, 0.0, 0.0, dummy, None, None) == 1
    assert L.ez_epstein_zeta(3, dummy, 1, nu_inf, 1, dummy, dummy, 0.0, 0.0, dummy, None, None) == 1
    assert L.ez_epstein_zeta(3, dummy, 1, nu, -1, dummy, dummy, 0.0, 0.0, dummy, None, None) == 1
    # derivatives: at most 2 results per call
    one = (ctypes.c_int * 3)(0, 1, 2)
    cf = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    nf = (ctypes.c_int * 3)(1, 1, 1)
    fac = (ctypes.c_int * 12)()
    mult = (ctypes.c_int * 12)(2, 0, 0, 0, 2, 0, 0, 0, 2, 0, 0, 0)
    sp = (nat.QuadSpec * 1)(_spec(nat))
    assert L.ez_lattice_sums_grad(1, 3, dummy, 1, nu, 3, one, cf, nf, fac, mult, 3, sp, 1, dummy, dummy,
                                  None, None) == 1
    assert b"at most 2" in L.ez_last_error()
    # the bound entry point needs its output pointer; the no-allocation one is FP64 only
    assert L.ez_lattice_sums_bound(1, 3, dummy, 1, nu, 3, one, cf, nf, fac, mult, 3, sp, 1, dummy, None,
                                   None, None) == 1
    spm = (nat.QuadSpec * 1)(_spec(nat, precision=1))
    assert L.ez_lattice_sums_noalloc(1, 3, dummy, 1, nu, 3, one, cf, nf, fac, mult, 3, spm, 1, dummy,
                                     None, None) == 4


def test_version_string():
    nat = _lib()
    assert b"gfx950" in nat.lib().ez_version()


def test_workspace_generation_is_exported_and_stable():
    nat = _lib()
    g = nat.workspace_generation()
    assert g >= 1 and nat.workspace_generation() == g
