"""Non-integer exponents in the quadrature (paper, Sec. 4.3: the meromorphic
continuation of the three-body zeta function in nu): the GPU against the oracle
on the same plans in d = 1, 2, 3, the 1-D scan over -2 <= nu <= 3 on a sample of
its points, and the two-body identity zeta^(2)(nu_1, nu_2) = Z_{nu_1 + nu_2}(0)
(Sec. 2, Corollary) across a non-integer split of an integer sum."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ez():
    import paper_2504_11989_amd as ez
    ez.version()
    return ez


def bar(A, nus, spec):
    """(oracle value, parity bar): 1e-12 relative, or the FP64 floor 4e-15 (|H| + |N|)
    where the Hadamard part and the node part cancel"""
    v, parts = O.nbody(A, list(nus), spec, parts=True)
    return v, max(TOL * abs(v), 4e-15 * float(np.abs(parts).sum()))


@pytest.mark.parametrize("nus", [(2.52, 3.02, 4.52), (1.52, 1.52, 2.02), (0.52, 0.52, 0.52),
                                 (-1.98, 2.52, 2.52), (-0.98, 1.02, 2.52), (3.3, 3.3, 3.3)])
def test_three_body_1d(ez, nus):
    got = ez.nbody_lattice_sum(np.eye(1), list(nus), W.SPEC_1D).item()
    ref, b = bar(np.eye(1), nus, W.SPEC_1D)
    assert abs(got - ref) <= b, (nus, got, ref, b)


def test_meromorphic_scan_1d_sample(ez):
    """points of the diagonal scan nu_1 = nu_2 = nu_3 = -2 + j/20 + 1/50 (the paper's
    grid and offset), one per unit interval of nu and the ends"""
    for j in (0, 13, 27, 40, 58, 71, 86, 100):
        nu = -2.0 + j / 20.0 + 1.0 / 50.0
        got = ez.nbody_lattice_sum(np.eye(1), [nu] * 3, W.SPEC_1D).item()
        ref, b = bar(np.eye(1), [nu] * 3, W.SPEC_1D)
        assert abs(got - ref) <= b, (nu, got, ref, b)


def test_three_body_2d_and_3d(ez):
    spec2 = dict(W.SPEC_2D, n_q=6, n_panels=3, n_g=8)
    for A, nus, spec in ((W.A_HEX, (2.5, 3.3, 4.7), spec2), (np.eye(2), (1.25, 2.75, 3.6), spec2),
                         (W.fcc(), (3.5, 4.25, 6.1), W.SPEC_SMALL_3D), (W.bcc(), (2.2, 3.7, 5.3), W.SPEC_SMALL_3D)):
        got = ez.nbody_lattice_sum(A, list(nus), spec).item()
        ref, b = bar(A, nus, spec)
        assert abs(got - ref) <= b, (nus, got, ref, b)


def test_two_body_non_integer_split(ez):
    """zeta^(2)(2.7, 3.3) = Z_6(0) and zeta^(2)(1.5, 4.5) = Z_6(0) on the full d = 3
    plan: the integer sum of two non-integer exponents, against the direct Epstein
    zeta at the origin"""
    for A in (W.sc(), W.fcc()):
        z6 = O.epstein(A, 6.0, np.zeros(3), np.zeros(3)).real
        a = ez.nbody_lattice_sum(A, [2.7, 3.3], W.SPEC_FULL_3D).item()
        b = ez.nbody_lattice_sum(A, [1.5, 4.5], W.SPEC_FULL_3D).item()
        assert abs(a - z6) <= 1e-12 * abs(z6), (a, z6)
        assert abs(b - z6) <= 1e-12 * abs(z6), (b, z6)


def test_real_exponents_take_no_mixed_path(ez):
    """mixed precision does not apply to non-integer exponents: bound 0, FP64 values"""
    from paper_2504_11989_amd import _native as nat
    nu = [2.52, 3.02]
    terms = [(0, 1.0, [(0, 1), (1, 2)])]
    v, b = ez.lattice_sums(np.eye(1)[None], nu, terms, 1, W.SPEC_1D, with_bound=True)
    vm, bm = ez.lattice_sums(np.eye(1)[None], nu, terms, 1, dict(W.SPEC_1D, precision=nat.PREC_MIXED),
                             with_bound=True)
    assert bm.item() == 0.0 and vm.item() == v.item()
