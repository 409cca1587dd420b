"""fcc / bcc phase diagram and Bain path (paper, Sec. 5) on the GPU: the
lattice constants against the oracle on the same plan, the two-body values
against direct Epstein sums (Sec. 2, Corollary), and the physics the paper
states for the phase boundary."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11989_amd import phase
    return phase


@pytest.fixture(scope="module")
def consts(ph):
    A = np.stack([W.A_FCC_NN1, W.A_BCC_NN1])
    return ph.lattice_constants(A, W.SPEC_FULL_3D)


def _split(c, i):
    return {k: v[i:i + 1] for k, v in c.items()}


def test_lattice_constants_vs_oracle(ph):
    """Z_12, Z_6, Z_8, Z_4 as two-body zeta functions and E_ATM, small plan,
    fcc and bcc at unit nearest-neighbour distance, identical plans"""
    spec = W.SPEC_SMALL_3D
    A = np.stack([W.A_FCC_NN1, W.A_BCC_NN1])
    got = ph.lattice_constants(A, spec)
    pairs = {"Z12": (5.0, 7.0), "Z6": (3.0, 3.0), "Z8": (3.0, 5.0), "Z4": (1.0, 3.0)}
    for i in range(2):
        for name, nu in pairs.items():
            ref = oracle.nbody(A[i], list(nu), spec)
            assert abs(got[name][i] - ref) <= TOL * abs(ref), (i, name, got[name][i], ref)
        ref = oracle.atm(A[i], spec)
        assert abs(got["E_ATM"][i] - ref) <= TOL * abs(ref), (i, got["E_ATM"][i], ref)


def test_two_body_values_are_direct_epstein_sums(consts):
    """zeta^(2)(nu1, nu2) = Z_{nu1+nu2}(0) (Sec. 2, Corollary): the full-plan
    quadrature against the oracle's Epstein zeta at the origin"""
    A = [W.A_FCC_NN1, W.A_BCC_NN1]
    for i in range(2):
        for name, nu in (("Z12", 12.0), ("Z6", 6.0), ("Z8", 8.0), ("Z4", 4.0)):
            ref = oracle.epstein(A[i], nu, np.zeros(3), np.zeros(3)).real
            assert abs(consts[name][i] - ref) <= 1e-12 * abs(ref), (i, name, consts[name][i], ref)


def test_no_three_body_coupling_means_fcc(ph, consts):
    """without the ATM term fcc has the lower enthalpy at every pressure, for
    both Lennard-Jones potentials (Sec. 5)"""
    f, b = _split(consts, 0), _split(consts, 1)
    for lj in ((12, 6), (8, 4)):
        dh = ph.phase_diagram(f, b, np.linspace(0.0, 2.0, 9), [0.0], lj)
        assert np.all(dh > 0.0), (lj, dh)


def test_strong_coupling_favours_bcc_and_pressure_favours_fcc(ph, consts):
    """a large enough ATM coupling makes bcc stable; pressure raises the
    critical coupling for (12,6) markedly and for (8,4) only slightly (Sec. 5)"""
    f, b = _split(consts, 0), _split(consts, 1)
    ps = np.linspace(0.0, 2.0, 5)
    lc126 = ph.critical_coupling(f, b, ps, (12, 6), lam_max=20.0)
    lc84 = ph.critical_coupling(f, b, ps, (8, 4), lam_max=20.0)
    assert np.all(np.isfinite(lc126)) and np.all(np.isfinite(lc84)), (lc126, lc84)
    assert np.all(np.diff(lc126) > 0.0), lc126
    rel126 = (lc126[-1] - lc126[0]) / lc126[0]
    rel84 = abs(lc84[-1] - lc84[0]) / lc84[0]
    assert rel84 < 0.5 * rel126, (lc126, lc84)
    dh = ph.phase_diagram(f, b, [0.0], [1.2 * lc126[0]], (12, 6))
    assert dh[0, 0] < 0.0


def test_bain_path_endpoints_and_stationarity(ph, consts):
    """bct at c/a = 1 and sqrt 2 has the minimised enthalpy of bcc and fcc, and
    the Bain path is stationary there (cubic symmetry: zero first-order change
    under a volume-preserving tetragonal strain once the volume is relaxed), so
    the central difference D(h) = (H(x+h) - H(x-h)) / 2h shrinks like h^2"""
    h = 0.02
    r2 = np.sqrt(2.0)
    cas = np.concatenate([x + np.array([-h, -h / 2, 0.0, h / 2, h]) for x in (1.0, r2)])
    for lj, p, lam in (((12, 6), 0.0, 0.0), ((12, 6), 0.5, 0.3), ((8, 4), 1.0, 0.5)):
        H, s, _ = ph.bain_path(cas, W.SPEC_FULL_3D, lj, p, lam)
        hb, _ = ph.h_min(_split(consts, 1), lj, p, lam)
        hf, _ = ph.h_min(_split(consts, 0), lj, p, lam)
        assert abs(H[2] - hb[0]) <= 1e-11 * abs(hb[0]), (lj, H[2], hb[0])
        assert abs(H[7] - hf[0]) <= 1e-11 * abs(hf[0]), (lj, H[7], hf[0])
        for j in (2, 7):
            d_h = (H[j + 2] - H[j - 2]) / (2 * h)
            d_h2 = (H[j + 1] - H[j - 1]) / h
            noise = 1e-11 * abs(H[j]) / h
            assert abs(d_h2) < 0.4 * abs(d_h) + noise, (lj, j, d_h, d_h2)
