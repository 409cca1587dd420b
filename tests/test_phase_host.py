"""Host logic of the phase-diagram module: the scalar minimisation over the
lattice scale and the critical coupling, on synthetic lattice constants (no GPU)."""
import numpy as np
import pytest

from paper_2504_11989_amd import phase


def _const(z12, z6, z8, z4, e3, v):
    return {"Z12": np.array([z12]), "Z6": np.array([z6]), "Z8": np.array([z8]), "Z4": np.array([z4]),
            "E_ATM": np.array([e3]), "V": np.array([v])}


# values of the size of fcc / bcc lattice sums at unit nearest-neighbour distance
FCC = _const(12.13, 14.45, 12.80, 25.3, 9.6, 1.0 / np.sqrt(2.0))
BCC = _const(9.11, 12.25, 10.4, 22.6, 9.9, 4.0 / (3.0 * np.sqrt(3.0)))


@pytest.mark.parametrize("lj", [(12, 6), (8, 4)])
@pytest.mark.parametrize("p,lam", [(0.0, 0.0), (0.5, 0.3), (1.0, 1.5), (0.0, 2.0)])
def test_h_min_matches_dense_grid(lj, p, lam):
    """the bisection minimum agrees with a brute-force minimum over a dense grid
    in R (refined around the grid's best point)"""
    H, R = phase.h_min(FCC, lj, p, lam)
    a, b, c, d = phase._coeffs(FCC, lj, p, lam)
    n, m = lj
    Rs = np.linspace(0.3, 3.0, 200001)
    Hs = a * Rs ** -n - b * Rs ** -m + c * Rs ** -9 + d * Rs ** 3
    j = int(np.argmin(Hs))
    assert abs(R[0] - Rs[j]) < 2e-5
    assert Hs[j] >= H[0] - 1e-13 * abs(H[0])
    assert abs(Hs[j] - H[0]) < 1e-7 * abs(H[0])          # grid spacing 1.35e-5 in R


def test_h_min_broadcasts_over_a_grid():
    ps = np.linspace(0.0, 1.0, 5)[:, None]
    lams = np.linspace(0.0, 2.0, 4)[None, :]
    H, R = phase.h_min(FCC, (12, 6), ps, lams)
    assert H.shape == (5, 4) and R.shape == (5, 4)
    for i in range(5):
        for j in range(4):
            h1, r1 = phase.h_min(FCC, (12, 6), ps[i, 0], lams[0, j])
            assert h1[0] == H[i, j] and r1[0] == R[i, j]
    # pressure compresses, repulsive three-body coupling expands
    assert np.all(np.diff(R, axis=0) < 0) and np.all(np.diff(R, axis=1) > 0)


def test_critical_coupling_is_the_crossing():
    ps = np.array([0.0, 0.3, 0.8])
    lc = phase.critical_coupling(FCC, BCC, ps, (12, 6))
    for p, l in zip(ps, lc):
        if np.isnan(l):
            continue
        hf, _ = phase.h_min(FCC, (12, 6), p, l)
        hb, _ = phase.h_min(BCC, (12, 6), p, l)
        assert abs(hb[0] - hf[0]) < 1e-12 * abs(hf[0])


def test_h_min_rejects_collapse():
    """an attractive three-body term stronger than the (8,4) repulsion has no
    minimum on the bracket"""
    with pytest.raises(ValueError):
        phase.h_min(FCC, (8, 4), 0.0, -5.0)


def test_bct_unit_density_endpoints():
    """c/a = 1 is bcc and c/a = sqrt 2 is fcc (equal Gram matrices up to a
    unimodular change of basis: equal sorted lists of short vector lengths)"""
    import workloads as W

    def shell(A):
        n = np.arange(-3, 4)
        Z = np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3)
        r = np.linalg.norm(Z @ np.asarray(A).T, axis=1)
        return np.sort(r[r > 0])[:40]

    assert np.allclose(shell(phase.bct_unit_density(1.0)), shell(W.bcc()), atol=1e-12)
    assert np.allclose(shell(phase.bct_unit_density(np.sqrt(2.0))), shell(W.fcc()), atol=1e-12)
    assert abs(np.linalg.det(phase.bct_unit_density(1.3)) - 1.0) < 1e-14
