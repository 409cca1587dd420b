"""Seeded synthetic inputs for the Epstein-zeta lattice-sum workloads.

This module holds no arithmetic of the method: it only builds lattice
generator matrices, exponent lists, shifts and quadrature specs.  Both the
oracle-side tests and the GPU path draw their inputs from here, so that the
two sides see identical inputs.

Lattices are given by their generator matrix A (row-major, d x d) whose
COLUMNS are the basis vectors, Lambda = A Z^d (paper, Sec. 2, Definition
(Lattices)).  The paper's fcc/bcc matrices (Sec. 5) have unit nearest-
neighbour distance; "unit density" rescales them to |det A| = 1.
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)
SQRT3 = np.sqrt(3.0)

# paper, Sec. 4 and Sec. 5: fcc / bcc with unit nearest-neighbour distance
A_FCC_NN1 = np.array([[1.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 1.0]]) / SQRT2
A_BCC_NN1 = np.array([[1.0, 1.0, 0.0], [SQRT2, 0.0, SQRT2], [0.0, SQRT2, SQRT2]]) / SQRT3
# paper, Sec. 4: hexagonal lattice
A_HEX = np.array([[1.0, 0.5], [0.0, SQRT3 / 2.0]])


def a_kappa(kappa: float) -> np.ndarray:
    """2D lattice matrix with condition number kappa (paper, Sec. 4, eq. A_kappa)."""
    return np.array([[1.0, (kappa - 1.0 / kappa) / 2.0], [0.0, (kappa + 1.0 / kappa) / 2.0]])


def unit_density(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[0]
    return A / abs(np.linalg.det(A)) ** (1.0 / d)


def sc() -> np.ndarray:
    return np.eye(3)


def fcc() -> np.ndarray:
    return unit_density(A_FCC_NN1)


def bcc() -> np.ndarray:
    return unit_density(A_BCC_NN1)


def bct(c_over_a: float) -> np.ndarray:
    """Body-centred tetragonal lattice at unit density: generators (a,0,0),
    (0,a,0), (a/2,a/2,c/2) with c = (c/a) a and a^3 (c/a)/2 = 1
    (bcc at c/a = 1, fcc at c/a = sqrt 2)."""
    a = (2.0 / c_over_a) ** (1.0 / 3.0)
    c = c_over_a * a
    return np.array([[a, 0.0, a / 2.0], [0.0, a, a / 2.0], [0.0, 0.0, c / 2.0]])


# ---------------------------------------------------------------- quadrature specs
# n_q: Gauss points per v-dimension (paper: 14); u on (eps, 1/2]: n_panels
# geometric panels x n_g Gauss points; ell: Taylor cutoff (paper: 4);
# eps: split point (paper: 1e-2); lam: Ewald parameter in units of V^{1/d};
# a_cut: largest incomplete-gamma argument kept.  The full d = 3 plan uses
# lam = 1.3, where the real-space and reciprocal work per node balance.  The
# sums do not depend on lam mathematically; in FP64 the d = 3 ATM values move by
# about 1e-13 relative between lam = 1 and 1.3 (the conditioning of the ATM
# combination), and by a few 1e-12 below lam ~ 0.7.
SPEC_FULL_3D = dict(n_q=14, n_panels=7, n_g=16, ell=4, eps=1e-2, lam=1.3, a_cut=36.0)
SPEC_SMALL_3D = dict(n_q=6, n_panels=3, n_g=8, ell=4, eps=1e-2, lam=1.0, a_cut=36.0)
SPEC_1D = dict(n_q=1, n_panels=16, n_g=64, ell=4, eps=1e-2, lam=1.0, a_cut=36.0)   # 1024 u-nodes on (0,1/2]
SPEC_2D = dict(n_q=14, n_panels=6, n_g=16, ell=4, eps=1e-2, lam=1.0, a_cut=36.0)


def n_nodes(d: int, spec: dict) -> int:
    return d * (1 << (d - 1)) * spec["n_q"] ** (d - 1) * spec["n_panels"] * spec["n_g"]


# ---------------------------------------------------------------- configurations
def c1_spot_values(seed: int = 1):
    """64 spot values of Z_{Z,nu}(x,y): nu from {1.5,2,3,4.5} (16 each, shuffled),
    x, y uniform in [0,1)."""
    rng = np.random.default_rng(seed)
    nus = np.repeat(np.array([1.5, 2.0, 3.0, 4.5]), 16)
    rng.shuffle(nus)
    x = rng.random(64)
    y = rng.random(64)
    return nus, x, y


def c2_lattices():
    """sc, fcc, bcc at unit density."""
    return {"sc": sc(), "fcc": fcc(), "bcc": bcc()}


def c3_scan(seed: int = 3, count: int = 4096):
    """Batched bct scan: c/a ~ U[0.8, 1.6], node budget n^3 with n ~ U{16..64}."""
    rng = np.random.default_rng(seed)
    ca = rng.uniform(0.8, 1.6, size=count)
    nside = rng.integers(16, 65, size=count)
    A = np.stack([bct(c) for c in ca])
    return ca, nside, A


def c3_spec(nside: int, eps: float = 1e-2, lam: float = 1.0, a_cut: float = 36.0) -> dict:
    """Quadrature spec with about nside^3 nodes in d = 3: 12 n_q^2 directions x
    n_panels n_g u-nodes, n_q growing with nside."""
    n_q = max(4, int(round(14.0 * nside / 64.0)))
    n_u = max(8, int(round(nside ** 3 / (12.0 * n_q * n_q))))
    n_g = 8 if n_u < 40 else 16
    n_panels = max(1, int(round(n_u / n_g)))
    return dict(n_q=n_q, n_panels=n_panels, n_g=n_g, ell=4, eps=eps, lam=lam, a_cut=a_cut)


def c4_shifts(A: np.ndarray, seed: int = 4, count: int = 512) -> np.ndarray:
    """Real-space shifts x = A t, t ~ U[0,1)^3 (rows are shifts)."""
    rng = np.random.default_rng(seed)
    t = rng.random((count, A.shape[0]))
    return t @ np.asarray(A).T


def c4_points(A: np.ndarray, seed: int = 40, count: int = 8192) -> np.ndarray:
    """Points of the reciprocal cell y = A^{-T} s, s ~ U[-1/2,1/2)^d (rows are points)."""
    rng = np.random.default_rng(seed)
    s = rng.random((count, A.shape[0])) - 0.5
    return s @ np.linalg.inv(np.asarray(A))


def c5_perturbed(seed: int = 5, count: int = 64):
    """Generator matrices with entries perturbed by up to +-10% from unit-density fcc / bcc."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        A0 = fcc() if i % 2 == 0 else bcc()
        out.append(A0 * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, size=(3, 3))))
    return np.stack(out)


def c5_grid(n: int = 32):
    return np.linspace(0.0, 2.0, n), np.linspace(0.0, 1.0, n)
