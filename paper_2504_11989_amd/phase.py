"""fcc / bcc phase diagram and Bain-path enthalpy of Lennard-Jones (n, m) plus
Axilrod-Teller-Muto crystals (paper, Sec. 5).

For a lattice shape Lambda (fixed generator matrix A) scaled by R > 0, every
energy is a power of R times a lattice constant:

    H(R) = k [Z_n / (n R^n) - Z_m / (m R^m)] + lam E3 / R^9 + p V R^3,
    k = n m / (2 (n - m)),

with Z_nu = Z_{Lambda,nu}(0) (the pair sums), E3 the ATM cohesive energy at R = 1
(Sec. 2, Proposition) and V = |det A|.  The lattice constants come from one
lattice-sum program on the GPU (two-body values through Sec. 2, Corollary:
Z_nu(0) = zeta^(2)(nu_1, nu_2) with nu_1 + nu_2 = nu), so each shape costs one
quadrature; the minimisation over R for every (p, lam) is then a scalar
problem solved on the host, vectorised over the (p, lam) grid.

  * phase_diagram: fcc and bcc with unit nearest-neighbour distance (Sec. 5),
    H minimised over R for each (p, lam); the sign of H_bcc - H_fcc and the
    critical coupling lam_c(p) where the two enthalpies cross.
  * bain_path: the body-centred tetragonal family at unit density, bcc at
    c/a = 1 and fcc at c/a = sqrt 2, H minimised over the scale at each c/a.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lattice_sums

__all__ = ["PHASE_NU", "PHASE_TERMS", "PHASE_RESULTS", "bct_unit_density", "lattice_constants", "h_min",
           "phase_diagram", "critical_coupling", "bain_path"]

# exponents and terms: Z_12 = zeta^(2)(5,7), Z_6 = zeta^(2)(3,3), Z_8 = zeta^(2)(3,5),
# Z_4 = zeta^(2)(1,3), and the ATM energy (Sec. 2, Proposition)
PHASE_NU = [-1.0, 1.0, 3.0, 5.0, 7.0]
PHASE_RESULTS = ["Z12", "Z6", "Z8", "Z4", "E_ATM"]
PHASE_TERMS = [
    (0, 1.0, [(3, 1), (4, 1)]),
    (1, 1.0, [(2, 2)]),
    (2, 1.0, [(2, 1), (3, 1)]),
    (3, 1.0, [(1, 1), (2, 1)]),
    (4, 1.0 / 24.0, [(2, 3)]),
    (4, -3.0 / 16.0, [(0, 1), (3, 2)]),
    (4, 3.0 / 8.0, [(1, 1), (2, 1), (3, 1)]),
]
_LJ = {(12, 6): (0, 1), (8, 4): (2, 3)}


def bct_unit_density(c_over_a: float) -> np.ndarray:
    """Body-centred tetragonal generator matrix (columns (a,0,0), (0,a,0),
    (a/2,a/2,c/2)) with c = (c/a) a and |det| = a^3 (c/a)/2 = 1."""
    a = (2.0 / c_over_a) ** (1.0 / 3.0)
    c = c_over_a * a
    return np.array([[a, 0.0, a / 2.0], [0.0, a, a / 2.0], [0.0, 0.0, c / 2.0]])


def lattice_constants(A, spec=None) -> dict:
    """Z_12, Z_6, Z_8, Z_4, E_ATM and V of a batch of 3 x 3 generator matrices (numpy)."""
    At = torch.as_tensor(np.asarray(A, dtype=np.float64), device="cuda")
    out = lattice_sums(At, PHASE_NU, PHASE_TERMS, len(PHASE_RESULTS), spec).cpu().numpy()
    res = {name: out[:, i] for i, name in enumerate(PHASE_RESULTS)}
    res["V"] = np.abs(np.linalg.det(np.asarray(A, dtype=np.float64)))
    return res


def _coeffs(const: dict, lj, p, lam):
    n, m = lj
    i_n, i_m = _LJ[tuple(lj)]
    k = n * m / (2.0 * (n - m))
    zn, zm = const[PHASE_RESULTS[i_n]], const[PHASE_RESULTS[i_m]]
    return k * zn / n, k * zm / m, lam * const["E_ATM"], p * const["V"]


def h_min(const: dict, lj=(12, 6), p=0.0, lam=0.0, iters: int = 90):
    """min over R > 0 of H(R) = a/R^n - b/R^m + c/R^9 + d R^3 for every lattice of
    `const` and every (p, lam) broadcast against them.  Returns (H_min, R_min).

    R dH/dR = -n a R^-n + m b R^-m - 9 c R^-9 + 3 d R^3 is negative at small R
    (there -n a R^-n dominates when c >= 0) and positive at large R (the
    attraction m b R^-m with m < 9, or the pressure term); with one sign change
    on [0.2, 5] the minimiser is found by bisection in log R and H is evaluated
    there.  A bracket without a sign change raises ValueError."""
    n, m = lj
    a, b, c, d = np.broadcast_arrays(*_coeffs(const, lj, np.asarray(p, dtype=np.float64),
                                              np.asarray(lam, dtype=np.float64)))

    def rdh(R):
        return -n * a * R ** -n + m * b * R ** -m - 9.0 * c * R ** -9 + 3.0 * d * R ** 3

    lo = np.full(a.shape, 0.2)
    hi = np.full(a.shape, 5.0)
    if np.any(rdh(lo) >= 0.0) or np.any(rdh(hi) <= 0.0):
        raise ValueError("no sign change of dH/dR on [0.2, 5]: coefficients out of range")
    for _ in range(iters):
        mid = np.sqrt(lo * hi)
        neg = rdh(mid) < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    R = np.sqrt(lo * hi)
    H = a * R ** -n - b * R ** -m + c * R ** -9 + d * R ** 3
    return H, R


def phase_diagram(const_fcc: dict, const_bcc: dict, ps, lams, lj=(12, 6)):
    """H_bcc - H_fcc on the (p, lam) grid (rows p, columns lam); negative means bcc."""
    P, L = np.meshgrid(np.asarray(ps, dtype=np.float64), np.asarray(lams, dtype=np.float64), indexing="ij")
    hf, _ = h_min(const_fcc, lj, P, L)
    hb, _ = h_min(const_bcc, lj, P, L)
    return hb - hf


def critical_coupling(const_fcc: dict, const_bcc: dict, ps, lj=(12, 6), lam_max: float = 4.0,
                      iters: int = 100):
    """lam_c(p): the ATM coupling at which H_bcc = H_fcc, by bisection in lam on
    [0, lam_max] (fcc below, bcc above); NaN where no crossing lies in the range."""
    ps = np.asarray(ps, dtype=np.float64)
    lo = np.zeros_like(ps)
    hi = np.full_like(ps, lam_max)

    def dh(lam):
        hf, _ = h_min(const_fcc, lj, ps, lam)
        hb, _ = h_min(const_bcc, lj, ps, lam)
        return hb - hf

    ok = (dh(lo) > 0.0) & (dh(hi) < 0.0)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        bcc = dh(mid) < 0.0
        hi = np.where(bcc, mid, hi)
        lo = np.where(bcc, lo, mid)
    return np.where(ok, 0.5 * (lo + hi), np.nan)


def bain_path(cas, spec=None, lj=(12, 6), p=0.0, lam=0.0):
    """H minimised over the scale along the Bain path: bct at unit density with
    c/a = cas (bcc at 1, fcc at sqrt 2).  Returns (H_min (len(cas),), scale,
    lattice constants)."""
    A = np.stack([bct_unit_density(ca) for ca in cas])
    const = lattice_constants(A, spec)
    H, s = h_min(const, lj, p, lam)
    return H, s, const
