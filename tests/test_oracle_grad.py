"""Pins of the oracle's derivative (oracle.grad_fd: fourth-order central
differences of the oracle's value on a fixed plan): a brute-force lattice-sum
gradient, homogeneity and rotation invariance."""
import numpy as np

import oracle as O
import workloads as W


def test_grad_fd_of_epstein_matches_direct_sum_gradient():
    """d Z_12(0)/dA = -12 sum' |An|^-14 (An) n^T, summed directly (|n|_inf <= 24)."""
    rng = np.random.default_rng(71)
    A = W.fcc() * (1.0 + 0.05 * rng.uniform(-1, 1, (3, 3)))
    z0 = [0.0, 0.0, 0.0]
    g = O.grad_fd(lambda B: O.epstein(B, 12.0, z0, z0).real, A, h=5e-4)
    r = np.arange(-24, 25)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    n = n[np.any(n != 0, axis=1)]
    z = n @ A.T
    r2 = np.einsum("ij,ij->i", z, z)
    G = -12.0 * np.einsum("i,ij,ik->jk", r2 ** -7, z, n)
    assert np.linalg.norm(g - G) <= 1e-9 * np.linalg.norm(G)


def test_grad_fd_of_atm_homogeneity_and_rotation():
    """E_ATM(t A) = t^-9 E_ATM(A) on a fixed fractional plan -> tr(A^T dE/dA) = -9 E;
    E_ATM(Q A) = E_ATM(A) -> (dE/dA) A^T symmetric."""
    rng = np.random.default_rng(72)
    A = W.bcc() * (1.0 + 0.1 * rng.uniform(-1, 1, (3, 3)))
    spec = dict(W.SPEC_SMALL_3D, n_q=4, n_g=6)
    E = O.atm(A, spec)
    g = O.grad_fd(lambda B: O.atm(B, spec), A, h=5e-4)
    assert abs(np.trace(A.T @ g) + 9.0 * E) <= 1e-9 * abs(9.0 * E)
    S = g @ A.T
    assert np.linalg.norm(S - S.T) <= 1e-9 * np.linalg.norm(S)


def test_grad_fd_is_exact_on_quartics():
    """the stencil is exact (to rounding) on polynomials of degree <= 4"""
    A = np.array([[1.1, 0.2], [-0.3, 0.9]])
    f = lambda B: B[0, 0] ** 4 + 3.0 * B[0, 1] ** 3 * B[1, 0] - B[1, 1] ** 2
    g = O.grad_fd(f, A, h=0.1)
    ref = np.array([[4 * A[0, 0] ** 3, 9 * A[0, 1] ** 2 * A[1, 0]], [3 * A[0, 1] ** 3, -2 * A[1, 1]]])
    assert np.allclose(g, ref, rtol=1e-12, atol=1e-12)
