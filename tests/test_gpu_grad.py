"""GPU: derivatives of the lattice sums with respect to the generator matrix
(adjoint kernels, through the C ABI), against
  - the oracle's derivative of its own value on the same plan (fourth-order
    central differences of the oracle, oracle.grad_fd),
  - central differences of the GPU forward value,
  - exact identities: homogeneity tr(A^T dR/dA) = -(sum nu) R and rotation
    invariance ((dR/dA) A^T symmetric),
  - a brute-force lattice-sum gradient for the two-body sum zeta^(2)(6,6) = Z_12(0)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL_1D = dict(W.SPEC_1D, n_panels=6, n_g=16)


@pytest.fixture(scope="module")
def ez():
    import paper_2504_11989_amd as ez
    ez.version()
    return ez


def perturbed(A0, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    return A0 * (1.0 + amp * rng.uniform(-1.0, 1.0, A0.shape))


def gpu_fd(fn, A, h=1e-3):
    """fourth-order central differences of a GPU scalar function of A (float)"""
    d = A.shape[0]
    g = np.zeros((d, d))
    for i in range(d):
        for j in range(d):
            v = []
            for s in (-2, -1, 1, 2):
                B = A.copy()
                B[i, j] += s * h
                v.append(fn(B))
            g[i, j] = (v[0] - 8 * v[1] + 8 * v[2] - v[3]) / (12 * h)
    return g


def relnorm(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("d,spec,A", [
    (1, SMALL_1D, np.array([[1.3]])),
    (2, dict(W.SPEC_2D, n_q=8, n_panels=4, n_g=10), np.array([[1.0, 0.31], [0.12, 0.93]])),
    (3, W.SPEC_SMALL_3D, None),
])
def test_atm_grad_vs_oracle(ez, d, spec, A):
    if A is None:
        A = perturbed(W.fcc(), 51)
    E, g = ez.atm_energy(A, spec, grad=True)
    E0 = ez.atm_energy(A, spec)
    E, E0, g = E.item(), E0.item(), g[0].cpu().numpy()
    # the adjoint launch returns the same value as the plain forward one
    assert abs(E - E0) <= 1e-14 * abs(E0)
    ref = O.grad_fd(lambda B: O.atm(B, spec), A, h=5e-4)
    assert relnorm(g, ref) <= 1e-8, (g, ref)


@pytest.mark.parametrize("name,seed", [("sc", 52), ("fcc", 53), ("bcc", 54)])
def test_atm_grad_identities(ez, name, seed):
    A = perturbed(getattr(W, name)(), seed)
    E, g = ez.atm_energy(A, W.SPEC_SMALL_3D, grad=True)
    E, g = E.item(), g[0].cpu().numpy()
    # homogeneity of degree -9 of every ATM term (sum of exponents 9)
    assert abs(np.trace(A.T @ g) + 9.0 * E) <= 1e-11 * abs(9.0 * E)
    S = g @ A.T
    assert np.linalg.norm(S - S.T) <= 1e-11 * np.linalg.norm(S)


def test_grad_schedules_give_identical_results(ez):
    """the adjoint direction kernel on the second stream (default) or before the
    nodes on the caller's stream (serial flag): same partials, same sums, bit for bit"""
    from paper_2504_11989_amd._native import SPEC_SERIAL
    lat = np.stack([perturbed(W.sc(), 55), perturbed(W.fcc(), 56), perturbed(W.bcc(), 57)])
    E0, g0 = ez.atm_energy(lat, W.SPEC_SMALL_3D, grad=True)
    E1, g1 = ez.atm_energy(lat, dict(W.SPEC_SMALL_3D, flags=SPEC_SERIAL), grad=True)
    assert np.array_equal(E0.cpu().numpy(), E1.cpu().numpy())
    assert np.array_equal(g0.cpu().numpy(), g1.cpu().numpy())


def test_atm_grad_vs_gpu_central_differences(ez):
    A = perturbed(W.bcc(), 55)
    spec = W.SPEC_SMALL_3D
    _, g = ez.atm_energy(A, spec, grad=True)
    ref = gpu_fd(lambda B: ez.atm_energy(B, spec).item(), A)
    assert relnorm(g[0].cpu().numpy(), ref) <= 1e-8


def test_two_body_grad_vs_brute_force(ez):
    """zeta^(2)(6,6) = Z_12(0) (Sec. 2, Corollary); d Z_12(0)/dA = -12 sum' |An|^-14 (An) n^T."""
    A = perturbed(W.fcc(), 56, amp=0.05)
    val, g = ez.lattice_sums(A, [6.0], [(0, 1.0, [(0, 2)])], 1, W.SPEC_FULL_3D, grad=True)
    L = 24
    r = np.arange(-L, L + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    n = n[np.any(n != 0, axis=1)]
    z = n @ A.T
    r2 = np.einsum("ij,ij->i", z, z)
    Z12 = np.sum(r2 ** -6)
    G = -12.0 * np.einsum("i,ij,ik->jk", r2 ** -7, z, n)
    assert abs(val.item() - Z12) <= 1e-12 * Z12
    assert relnorm(g[0, 0].cpu().numpy(), G) <= 1e-11


def test_lj_atm_program_grad(ez):
    """two results (E_LJ, E_ATM) with derivatives in one call, against the oracle on the same plan"""
    from paper_2504_11989_amd import enthalpy as H
    A = perturbed(W.fcc(), 57)
    spec = W.SPEC_SMALL_3D
    E, g = H.energies(A, spec, grad=True)
    E, g = E[0].cpu().numpy(), g[0].cpu().numpy()

    def elj(B):
        return 0.5 * O.nbody(B, [5, 7], spec) - O.nbody(B, [3, 3], spec)

    assert abs(E[0] - elj(A)) <= 1e-12 * abs(E[0])
    assert abs(E[1] - O.atm(A, spec)) <= 1e-12 * abs(E[1])
    assert relnorm(g[0], O.grad_fd(elj, A, h=5e-4)) <= 1e-8
    assert relnorm(g[1], O.grad_fd(lambda B: O.atm(B, spec), A, h=5e-4)) <= 1e-8


def test_lj_full_plan_matches_epstein(ez):
    """E_LJ = Z_12(0)/2 - Z_6(0) through the two-body quadrature (Sec. 2, Corollary)
    against the Epstein values computed directly by the oracle"""
    from paper_2504_11989_amd import enthalpy as H
    A = perturbed(W.bcc(), 61)
    E = H.energies(A, W.SPEC_FULL_3D)[0].cpu().numpy()
    z = [0.0, 0.0, 0.0]
    elj = O.epstein(A, 12.0, z, z).real / 2 - O.epstein(A, 6.0, z, z).real
    assert abs(E[0] - elj) <= 1e-12 * abs(elj)


def test_batch_with_bad_lattice_grad(ez):
    A = np.stack([W.sc(), np.zeros((3, 3)), W.bcc()])
    E, g, st = ez.atm_energy(A, W.SPEC_SMALL_3D, grad=True, with_status=True)
    st = st.cpu().numpy()
    assert st[1] & 0x1 and st[0] == 0 and st[2] == 0
    g = g.cpu().numpy()
    assert np.isnan(g[1]).all() and np.isfinite(g[0]).all() and np.isfinite(g[2]).all()
    E1, g1 = ez.atm_energy(W.bcc(), W.SPEC_SMALL_3D, grad=True)
    assert relnorm(g[2], g1[0].cpu().numpy()) <= 1e-14


def test_autograd_function(ez):
    from paper_2504_11989_amd.autograd import atm_energy_t
    A = torch.tensor(perturbed(W.sc(), 58), dtype=torch.float64, device="cuda", requires_grad=True)
    E = atm_energy_t(A, W.SPEC_SMALL_3D)
    (3.0 * E).backward()
    _, g = ez.atm_energy(A.detach(), W.SPEC_SMALL_3D, grad=True)
    assert torch.allclose(A.grad, 3.0 * g[0], rtol=0, atol=0)


def test_enthalpy_minimisation_decreases_and_converges(ez):
    from paper_2504_11989_amd import enthalpy as H
    A0 = np.stack([perturbed(W.fcc(), 59, 0.05), perturbed(W.bcc(), 60, 0.05)])
    res = H.minimise(A0, 0.0, 0.0, W.SPEC_SMALL_3D, max_iter=150, gtol=1e-7)
    H0, _, _, _ = H.enthalpy(torch.tensor(A0, device="cuda"), 0.0, 0.0, W.SPEC_SMALL_3D)
    assert np.all(res["H"] < H0.cpu().numpy())
    assert res["converged"].all(), res["grad_norm"]
    # pure LJ: the minimum from an fcc start is fcc; its energy is below the bcc-start one
    assert H.classify(res["A"][0]) == "fcc"
    assert res["H"][0] <= res["H"][1] + 1e-9


def test_eight_exponents_taylor_order_six(ez):
    """large probe and adjoint-direction LDS layouts (86 and 113 KB): 8 exponents,
    Taylor order 6 (the oracle's largest), four-factor products (degree 24 on
    (0, eps)); values against the oracle, derivatives by homogeneity of degree
    -sum(nu) and the symmetry of the strain derivative"""
    nu = [-1.0, 1.0, 3.0, 5.0, 6.0, 7.0, 9.0, 12.0]
    terms = [(0, 1.0, [(0, 1), (1, 1), (2, 1), (3, 1)]), (1, 1.0, [(4, 1), (5, 1), (6, 1), (7, 1)])]
    spec = dict(W.SPEC_SMALL_3D, ell=6)
    A = perturbed(W.fcc(), 58)
    R, g = ez.lattice_sums(A, nu, terms, 2, spec, grad=True)
    R, g = R[0].cpu().numpy(), g[0].cpu().numpy()
    for r, nus in enumerate([(-1, 1, 3, 5), (6, 7, 9, 12)]):
        # (-1, 1, 3, 5): the Hadamard and node parts (about 7.5e6 each) cancel to
        # -556, a factor 2.7e4; the bar scales with the parts (see nbody_bar)
        ref, parts = O.nbody(A, nus, spec, parts=True)
        kappa = float(np.abs(parts).sum()) / abs(ref)
        tol = max(1e-12, 4e-15 * kappa)
        assert abs(R[r] - ref) <= tol * abs(ref), (r, R[r], ref, kappa)
        deg = -float(sum(nus))
        assert abs(np.trace(A.T @ g[r]) - deg * R[r]) <= 4 * tol * abs(deg * R[r]), r
        S = g[r] @ A.T
        assert np.linalg.norm(S - S.T) <= 4 * tol * np.linalg.norm(S), r


def test_enthalpy_gradient_finite_coupling_and_pressure(ez):
    """dH/dA of H = E_LJ + c E_ATM + p V at c, p > 0 (the p V term and its
    derivative |det A| A^{-T} included): against central differences of the GPU
    value with h = 1e-6 (rounding of the difference ~ 1e-16 |H| / h, truncation
    ~ h^2), and against the oracle's fourth-order differences of its own H on the
    same plan"""
    from paper_2504_11989_amd import enthalpy as H
    spec = W.SPEC_SMALL_3D
    c, p = 1.3, 0.6
    for seed, A0 in [(71, W.fcc()), (72, W.bcc())]:
        A = perturbed(A0, seed)
        Hv, g, E, V = H.enthalpy(torch.tensor(A[None], device="cuda"), c, p, spec)
        Hv, g = Hv.item(), g[0].cpu().numpy()

        def h_gpu(B):
            return H.enthalpy(torch.tensor(B[None], device="cuda"), c, p, spec)[0].item()

        def h_oracle(B):
            elj = 0.5 * O.nbody(B, [5, 7], spec) - O.nbody(B, [3, 3], spec)
            return elj + c * O.atm(B, spec) + p * abs(np.linalg.det(B))

        assert abs(Hv - h_oracle(A)) <= 1e-12 * abs(Hv)
        fd = np.zeros((3, 3))
        hh = 1e-6
        for i in range(3):
            for j in range(3):
                Bp, Bm = A.copy(), A.copy()
                Bp[i, j] += hh
                Bm[i, j] -= hh
                fd[i, j] = (h_gpu(Bp) - h_gpu(Bm)) / (2 * hh)
        assert relnorm(g, fd) <= 1e-7, (seed, relnorm(g, fd))
        assert relnorm(g, O.grad_fd(h_oracle, A, h=5e-4)) <= 1e-8, seed



def test_phase_scan_small_grid(ez):
    """the (c, p) scan on a 2 x 2 grid: the minimisation of H over the scale of
    the fcc and bcc lattices converges everywhere, pure LJ (c = p = 0) gives the
    fcc cohesive energy -8.6102 at R slightly below 1 and picks fcc, the final H
    equals the oracle's H at the final matrix, pressure compresses, and the
    general-matrix minimisation from the perturbed pure-LJ winner returns to fcc"""
    from paper_2504_11989_amd import enthalpy as H
    spec = W.SPEC_SMALL_3D
    cs, ps = [0.0, 1.5], [0.0, 0.8]
    res = H.phase_scan(cs, ps, spec, stability=True, stability_iter=150)
    assert res["converged"].all(), res["H"]
    assert res["phase"][0, 0] == "fcc" and abs(res["H"][0, 0, 0] + 8.6102) < 1e-3, res["H"][0, 0]
    assert 0.95 < res["R"][0, 0, 0] < 1.0
    assert res["general"][0, 0] == "fcc", res["general"]
    i, j = 1, 1
    Af = res["A"][i, j]
    elj = 0.5 * O.nbody(Af, [5, 7], spec) - O.nbody(Af, [3, 3], spec)
    ref = elj + cs[i] * O.atm(Af, spec) + ps[j] * abs(np.linalg.det(Af))
    k = 0 if res["phase"][i, j] == "fcc" else 1
    assert abs(res["H"][i, j, k] - ref) <= 1e-12 * abs(ref)
    assert res["V"][0, 1] < res["V"][0, 0] and res["V"][1, 1] < res["V"][1, 0]
