"""GPU parity: the HIP path (through the C ABI) against the oracle on the same
seeded inputs and the same quadrature plans.  FP64 bar: 1e-12 relative."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ez():
    import paper_2504_11989_amd as ez
    ez.version()                     # raises if the HIP library is missing
    return ez


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def nbody_bar(A, nus, spec):
    """(oracle value, parity bar) of one n-body sum on a plan.  The result is the
    sum v = H + N of the Hadamard part on (0, eps) and the node part on (eps, 1/2];
    each part carries a relative rounding error of about 4e-15 (products of up
    to four Z values, each good to ~1e-15), so FP64 fixes v to about
    4e-15 (|H| + |N|).  The bar is 1e-12 |v|, or that floor where the parts
    cancel (strongly singular exponents such as (-1, 1, 3, 5))."""
    v, parts = O.nbody(A, nus, spec, parts=True)
    return v, max(TOL * abs(v), 4e-15 * float(np.abs(parts).sum()))


# ---------------------------------------------------------------- Epstein zeta at points
def test_c1_spot_values(ez):
    nus, xs, ys = W.c1_spot_values()
    z = ez.epstein_zeta(np.eye(1), [1.5, 2.0, 3.0, 4.5], xs, ys).cpu().numpy()
    col = {1.5: 0, 2.0: 1, 3.0: 2, 4.5: 3}
    for i, (nu, x, y) in enumerate(zip(nus, xs, ys)):
        ref = O.epstein(np.eye(1), nu, [x], [y])
        assert abs(z[col[nu], i] - ref) <= TOL * abs(ref), (i, nu, x, y)


def test_epstein_origin_and_lattice_points(ez):
    # Z(0,0) (y on Lambda*: continuation), x on the lattice, y on the reciprocal lattice
    for A in [np.eye(1), np.eye(2), W.A_HEX, W.sc(), W.fcc(), W.bcc()]:
        d = A.shape[0]
        B = np.linalg.inv(A).T
        pts_x = np.stack([np.zeros(d), A @ np.ones(d), np.full(d, 0.3)])
        pts_y = np.stack([np.zeros(d), np.full(d, 0.17), B @ np.ones(d)])
        nus = [-1.0, 1.5, 4.0, 6.0] if d != 1 else [-1.0, 0.5, 3.0, 4.0]
        z = ez.epstein_zeta(A, nus, pts_x, pts_y).cpu().numpy()
        for j, nu in enumerate(nus):
            for i in range(3):
                ref = O.epstein(A, nu, pts_x[i], pts_y[i])
                assert abs(z[j, i] - ref) <= TOL * max(abs(ref), 1.0), (d, nu, i)


def test_epstein_random_points_3d(ez):
    rng = np.random.default_rng(11)
    A = W.bct(1.23)
    x = rng.uniform(-2, 2, size=(37, 3))
    y = rng.uniform(-2, 2, size=(37, 3))
    nus = [-1.0, 1.0, 2.5, 5.0, 9.0]
    z = ez.epstein_zeta(A, nus, x, y).cpu().numpy()
    for j, nu in enumerate(nus):
        for i in range(0, 37, 6):
            ref = O.epstein(A, nu, x[i], y[i])
            assert abs(z[j, i] - ref) <= TOL * max(abs(ref), 1.0), (nu, i)


def test_epstein_empty_batch(ez):
    z = ez.epstein_zeta(np.eye(3), [3.0], np.zeros((0, 3)), np.zeros((0, 3)))
    assert z.shape == (1, 0)


# ---------------------------------------------------------------- quadrature: n-body sums
def test_c1_three_body_1d(ez):
    v = ez.nbody_lattice_sum(np.eye(1), [3, 3, 3], W.SPEC_1D).item()
    ref = O.nbody(np.eye(1), [3, 3, 3], W.SPEC_1D)
    assert rel(v, ref) <= TOL


@pytest.mark.parametrize("d", [1, 2, 3])
def test_atm_small_plans(ez, d):
    lats = {1: [np.eye(1)], 2: [np.eye(2), W.A_HEX], 3: [W.sc(), W.fcc(), W.bcc()]}[d]
    spec = {1: W.SPEC_1D, 2: dict(W.SPEC_2D, n_q=9, n_panels=3, n_g=11), 3: W.SPEC_SMALL_3D}[d]
    A = np.stack(lats)
    got = ez.atm_energy(A, spec).cpu().numpy()
    for i, Ai in enumerate(lats):
        assert rel(got[i], O.atm(Ai, spec)) <= TOL, (d, i)


@pytest.mark.parametrize("nus", [(3, 3), (-1, 5), (1, 3), (6, 6, 6), (3, 5, 7, 9)])
def test_nbody_3d_small_plan(ez, nus):
    spec = dict(W.SPEC_SMALL_3D, n_q=5, n_panels=2, n_g=7)     # 12*25*14 = 4200 nodes: ragged tile
    A = np.stack([W.fcc(), W.bct(0.9)])
    got = ez.nbody_lattice_sum(A, nus, spec).cpu().numpy()
    for i in range(2):
        assert rel(got[i], O.nbody(A[i], nus, spec)) <= TOL, (nus, i)


def test_lattice_sums_multi_result(ez):
    # scan-style program: zeta(nu,nu,nu) for nu in {3,6,9,12} plus ATM, one node pass
    nu = [-1.0, 1.0, 3.0, 5.0, 6.0, 9.0, 12.0]
    terms = [(0, 1.0, [(2, 3)]), (1, 1.0, [(4, 3)]), (2, 1.0, [(5, 3)]), (3, 1.0, [(6, 3)]),
             (4, 1.0 / 24.0, [(2, 3)]), (4, -3.0 / 16.0, [(0, 1), (3, 2)]), (4, 3.0 / 8.0, [(1, 1), (2, 1), (3, 1)])]
    ca = [0.85, 1.0, 1.3]
    A = np.stack([W.bct(c) for c in ca])
    specs = [W.c3_spec(n) for n in (16, 20, 24)]
    got = ez.lattice_sums(A, nu, terms, 5, specs).cpu().numpy()
    for i in range(3):
        for r, nus in enumerate([(3, 3, 3), (6, 6, 6), (9, 9, 9), (12, 12, 12)]):
            assert rel(got[i, r], O.nbody(A[i], nus, specs[i])) <= TOL, (i, r)
        assert rel(got[i, 4], O.atm(A[i], specs[i])) <= TOL, i


def test_bad_lattice_flags_without_failing_batch(ez):
    A = np.stack([W.sc(), np.zeros((3, 3)), W.fcc()])
    out, st = ez.atm_energy(A, W.SPEC_SMALL_3D, with_status=True)
    out = out.cpu().numpy()
    st = st.cpu().numpy()
    assert st[0] == 0 and st[2] == 0 and (st[1] & ez.FLAG_SINGULAR)
    assert np.isnan(out[1]) and np.isfinite(out[0]) and np.isfinite(out[2])
    assert rel(out[2], O.atm(W.fcc(), W.SPEC_SMALL_3D)) <= TOL


def test_determinism(ez):
    A = np.stack([W.sc(), W.bcc()])
    a = ez.atm_energy(A, W.SPEC_SMALL_3D).cpu().numpy()
    b = ez.atm_energy(A, W.SPEC_SMALL_3D).cpu().numpy()
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- full-size three-lattice ATM plan (as timed by bench.py)
def test_c2_full_size_vs_stored_oracle(ez):
    g = json.load(open(os.path.join(GOLD, "oracle_c2_full.json")))
    names = ["sc", "fcc", "bcc"]
    A = np.stack([W.c2_lattices()[n] for n in names])
    got = ez.atm_energy(A, g["spec"]).cpu().numpy()
    for i, n in enumerate(names):
        assert rel(got[i], g["atm"][n]) <= TOL, n


# ---------------------------------------------------------------- ring n-body sums, nu = 6
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_ring_nbody_sums_cubic(ez, n):
    """zeta^(n)_{Z^3}(6, ..., 6) for n = 2..6 (Sec. 2, Definition (many-body zeta))"""
    spec = W.SPEC_SMALL_3D
    got = ez.nbody_lattice_sum(W.sc(), [6.0] * n, spec).item()
    ref = O.nbody(W.sc(), [6.0] * n, spec)
    assert rel(got, ref) <= TOL, (n, got, ref)


def test_ring_two_body_is_epstein_full_plan(ez):
    """zeta^(2)(6, 6) = Z_12(0) (Sec. 2, Corollary) on the full plan"""
    got = ez.nbody_lattice_sum(W.sc(), [6.0, 6.0], W.SPEC_FULL_3D).item()
    ref = O.epstein(W.sc(), 12.0, [0, 0, 0], [0, 0, 0]).real
    assert rel(got, ref) <= TOL


# ---------------------------------------------------------------- the Ewald parameter is the spec's
SKEW_3D = np.array([[1.0, 0.9, 0.3], [0.0, 1.1, 0.6], [0.0, 0.0, 0.9]])


@pytest.mark.parametrize("lam", [0.8, 1.0])
def test_lambda_honoured_small_arguments(ez, lam):
    """spec.lam is used as given: at small lam (and on a skewed lattice) some
    reciprocal terms m* != 0 reach incomplete-gamma arguments below 1/4 near the
    faces and corners of the cell, where the node kernel takes the series forms
    of E_1 and E_{1/2} (the culling's near list); the oracle runs the same split.
    (Below lam ~ 0.7 the split itself is ill-conditioned in FP64: the oracle's
    own ATM values move by 3e-12 between lam = 0.5 and lam = 1.3.)"""
    lats = [W.sc(), W.fcc(), W.bcc(), W.unit_density(SKEW_3D)]
    spec = dict(W.SPEC_SMALL_3D, n_q=5, n_panels=3, n_g=7, lam=lam)
    A = np.stack(lats)
    got = ez.atm_energy(A, spec).cpu().numpy()
    for i, Ai in enumerate(lats):
        assert rel(got[i], O.atm(Ai, spec)) <= TOL, (lam, i)
    # half-integer p (nu = 6 in d = 3) takes the E_{1/2} series on the near list
    got = ez.nbody_lattice_sum(A, [6.0, 6.0, 6.0], spec).cpu().numpy()
    for i, Ai in enumerate(lats):
        v, bar = nbody_bar(Ai, [6.0, 6.0, 6.0], spec)
        assert abs(got[i] - v) <= bar, (lam, i)
