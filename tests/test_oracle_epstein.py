"""Oracle Epstein zeta (incomplete-gamma split) pinned to closed forms, number
theory, the functional equation, direct sums and the paper's decomposition."""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
import oracle as O
import workloads as W

mp.mp.dps = 30
Z1 = np.array([[1.0]])


def lerch_ref(nu, x, y):
    # Z_{Z,nu}(x,y) = Phi(e^{2 pi i y}, nu, x) + e^{-2 pi i y} Phi(e^{-2 pi i y}, nu, 1-x), 0<x<1
    e = mp.exp(2j * mp.pi * y)
    return complex(mp.lerchphi(e, nu, x) + mp.exp(-2j * mp.pi * y) * mp.lerchphi(1 / e, nu, 1 - x))


def test_c1_spot_values_vs_lerch():
    nus, xs, ys = W.c1_spot_values()
    for nu, x, y in zip(nus, xs, ys):
        z = O.epstein(Z1, nu, [x], [y])
        ref = lerch_ref(nu, x, y)
        assert abs(z - ref) <= 1e-14 * abs(ref), (nu, x, y)


@pytest.mark.parametrize("nu", [-3.0, -1.0, -0.5, 0.5, 1.5, 2.0, 3.0, 4.5, 6.0, 12.0])
def test_1d_origin_is_2zeta(nu):
    # Z_{Z,nu}(0,0) = 2 zeta(nu) (meromorphic continuation for nu < 1)
    ref = 2.0 * float(mp.zeta(nu))
    assert abs(O.epstein(Z1, nu, [0.0], [0.0]).real - ref) <= 2e-15 * abs(ref)


@pytest.mark.parametrize("nu", [-1.0, 1.5, 2.0, 3.0, 4.5])
def test_1d_half_is_eta(nu):
    # Z_{Z,nu}(0,1/2) = -2 (1 - 2^{1-nu}) zeta(nu)
    ref = float(-2.0 * (1.0 - mp.mpf(2) ** (1.0 - nu)) * mp.zeta(nu))
    assert abs(O.epstein(Z1, nu, [0.0], [0.5]).real - ref) <= 1e-14 * abs(ref)


@pytest.mark.parametrize("nu", [1.5, 3.0, 4.5])
def test_1d_shift_is_hurwitz(nu):
    # Z_{Z,nu}(x,0) = zeta(nu,x) + zeta(nu,1-x)
    for x in [0.1, 0.37, 0.8]:
        ref = float(mp.zeta(nu, x) + mp.zeta(nu, 1 - x))
        assert abs(O.epstein(Z1, nu, [x], [0.0]).real - ref) <= 2e-15 * abs(ref)


def test_1d_polylog_and_elementary():
    for y in [0.05, 0.21, 0.5, 0.77]:
        # Z_{Z,nu}(0,y) = 2 Re Li_nu(e^{2 pi i y})
        for nu in [0.5, 2.5, 3.0]:
            ref = 2.0 * float(mp.re(mp.polylog(nu, mp.exp(2j * mp.pi * y))))
            assert abs(O.epstein(Z1, nu, [0.0], [y]).real - ref) <= 1e-14 * max(1.0, abs(ref))
        # Z_{Z,-1}(0,y) = -1/(2 sin^2 pi y);  Z_{Z,2}(0,y) = 2 pi^2 (y^2 - y + 1/6)
        assert abs(O.epstein(Z1, -1.0, [0.0], [y]).real + 0.5 / np.sin(np.pi * y) ** 2) < 1e-13
        assert abs(O.epstein(Z1, 2.0, [0.0], [y]).real - 2 * np.pi ** 2 * (y * y - y + 1 / 6)) < 1e-13


@pytest.mark.parametrize("s", [1.5, 2.0, 3.0, 4.5])
def test_2d_square_and_hex_lattice_sums(s):
    # Z_{Z^2,2s}(0,0) = 4 zeta(s) beta(s);  Z_{hex,2s}(0,0) = 6 zeta(s) L(s, chi_{-3})
    sq = 4.0 * float(mp.zeta(s) * mp.dirichlet(s, [0, 1, 0, -1]))
    hx = 6.0 * float(mp.zeta(s) * mp.dirichlet(s, [0, 1, -1]))
    assert abs(O.epstein(np.eye(2), 2 * s, [0, 0], [0, 0]).real - sq) <= 2e-15 * sq
    assert abs(O.epstein(W.A_HEX, 2 * s, [0, 0], [0, 0]).real - hx) <= 2e-15 * hx


@pytest.mark.parametrize("name", ["sc", "fcc", "bcc"])
def test_3d_functional_equation_and_periodicity(name):
    A = W.c2_lattices()[name]
    d = 3
    B = np.linalg.inv(A).T
    V = abs(np.linalg.det(A))
    x = np.array([0.1, 0.25, -0.3])
    y = np.array([0.2, -0.1, 0.05])
    for nu in [-1.0, 1.0, 2.5, 4.0, 6.0]:     # nu - d in 2N0 is a pole of the prefactor
        lhs = O.epstein(A, nu, x, y)
        pref = complex(mp.pi ** (nu - d / 2) * mp.gamma((d - nu) / 2) / mp.gamma(nu / 2) / V)
        rhs = pref * np.exp(-2j * np.pi * (x @ y)) * O.epstein(B, d - nu, y, -x)
        assert abs(lhs - rhs) <= 1e-14 * abs(lhs)
        # periodic in y with Lambda*, quasi-periodic in x with Lambda
        m = B @ np.array([1, -2, 1])
        assert abs(O.epstein(A, nu, x, y + m) - lhs) <= 1e-13 * abs(lhs)
        z0 = A @ np.array([2, 0, -1])
        assert abs(O.epstein(A, nu, x + z0, y) - np.exp(-2j * np.pi * (y @ z0)) * lhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("name", ["sc", "fcc", "bcc"])
def test_lambda_invariance_and_bound(name):
    A = W.c2_lattices()[name]
    k = np.array([0.13, -0.21, 0.07])
    for nu in [-1.0, 1.0, 3.0, 5.0, 6.0, 9.0, 12.0]:
        # a wider cutoff (48) so that the truncation is negligible at every lam tried;
        # lam well below 1 makes the self term large for large nu (cancellation), so
        # the check stays at lam >= 0.9
        z = O.epstein(A, nu, np.zeros(3), k, lam=1.0, a_cut=48.0)
        for lam in [0.9, 1.6]:
            assert abs(O.epstein(A, nu, np.zeros(3), k, lam=lam, a_cut=48.0) - z) <= 3e-14 * abs(z)
        assert abs(z.imag) <= 1e-15 * abs(z)          # real at x = 0
        if nu > 3:                                    # |Z(0,k)| <= Z(0,0) for nu > d
            assert abs(z) <= O.epstein(A, nu, np.zeros(3), np.zeros(3)).real


def test_3d_direct_sum_large_nu():
    # Z_{Lambda,12}(0,0) by brute force over the box |n|_inf <= L.  Every omitted
    # point has |A n| >= R0 = L sigma_min(A); with mu = (|a1|+|a2|+|a3|)/2 a bound
    # on the covering radius, the tail is at most 4 pi (R0 - mu)^{-9} / (9 V).
    import math
    L = 40
    for name, A in W.c2_lattices().items():
        n = np.arange(-L, L + 1)
        N = np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3)
        N = N[np.any(N != 0, axis=1)]
        r2 = np.sum((N @ A.T) ** 2, axis=1)
        direct = math.fsum(r2 ** -6.0)
        R0 = L * np.linalg.svd(A, compute_uv=False).min()
        mu = 0.5 * np.linalg.norm(A, axis=0).sum()
        tail = 4 * np.pi * (R0 - mu) ** -9 / (9 * abs(np.linalg.det(A)))
        z = O.epstein(A, 12.0, np.zeros(3), np.zeros(3)).real
        assert 0.0 <= z - direct <= tail + 1e-14 * direct, name


@pytest.mark.parametrize("nu", [-1.0, 0.5, 2.5, 4.0, 6.0])
def test_1d_regular_taylor_series(nu):
    # Z_{Z,nu}(k) = s_hat(k) + sum_n (-1)^n (2 pi k)^{2n}/(2n)! 2 zeta(nu - 2n), nu not in 1+2N0
    C = O.reg_taylor(Z1, nu, [1.0], ell=6)
    for n in range(7):
        ref = (-1) ** n * (2 * np.pi) ** (2 * n) / float(mp.factorial(2 * n)) * 2.0 * float(mp.zeta(nu - 2 * n))
        # high orders carry more cancellation; they enter the Hadamard part with eps^{2n}
        assert abs(C[n] - ref) <= 1e-14 * 4 ** n * max(abs(ref), 1.0), (nu, n)


@pytest.mark.parametrize("name", ["sc", "fcc", "bcc"])
def test_3d_taylor_matches_regular_part(name):
    # the multinomial Taylor polynomial of Z^reg reproduces Z(0,k) - s_hat(k)/V at small k
    A = W.c2_lattices()[name]
    w = np.linalg.inv(A).T @ np.array([0.3, -0.6, 1.0])
    for nu in [-1.0, 1.0, 3.0, 5.0]:
        C = O.reg_taylor(A, nu, w, ell=6)
        for u in [0.02, 0.05]:
            k = u * w
            full = O.epstein(A, nu, np.zeros(3), k).real - O.sing(A, nu, k)
            reg = O.epstein_reg(A, nu, k)
            taylor = sum(C[j] * u ** (2 * j) for j in range(7))
            scale = max(1.0, abs(reg))
            assert abs(reg - taylor) <= 1e-13 * scale, (nu, u)
            # subtraction of the large singular part loses digits near k = 0
            assert abs(full - reg) <= 1e-15 * max(1.0, abs(O.sing(A, nu, k))) * 50


def test_singular_part_closed_forms():
    # s_hat for nu = d + 2m carries log(pi k^2); d = 3, nu = 3: -2 pi log(pi k^2) / V
    A = W.sc()
    k = np.array([0.03, 0.01, -0.02])
    k2 = k @ k
    assert abs(O.sing(A, 3.0, k) - (-2 * np.pi * np.log(np.pi * k2))) < 1e-13
    # nu = -1, d = 3: pi^{-5/2} Gamma(2)/Gamma(-1/2) |k|^-4
    ref = np.pi ** -2.5 * 1.0 / float(mp.gamma(-0.5)) * k2 ** -2
    assert abs(O.sing(A, -1.0, k) - ref) <= 1e-14 * abs(ref)
