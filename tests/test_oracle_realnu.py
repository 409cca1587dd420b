"""Pins of the oracle at non-integer exponents (paper, Sec. 4.3: the one-dimensional
three-body zeta function and its meromorphic continuation in nu), against
references that share nothing with the Crandall split:

* Z_{Z,nu}(0, y) = 2 Re Li_nu(e^{2 pi i y}) (polylogarithm, mpmath);
* the series Z_{Z,nu}(k) = s_nu(k) + sum_n (-1)^n (2 pi k)^{2n} / (2n)! 2 zeta(nu - 2n),
  s_nu(k) = pi^{nu - 1/2} Gamma((1 - nu)/2) / Gamma(nu/2) |k|^{nu - 1} (the paper's 1-D
  series, read as in the design notes; it converges for |k| < 1, with terms falling
  like 4^{-n} at k = 1/2, and matches the polylogarithm to 1e-15, checked below).
  The products of the series integrate term by term: the continuation of
  int_0^{1/2} k^e dk is 2^{-(e+1)} / (e + 1), so
  zeta^(3) = 2 int_0^{1/2} prod_i Z_{nu_i}(k) dk needs no quadrature."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W

mp = pytest.importorskip("mpmath")


def z_polylog(nu, k):
    return 2 * mp.re(mp.polylog(nu, mp.exp(2j * mp.pi * k)))


def z_series(nu, k, N=60):
    A = mp.pi ** (nu - mp.mpf(1) / 2) * mp.gamma((1 - nu) / 2) / mp.gamma(nu / 2)
    s = A * abs(k) ** (nu - 1)
    for n in range(N + 1):
        s += (-1) ** n * (2 * mp.pi * k) ** (2 * n) / mp.factorial(2 * n) * 2 * mp.zeta(nu - 2 * n)
    return s


def zeta_n_1d(nus, N=60):
    mp.mp.dps = 30
    nus = [mp.mpf(v) for v in nus]
    half = mp.mpf(1) / 2
    A = [mp.pi ** (v - half) * mp.gamma((1 - v) / 2) / mp.gamma(v / 2) for v in nus]
    R = [[(-1) ** n * (2 * mp.pi) ** (2 * n) / mp.factorial(2 * n) * 2 * mp.zeta(v - 2 * n) for n in range(N + 1)]
         for v in nus]
    tot = mp.mpf(0)
    for S in itertools.product([0, 1], repeat=len(nus)):
        coef, E, poly = mp.mpf(1), mp.mpf(0), [mp.mpf(1)]
        for i, v in enumerate(nus):
            if S[i]:
                coef *= A[i]
                E += v - 1
            else:
                new = [mp.mpf(0)] * (N + 1)
                for a_, pa in enumerate(poly):
                    for b_, rb in enumerate(R[i][:N + 1 - a_]):
                        new[a_ + b_] += pa * rb
                poly = new
        for m, c in enumerate(poly):
            e1 = E + 2 * m + 1
            tot += coef * c * half ** e1 / e1
    return float(2 * tot)


def test_series_matches_polylog():
    mp.mp.dps = 30
    for nu in (0.52, 2.52, -0.98, 3.02):
        for k in (0.05, 0.3, 0.5):
            a, b = z_series(mp.mpf(nu), mp.mpf(k)), z_polylog(mp.mpf(nu), mp.mpf(k))
            assert abs(a - b) <= 1e-14 * abs(b), (nu, k)


@pytest.mark.parametrize("nu", [-1.98, -0.48, 0.52, 0.98, 1.02, 2.52, 2.98, 3.02, 4.52])
def test_epstein_1d_polylog(nu):
    """Z at non-integer nu, also next to nu = d + 2m where the singular coefficient's
    Gamma((d - nu)/2) is large and the incomplete gamma of the split nears a pole"""
    mp.mp.dps = 30
    for y in (0.03, 0.2, 0.5):
        ref = float(z_polylog(nu, y))
        for lam in (0.8, 1.0, 1.3):
            got = O.epstein(np.eye(1), nu, [0.0], [y], lam=lam).real
            assert abs(got - ref) <= 2e-14 * abs(ref), (nu, y, lam, got, ref)


@pytest.mark.parametrize("nus", [(2.52, 3.02, 4.52), (1.52, 1.52, 2.02), (0.52, 0.52, 0.52),
                                 (-1.98, 2.52, 2.52), (-0.98, 1.02, 2.52)])
def test_three_body_1d_continuation(nus):
    """zeta^(3)_Z(nu) at non-integer nu: integrable cases and points of the
    meromorphic continuation (sum (nu_i - 1) < -1)"""
    ref = zeta_n_1d(nus)
    got = O.nbody(np.eye(1), list(nus), W.SPEC_1D)
    assert abs(got - ref) <= 1e-13 * abs(ref), (nus, got, ref)
