"""Oracle special functions pinned to mpmath (an independent arbitrary-precision
library) and Gauss-Legendre rules pinned to numpy and to polynomial exactness."""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
import oracle as O

mp.mp.dps = 30

S_VALUES = [-4.5, -3.0, -2.0, -1.75, -1.0, -0.5, -0.25, 0.0, 0.5, 0.75, 1.0, 1.5, 2.0, 2.25,
            3.0, 4.5, 5.0, 6.0, 9.0]


@pytest.mark.parametrize("s", S_VALUES)
def test_gamma_upper_vs_mpmath(s):
    # argument range used by the lattice sums: a in (0, ~60]
    worst = 0.0
    for a in np.logspace(-4, np.log10(60.0), 45):
        ref = float(mp.gammainc(s, a))
        worst = max(worst, abs(O.gamma_upper(s, a) - ref) / abs(ref))
    assert worst < 2e-14


def test_e1_vs_mpmath():
    for a in np.concatenate([np.logspace(-6, 0, 20), np.linspace(1.0, 60.0, 40)]):
        ref = float(mp.e1(a))
        assert abs(O.e1(a) - ref) <= 5e-15 * abs(ref)


def test_rgamma_poles_and_values():
    for x in [0.0, -1.0, -2.0, -7.0]:
        assert O.rgamma(x) == 0.0
    for x in [-2.5, -0.5, 0.5, 1.5, 3.0, 6.0]:
        assert abs(O.rgamma(x) - float(mp.rgamma(x))) <= 1e-15 * max(1.0, abs(float(mp.rgamma(x))))


@pytest.mark.parametrize("n", [1, 2, 5, 8, 14, 16, 20, 32, 64])
def test_gauss_legendre_vs_numpy(n):
    x, w = O.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


def test_gauss_legendre_exactness_on_interval():
    # an n-point rule integrates polynomials of degree <= 2n-1 exactly
    n, lo, hi = 9, 0.01, 0.5
    x, w = O.gauss_legendre(n, lo, hi)
    for k in range(2 * n):
        exact = (hi ** (k + 1) - lo ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) <= 1e-15 * max(1.0, abs(exact))
