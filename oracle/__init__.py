"""Plain FP64 CPU oracle for the Epstein zeta method (arXiv 2504.11989).

TEST INFRASTRUCTURE ONLY: this package may be imported by the tests, by the
smoke check in ``__graft_entry__`` and by the CPU-baseline leg of
``bench.py`` -- nothing in the product path may import it.  It shares no
code with the HIP library (``paper_2504_11989_amd``); the C source
``ezo.c`` states the mathematics it follows, section by section.

Functions whose parity has no external pin are listed in ``UNPINNED``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ezo.c")
_LIB = os.path.join(_HERE, "libezo.so")

# every oracle function below has at least one pin in tests/test_oracle_*.py
UNPINNED: tuple = ()

_STATUS = {0: "ok", 1: "invalid argument", 2: "singular lattice", 3: "pole",
           4: "unsupported (Hadamard mu = 0)", 5: "out of memory", 6: "no convergence"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile ezo.c with gcc into oracle/libezo.so (plain -O2, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        D, I, P = ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.ezo_rgamma.restype = D; L.ezo_rgamma.argtypes = [D]
        L.ezo_e1.restype = D; L.ezo_e1.argtypes = [D]
        L.ezo_gamma_upper.restype = D; L.ezo_gamma_upper.argtypes = [D, D]
        L.ezo_gauss_legendre.restype = I; L.ezo_gauss_legendre.argtypes = [I, D, D, P, P]
        L.ezo_epstein.restype = I
        L.ezo_epstein.argtypes = [I, P, D, P, P, D, D, P, P]
        L.ezo_epstein_reg.restype = I
        L.ezo_epstein_reg.argtypes = [I, P, D, P, D, D, P]
        L.ezo_sing.restype = D; L.ezo_sing.argtypes = [I, P, D, P]
        L.ezo_reg_taylor.restype = I
        L.ezo_reg_taylor.argtypes = [I, P, D, P, I, D, D, P]
        L.ezo_hadamard_I.restype = I; L.ezo_hadamard_I.argtypes = [D, I, D, D, P]
        L.ezo_nbody_dirs.restype = I
        L.ezo_nbody_dirs.argtypes = [I, P, I, P, I, I, I, I, D, D, D, I, I, P, P, P]
        L.ezo_nbody.restype = I
        L.ezo_nbody.argtypes = [I, P, I, P, I, I, I, I, D, D, D, P, P]
        L.ezo_atm.restype = I
        L.ezo_atm.argtypes = [I, P, I, I, I, I, D, D, D, P, P]
        L.ezo_direct_nbody.restype = I
        L.ezo_direct_nbody.argtypes = [I, P, I, P, I, P]
        L.ezo_direct_atm.restype = I; L.ezo_direct_atm.argtypes = [I, P, I, P]
        L.ezo_num_threads.restype = I; L.ezo_num_threads.argtypes = []
        L.ezo_set_num_threads.restype = None; L.ezo_set_num_threads.argtypes = [I]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _mat(A):
    A = np.ascontiguousarray(np.atleast_2d(np.asarray(A, dtype=np.float64)))
    d = A.shape[0]
    if A.shape != (d, d) or d not in (1, 2, 3):
        raise ValueError("A must be d x d with d in {1,2,3}")
    return d, A


def _vec(v, d):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
    if v.size != d:
        raise ValueError("vector length must equal d")
    return v


def _check(st):
    if st != 0:
        raise OracleError(_STATUS.get(st, str(st)))


# default plan (paper: n_q = 14, eps = 1e-2, ell = 4)
DEFAULT_SPEC = dict(n_q=14, n_panels=7, n_g=16, ell=4, eps=1e-2, lam=1.0, a_cut=36.0)


def _spec(spec):
    s = dict(DEFAULT_SPEC)
    if spec:
        s.update(spec)
    return s


# ----------------------------------------------------------------- special functions
def rgamma(x: float) -> float:
    return lib().ezo_rgamma(float(x))


def e1(a: float) -> float:
    return lib().ezo_e1(float(a))


def gamma_upper(s: float, a: float) -> float:
    return lib().ezo_gamma_upper(float(s), float(a))


def gauss_legendre(n: int, lo: float = -1.0, hi: float = 1.0):
    x = np.zeros(n); w = np.zeros(n)
    _check(lib().ezo_gauss_legendre(int(n), float(lo), float(hi), _p(x), _p(w)))
    return x, w


# ----------------------------------------------------------------- Epstein zeta
def epstein(A, nu, x, y, lam=1.0, a_cut=36.0) -> complex:
    """Z_{A Z^d, nu}(x, y) by the incomplete-gamma split."""
    d, A = _mat(A)
    x = _vec(x, d); y = _vec(y, d)
    re = ctypes.c_double(); im = ctypes.c_double()
    _check(lib().ezo_epstein(d, _p(A), float(nu), _p(x), _p(y), float(lam), float(a_cut),
                             ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


def epstein_reg(A, nu, k, lam=1.0, a_cut=36.0) -> float:
    """Z^reg_{nu}(k) = Z(0,k) - s_hat(k)/|det A| (also at k = 0)."""
    d, A = _mat(A)
    k = _vec(k, d)
    out = ctypes.c_double()
    _check(lib().ezo_epstein_reg(d, _p(A), float(nu), _p(k), float(lam), float(a_cut), ctypes.byref(out)))
    return out.value


def sing(A, nu, k) -> float:
    """s_hat_nu(k) / |det A|."""
    d, A = _mat(A)
    k = _vec(k, d)
    return lib().ezo_sing(d, _p(A), float(nu), _p(k))


def reg_taylor(A, nu, w, ell=4, lam=1.0, a_cut=36.0):
    """Directional Taylor coefficients C_{k,nu}(w), k = 0..ell, of Z^reg(u w) in u."""
    d, A = _mat(A)
    w = _vec(w, d)
    C = np.zeros(ell + 1)
    _check(lib().ezo_reg_taylor(d, _p(A), float(nu), _p(w), int(ell), float(lam), float(a_cut), _p(C)))
    return C


def hadamard_I(mu, q, eps, Leps) -> float:
    out = ctypes.c_double()
    _check(lib().ezo_hadamard_I(float(mu), int(q), float(eps), float(Leps), ctypes.byref(out)))
    return out.value


# ----------------------------------------------------------------- quadrature
def n_directions(d: int, n_q: int) -> int:
    return d * (1 << (d - 1)) * n_q ** (d - 1)


def nbody(A, nu, spec=None, parts=False):
    """n-body zeta zeta^(n)_Lambda(nu) by the Epstein representation."""
    d, A = _mat(A)
    s = _spec(spec)
    nu = np.ascontiguousarray(np.asarray(nu, dtype=np.float64).reshape(-1))
    out = ctypes.c_double()
    pr = np.zeros(2)
    _check(lib().ezo_nbody(d, _p(A), nu.size, _p(nu), s["n_q"], s["n_panels"], s["n_g"], s["ell"],
                           s["eps"], s["lam"], s["a_cut"], ctypes.byref(out), _p(pr)))
    return (out.value, pr) if parts else out.value


def nbody_dirs(A, nu, spec=None, dir_lo=0, dir_hi=None):
    """Per-direction pieces: (weight, hadamard part, numeric part) for directions
    [dir_lo, dir_hi); zeta = sum weight * (hadamard + numeric)."""
    d, A = _mat(A)
    s = _spec(spec)
    nd = n_directions(d, s["n_q"])
    if dir_hi is None:
        dir_hi = nd
    n = dir_hi - dir_lo
    nu = np.ascontiguousarray(np.asarray(nu, dtype=np.float64).reshape(-1))
    h = np.zeros(n); m = np.zeros(n); w = np.zeros(n)
    _check(lib().ezo_nbody_dirs(d, _p(A), nu.size, _p(nu), s["n_q"], s["n_panels"], s["n_g"], s["ell"],
                                s["eps"], s["lam"], s["a_cut"], int(dir_lo), int(dir_hi),
                                _p(h), _p(m), _p(w)))
    return w, h, m


ATM_TRIPLES = ((3.0, 3.0, 3.0), (-1.0, 5.0, 5.0), (1.0, 3.0, 5.0))
ATM_COEFS = (1.0 / 24.0, -3.0 / 16.0, 3.0 / 8.0)


def atm(A, spec=None, zetas=False):
    """ATM cohesive energy per particle via the three-body recombination."""
    d, A = _mat(A)
    s = _spec(spec)
    out = ctypes.c_double()
    z = np.zeros(3)
    _check(lib().ezo_atm(d, _p(A), s["n_q"], s["n_panels"], s["n_g"], s["ell"], s["eps"],
                         s["lam"], s["a_cut"], ctypes.byref(out), _p(z)))
    return (out.value, z) if zetas else out.value


# ----------------------------------------------------------------- direct sums
def direct_nbody(A, nu, L: int) -> float:
    d, A = _mat(A)
    nu = np.ascontiguousarray(np.asarray(nu, dtype=np.float64).reshape(-1))
    out = ctypes.c_double()
    _check(lib().ezo_direct_nbody(d, _p(A), nu.size, _p(nu), int(L), ctypes.byref(out)))
    return out.value


def direct_atm(A, L: int) -> float:
    d, A = _mat(A)
    out = ctypes.c_double()
    _check(lib().ezo_direct_atm(d, _p(A), int(L), ctypes.byref(out)))
    return out.value


def num_threads() -> int:
    return lib().ezo_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (for timing it as a CPU baseline)."""
    lib().ezo_set_num_threads(int(n))


# ----------------------------------------------------------------- derivatives
def grad_fd(f, A, h: float = 1e-3) -> np.ndarray:
    """d f / d A_ij of a scalar function of the generator matrix by the
    fourth-order central difference
        (f(A - 2h E_ij) - 8 f(A - h E_ij) + 8 f(A + h E_ij) - f(A + 2h E_ij)) / (12 h),
    truncation error h^4 f^(5) / 30.  With f an oracle lattice sum on a fixed plan
    this is the derivative of the oracle's value on that plan (nodes fixed in
    fractional coordinates, which is how the plan is defined)."""
    A = np.array(A, dtype=np.float64)
    d = A.shape[0]
    g = np.zeros((d, d))
    for i in range(d):
        for j in range(d):
            vals = []
            for s in (-2, -1, 1, 2):
                B = A.copy()
                B[i, j] += s * h
                vals.append(f(B))
            g[i, j] = (vals[0] - 8.0 * vals[1] + 8.0 * vals[2] - vals[3]) / (12.0 * h)
    return g
