"""MI355X (gfx950) implementation of the Epstein zeta method for many-body
lattice sums (Buchheit & Busse, arXiv 2504.11989).

Thin Python layer over libezeta.so (see include/ezeta.h): torch tensors on the
GPU are passed to the C ABI as device pointers on torch's current stream.

    epstein_zeta(A, nu, x, y)        Z_{A Z^d, nu}(x, y), complex
    epstein_grid(A, nu, xs, ys)      Z on every (shift, point) pair, FP64 or mixed precision
    nbody_lattice_sum(A, nu, spec)   zeta^(n)_Lambda(nu) for a batch of lattices
    atm_energy(A, spec)              ATM cohesive energy per particle (and dE/dA)
    lattice_sums(A, nu, terms, ...)  several product integrals per lattice (and d/dA)

Differentiable forms (torch.autograd.Function over the adjoint kernels) are in
paper_2504_11989_amd.autograd; the LJ + ATM enthalpy and its minimisation in
paper_2504_11989_amd.enthalpy.
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Sequence

from ._native import (FLAG_CAPACITY, FLAG_HADAMARD, FLAG_NONFINITE, FLAG_POLE, FLAG_SINGULAR,
                      PREC_FP64, PREC_MIXED, EzError, QuadSpec, check, lib)

__all__ = ["epstein_zeta", "epstein_grid", "nbody_lattice_sum", "atm_energy", "lattice_sums", "QuadSpec", "EzError",
           "DEFAULT_SPEC", "FLAG_SINGULAR", "FLAG_CAPACITY", "FLAG_NONFINITE", "FLAG_HADAMARD",
           "FLAG_POLE", "version", "finalize"]

# paper: n_q = 14, eps = 1e-2, ell = 4;  7 x 16 u-nodes on (eps, 1/2]
DEFAULT_SPEC = dict(n_q=14, n_panels=7, n_g=16, ell=4, eps=1e-2, lam=1.0, a_cut=36.0, precision=PREC_FP64)


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_f64(t, device=None):
    torch = _torch()
    t = torch.as_tensor(t, dtype=torch.float64, device=device if device is not None else "cuda")
    return t.contiguous()


def _host_f64(seq):
    vals = [float(v) for v in seq]
    return (ctypes.c_double * max(1, len(vals)))(*vals), len(vals)


def _spec(spec) -> QuadSpec:
    if spec is None:
        return QuadSpec.from_dict(DEFAULT_SPEC)
    if isinstance(spec, QuadSpec):
        return spec
    s = dict(DEFAULT_SPEC)
    s.update(spec)
    return QuadSpec.from_dict(s)


def _lattices(A):
    """A: (d, d) or (batch, d, d) tensor/array -> contiguous float64 CUDA tensor (batch, d, d)."""
    torch = _torch()
    A = _dev_f64(A)
    if A.dim() == 2:
        A = A.unsqueeze(0)
    if A.dim() != 3 or A.shape[1] != A.shape[2] or A.shape[1] not in (1, 2, 3):
        raise ValueError("A must have shape (d, d) or (batch, d, d), d in {1,2,3}")
    return A.contiguous(), int(A.shape[0]), int(A.shape[1])


def epstein_zeta(A, nu: Sequence[float], x, y, lam: float = 0.0, a_cut: float = 0.0, with_status=False):
    """Z_{A Z^d, nu_j}(x_i, y_i) for all j, i: complex128 tensor (len(nu), n_pts)."""
    torch = _torch()
    A, b, d = _lattices(A)
    if b != 1:
        raise ValueError("epstein_zeta takes one lattice")
    x = _dev_f64(x, A.device).reshape(-1, d).contiguous()
    y = _dev_f64(y, A.device).reshape(-1, d).contiguous()
    if x.shape != y.shape:
        raise ValueError("x and y must have the same number of points")
    n = x.shape[0]
    nu_h, n_nu = _host_f64(nu)
    out = torch.empty((n_nu, n, 2), dtype=torch.float64, device=A.device)
    st = torch.zeros(1, dtype=torch.int32, device=A.device)
    check(lib().ez_epstein_zeta(d, _dptr(A), n_nu, nu_h, n, _dptr(x), _dptr(y), float(lam), float(a_cut),
                                _dptr(out), _dptr(st), _stream_ptr(A.device)))
    z = torch.view_as_complex(out)
    return (z, st) if with_status else z


def epstein_grid(A, nu: Sequence[float], x, y, lam: float = 0.0, a_cut: float = 0.0, mixed: bool = False,
                 with_bound: bool = False, with_status: bool = False):
    """Z_{A Z^d, nu_k}(x_j, y_m) for every exponent, shift and point: complex128
    tensor (len(nu), n_x, n_y).  mixed=True: split-BF16 products for the far table
    entries (see include/ezeta.h); with_bound also returns the a-priori bound as
    float64 (len(nu), n_x + n_y): |Z_mixed - Z_fp64| at (nu_k, x_j, y_m) is at most
    b[k, j] + b[k, n_x + m]."""
    torch = _torch()
    A, b, d = _lattices(A)
    if b != 1:
        raise ValueError("epstein_grid takes one lattice")
    x = _dev_f64(x, A.device).reshape(-1, d).contiguous()
    y = _dev_f64(y, A.device).reshape(-1, d).contiguous()
    nu_h, n_nu = _host_f64(nu)
    out = torch.empty((n_nu, x.shape[0], y.shape[0], 2), dtype=torch.float64, device=A.device)
    bound = torch.empty((n_nu, x.shape[0] + y.shape[0]), dtype=torch.float64, device=A.device) if with_bound else None
    st = torch.zeros(1, dtype=torch.int32, device=A.device)
    check(lib().ez_epstein_grid(d, _dptr(A), n_nu, nu_h, x.shape[0], _dptr(x), y.shape[0], _dptr(y), float(lam),
                                float(a_cut), PREC_MIXED if mixed else PREC_FP64, _dptr(out),
                                _dptr(bound) if with_bound else None, _dptr(st), _stream_ptr(A.device)))
    z = torch.view_as_complex(out)
    ret = (z,)
    if with_bound:
        ret = ret + (bound,)
    if with_status:
        ret = ret + (st,)
    return ret if len(ret) > 1 else ret[0]


def nbody_lattice_sum(A, nu: Sequence[float], spec=None, with_status=False):
    """zeta^(n)_Lambda(nu) for each lattice of the batch: float64 tensor (batch,)."""
    torch = _torch()
    A, b, d = _lattices(A)
    nu_h, n = _host_f64(nu)
    sp = _spec(spec)
    out = torch.empty(b, dtype=torch.float64, device=A.device)
    st = torch.empty(b, dtype=torch.int32, device=A.device)
    check(lib().ez_nbody_lattice_sum(b, d, _dptr(A), n, nu_h, ctypes.byref(sp), _dptr(out), _dptr(st),
                                     _stream_ptr(A.device)))
    return (out, st) if with_status else out


def atm_energy(A, spec=None, with_status=False, grad=False):
    """ATM cohesive energy per particle for each lattice of the batch: float64 (batch,).
    grad=True also returns dE/dA, float64 (batch, d, d)."""
    torch = _torch()
    A, b, d = _lattices(A)
    sp = _spec(spec)
    out = torch.empty(b, dtype=torch.float64, device=A.device)
    st = torch.empty(b, dtype=torch.int32, device=A.device)
    g = torch.empty((b, d, d), dtype=torch.float64, device=A.device) if grad else None
    check(lib().ez_atm_energy(b, d, _dptr(A), ctypes.byref(sp), _dptr(out), _dptr(g) if grad else None,
                              _dptr(st), _stream_ptr(A.device)))
    ret = (out, g) if grad else (out,)
    if with_status:
        ret = ret + (st,)
    return ret if len(ret) > 1 else ret[0]


def lattice_sums(A, nu: Sequence[float], terms: Iterable, n_results: int, specs=None, with_status=False,
                 grad=False, out=None, status=None, noalloc=False, with_bound=False):
    """Several results per lattice, result_r = sum of coef * V int_BZ prod Z_nu^mult dk.

    terms: iterable of (result_index, coef, [(nu_index, multiplicity), ...]).
    specs: None, one spec, or a list with one spec per lattice.
    Returns float64 tensor (batch, n_results); grad=True (n_results <= 2) also
    returns the derivatives with respect to A, float64 (batch, n_results, d, d).
    out / status: optional preallocated result (batch, n_results) float64 and
    status (batch,) int32 tensors (nothing is allocated then, e.g. under graph capture).
    noalloc=True calls ez_lattice_sums_noalloc: the library allocates no device
    memory for the call (its intermediates live in a static 64 MiB array per GPU);
    values only.
    with_bound=True calls ez_lattice_sums_bound and also returns the a-priori bound
    of each result's mixed-precision error, float64 (batch, n_results) (zero for
    FP64 specs; specs with precision=PREC_MIXED select the mixed form)."""
    torch = _torch()
    A, b, d = _lattices(A)
    nu_h, n_nu = _host_f64(nu)
    terms = list(terms)
    nt = len(terms)
    res = (ctypes.c_int * max(1, nt))()
    coef = (ctypes.c_double * max(1, nt))()
    nfac = (ctypes.c_int * max(1, nt))()
    fac = (ctypes.c_int * max(4, 4 * nt))()
    mult = (ctypes.c_int * max(4, 4 * nt))()
    for t, (r, c, fl) in enumerate(terms):
        res[t] = int(r)
        coef[t] = float(c)
        fl = list(fl)
        nfac[t] = len(fl)
        if len(fl) > 4:
            raise ValueError("at most 4 distinct factors per term")
        for f, (i, m) in enumerate(fl):
            fac[4 * t + f] = int(i)
            mult[4 * t + f] = int(m)
    if specs is None or isinstance(specs, (dict, QuadSpec)):
        sp_list = [_spec(specs)]
    else:
        sp_list = [_spec(s) for s in specs]
    sp_arr = (QuadSpec * len(sp_list))(*sp_list)
    if out is None:
        out = torch.empty((b, n_results), dtype=torch.float64, device=A.device)
    elif out.shape != (b, n_results) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape (batch, n_results)")
    if status is None:
        st = torch.empty(b, dtype=torch.int32, device=A.device)
    elif status.shape != (b,) or status.dtype != torch.int32:
        raise ValueError("status must be an int32 tensor of shape (batch,)")
    else:
        st = status
    if noalloc:
        if grad:
            raise ValueError("the no-allocation entry point computes values only")
        check(lib().ez_lattice_sums_noalloc(b, d, _dptr(A), n_nu, nu_h, nt, res, coef, nfac, fac, mult,
                                            int(n_results), sp_arr, len(sp_list), _dptr(out), _dptr(st),
                                            _stream_ptr(A.device)))
        return (out, st) if with_status else out
    if with_bound:
        if grad or noalloc:
            raise ValueError("with_bound computes values only")
        bound = torch.empty((b, n_results), dtype=torch.float64, device=A.device)
        check(lib().ez_lattice_sums_bound(b, d, _dptr(A), n_nu, nu_h, nt, res, coef, nfac, fac, mult,
                                          int(n_results), sp_arr, len(sp_list), _dptr(out), _dptr(bound), _dptr(st),
                                          _stream_ptr(A.device)))
        return (out, bound, st) if with_status else (out, bound)
    g = torch.empty((b, n_results, d, d), dtype=torch.float64, device=A.device) if grad else None
    check(lib().ez_lattice_sums_grad(b, d, _dptr(A), n_nu, nu_h, nt, res, coef, nfac, fac, mult, int(n_results),
                                     sp_arr, len(sp_list), _dptr(out), _dptr(g) if grad else None, _dptr(st),
                                     _stream_ptr(A.device)))
    ret = (out, g) if grad else (out,)
    if with_status:
        ret = ret + (st,)
    return ret if len(ret) > 1 else ret[0]


def direct_atm(A, L: int, symmetry: bool = False) -> float:
    """ATM cohesive energy by direct summation over the box A{-L..L}^d on the GPU
    (ez_direct_atm); symmetry=True for square / cubic lattices."""
    import numpy as np
    torch = _torch()
    A_np = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    d = A_np.shape[0]
    if A_np.shape != (d, d):
        raise ValueError("A must be d x d")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    check(lib().ez_direct_atm(d, A_np.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(L), 1 if symmetry else 0,
                              _dptr(out), _stream_ptr(out.device)))
    return out.item()


def version() -> str:
    return lib().ez_version().decode()


def finalize():
    check(lib().ez_finalize())
