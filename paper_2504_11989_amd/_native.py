"""ctypes binding of libezeta.so (argument marshalling only).

Every numerical step runs in the HIP kernels of the library.  PyTorch is used
for device memory and streams: tensors are passed as raw device pointers and
the call is enqueued on torch's current HIP stream.  There is no CPU fallback:
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libezeta.so")

EZ_OK = 0
STATUS_NAMES = {0: "EZ_OK", 1: "EZ_ERR_INVALID_ARG", 2: "EZ_ERR_SINGULAR_LATTICE", 3: "EZ_ERR_POLE",
                4: "EZ_ERR_UNSUPPORTED", 5: "EZ_ERR_NOMEM", 6: "EZ_ERR_HIP"}
FLAG_SINGULAR, FLAG_CAPACITY, FLAG_NONFINITE, FLAG_HADAMARD, FLAG_POLE = 0x1, 0x2, 0x4, 0x8, 0x10
PREC_FP64, PREC_MIXED = 0, 1
SPEC_PERSISTENT, SPEC_SERIAL, SPEC_NO_SPLIT = 0x1, 0x2, 0x4


def spec_bpc(n: int) -> int:
    """spec.flags bits for n persistent workgroups per CU (0: as many as fit)"""
    return (int(n) & 0xFF) << 8


def spec_wave_u(k: int) -> int:
    """spec.flags bits for wave blocks of 2^(k+2) u-nodes x 2^(4-k) directions (k = 1..4; 0: automatic)"""
    return (int(k) & 0x7) << 24


def spec_mix_a(n: int) -> int:
    """spec.flags bits for the mixed-precision threshold a_mix = n (n >= 8; 0: 16)"""
    return (int(n) & 0xFF) << 16

# every symbol declared in include/ezeta.h
EXPORTED = ("ez_epstein_zeta", "ez_epstein_grid", "ez_nbody_lattice_sum", "ez_atm_energy", "ez_lattice_sums", "ez_lattice_sums_grad",
            "ez_timing_enable", "ez_timing_reset", "ez_timing_read",
            "ez_last_error", "ez_finalize", "ez_version", "ez_workspace_generation", "ez_lattice_sums_noalloc",
            "ez_lattice_sums_bound", "ez_direct_atm", "ez_grid_last_tables",
            "ez_last_sum_tiles")
(KERNEL_SETUP, KERNEL_NODES, KERNEL_HADAMARD, KERNEL_FINALIZE, KERNEL_EPSTEIN, KERNEL_NODES_ADJ, KERNEL_GRID,
 KERNEL_NODES_TAIL, KERNEL_TAYLOR, KERNEL_GRID_GEMM) = (0, 1, 2, 3, 4, 5, 6, 7, 8, 9)


class EzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class QuadSpec(ctypes.Structure):
    """Mirror of ez_quad_spec (include/ezeta.h)."""
    _fields_ = [("n_q", ctypes.c_int32), ("n_panels", ctypes.c_int32), ("n_g", ctypes.c_int32),
                ("ell", ctypes.c_int32), ("eps", ctypes.c_double), ("lam", ctypes.c_double),
                ("a_cut", ctypes.c_double), ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]

    @classmethod
    def from_dict(cls, s: dict) -> "QuadSpec":
        return cls(int(s.get("n_q", 14)), int(s.get("n_panels", 7)), int(s.get("n_g", 16)),
                   int(s.get("ell", 4)), float(s.get("eps", 1e-2)), float(s.get("lam", 1.0)),
                   float(s.get("a_cut", 36.0)), int(s.get("precision", PREC_FP64)), int(s.get("flags", 0)))


_lib = None


def lib():
    """Load libezeta.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    I, D, P, VP = ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    I64 = ctypes.c_int64
    L.ez_epstein_zeta.restype = I
    L.ez_epstein_zeta.argtypes = [I, VP, I, P, I64, VP, VP, D, D, VP, VP, VP]
    L.ez_epstein_grid.restype = I
    L.ez_epstein_grid.argtypes = [I, VP, I, P, I, VP, I, VP, D, D, I, VP, VP, VP, VP]
    L.ez_nbody_lattice_sum.restype = I
    L.ez_nbody_lattice_sum.argtypes = [I, I, VP, I, P, ctypes.POINTER(QuadSpec), VP, VP, VP]
    L.ez_atm_energy.restype = I
    L.ez_atm_energy.argtypes = [I, I, VP, ctypes.POINTER(QuadSpec), VP, VP, VP, VP]
    IP = ctypes.POINTER(ctypes.c_int)
    L.ez_lattice_sums.restype = I
    L.ez_lattice_sums.argtypes = [I, I, VP, I, P, I, IP, P, IP, IP, IP, I, ctypes.POINTER(QuadSpec), I,
                                  VP, VP, VP]
    L.ez_lattice_sums_noalloc.restype = I
    L.ez_lattice_sums_noalloc.argtypes = [I, I, VP, I, P, I, IP, P, IP, IP, IP, I, ctypes.POINTER(QuadSpec), I,
                                          VP, VP, VP]
    L.ez_lattice_sums_grad.restype = I
    L.ez_lattice_sums_grad.argtypes = [I, I, VP, I, P, I, IP, P, IP, IP, IP, I, ctypes.POINTER(QuadSpec), I,
                                       VP, VP, VP, VP]
    L.ez_direct_atm.restype = I
    L.ez_direct_atm.argtypes = [I, P, I, I, VP, VP]
    L.ez_lattice_sums_bound.restype = I
    L.ez_lattice_sums_bound.argtypes = [I, I, VP, I, P, I, IP, P, IP, IP, IP, I, ctypes.POINTER(QuadSpec), I,
                                        VP, VP, VP, VP]
    L.ez_last_error.restype = ctypes.c_char_p
    L.ez_last_error.argtypes = []
    L.ez_finalize.restype = I
    L.ez_finalize.argtypes = []
    L.ez_version.restype = ctypes.c_char_p
    L.ez_version.argtypes = []
    L.ez_workspace_generation.restype = ctypes.c_uint64
    L.ez_workspace_generation.argtypes = []
    L.ez_timing_enable.restype = I
    L.ez_timing_enable.argtypes = [I]
    L.ez_timing_reset.restype = I
    L.ez_timing_reset.argtypes = []
    L.ez_timing_read.restype = I
    L.ez_timing_read.argtypes = [I, P, ctypes.POINTER(I64)]
    L.ez_grid_last_tables.restype = I
    L.ez_grid_last_tables.argtypes = [ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.ez_last_sum_tiles.restype = I
    L.ez_last_sum_tiles.argtypes = [ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I)]
    _lib = L
    return L


def check(code: int):
    if code != EZ_OK:
        raise EzError(code, lib().ez_last_error().decode())


def timing_enable(on: bool = True):
    check(lib().ez_timing_enable(1 if on else 0))


def timing_reset():
    check(lib().ez_timing_reset())


def timing_read(kernel: int):
    """(total milliseconds, launches) recorded for one kernel kind."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(lib().ez_timing_read(int(kernel), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def last_sum_tiles():
    """(n_tiles, n_main, tail_mode) of the last lattice-sum call on the current device:
    tail_mode 0 none, 1 split kernel, 2 half-term workgroups in the tile kernel."""
    a = ctypes.c_int64()
    b = ctypes.c_int64()
    m = ctypes.c_int()
    check(lib().ez_last_sum_tiles(ctypes.byref(a), ctypes.byref(b), ctypes.byref(m)))
    return a.value, b.value, m.value


def grid_last_tables():
    """(n_real, n_rec): table sizes of the last grid call on the current device."""
    a = ctypes.c_int64()
    b = ctypes.c_int64()
    check(lib().ez_grid_last_tables(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def workspace_generation() -> int:
    """Changes whenever the library frees or moves device memory it owns."""
    return int(lib().ez_workspace_generation())
