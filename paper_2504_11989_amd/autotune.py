"""Autotuner for the lattice-sum launches.

What it chooses, by timing candidate configurations on a sample of the workload:

* lam, the Ewald split parameter (in units of V^{1/d}).  The result does not
  depend on it beyond rounding, but the work per node does: the reciprocal table
  shrinks like lam^-d and the real-space table grows like lam^d, and the two cost
  differently per entry (an incomplete-gamma evaluation against one complex
  rotation).
* the node-kernel schedule: one workgroup per 256-node tile, or a persistent grid
  of k workgroups per CU taking tiles from a work queue costliest-first
  (spec flags EZ_SPEC_PERSISTENT | EZ_SPEC_BPC(k));
* the shape of the 64-node wave blocks (EZ_SPEC_WAVE_U(k): 2^(k+2) consecutive
  u-nodes x 2^(4-k) directions, or the planner's choice), which sets how compact
  each wave's k-points are and so how many reciprocal entries its culling keeps.

Timing uses CUDA/HIP events on the current stream around whole calls (median of
`reps`).  Results are cached per (d, exponent set, sample shape) in-process and,
with `cache_file`, in a JSON file keyed by the device name, the HIP runtime
version and the library version.

It also gives the number of Gauss points n_q per v-dimension from the analytic
convergence rate (paper, Sec. 3, the corollary on the Bernstein ellipse): the
v-integrand is holomorphic on E_rho^(d-1) for rho < rho_bound = a + sqrt(1 + a^2),
a = 2 / (kappa(A) sqrt(d - 1)), so the Gauss error decays like rho_bound^(-2 n_q).
"""
from __future__ import annotations

import json
import math
import os
import statistics
from typing import Iterable, Sequence

import numpy as np
import torch

from . import lattice_sums, version
from ._native import SPEC_PERSISTENT, spec_bpc, spec_wave_u

__all__ = ["tune", "apply", "rho_bound", "nq_for", "DEFAULT_LAMS", "DEFAULT_SCHEDULES", "DEFAULT_WAVE_SHAPES"]

DEFAULT_LAMS = (1.0, 1.15, 1.3, 1.45, 1.6)
# (name, flags)
DEFAULT_SCHEDULES = (("tile-per-workgroup", 0),
                     ("persistent, fit", SPEC_PERSISTENT),
                     ("persistent, 2/CU", SPEC_PERSISTENT | spec_bpc(2)),
                     ("persistent, 4/CU", SPEC_PERSISTENT | spec_bpc(4)))

# (name, flags): the planner's choice, then 8, 16, 32, 64 u-nodes per wave block
DEFAULT_WAVE_SHAPES = (("auto", 0), ("8u x 8dir", spec_wave_u(1)), ("16u x 4dir", spec_wave_u(2)),
                       ("32u x 2dir", spec_wave_u(3)), ("64u x 1dir", spec_wave_u(4)))

_cache: dict = {}


def rho_bound(A) -> float:
    """rho_bound = a + sqrt(1 + a^2), a = 2 / (kappa(A) sqrt(d - 1)), kappa the
    2-norm condition number (d >= 2)."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[0]
    if d < 2:
        raise ValueError("the v-integral exists for d >= 2 only")
    a = 2.0 / (np.linalg.cond(A) * math.sqrt(d - 1))
    return a + math.sqrt(1.0 + a * a)


def nq_for(A, tol: float, margin: int = 2) -> int:
    """Gauss points per v-dimension for a relative error tol at the rate
    rho_bound^(-2 n_q), plus `margin` points for the unknown constant."""
    rho = rho_bound(A)
    return int(math.ceil(math.log(1.0 / tol) / (2.0 * math.log(rho)))) + int(margin)


def _file_key() -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return f"{dev}|hip {torch.version.hip}|{version()}"


def apply(specs, lam: float, flags: int):
    """specs (one dict or a list) with lam and flags replaced."""
    if isinstance(specs, dict):
        return dict(specs, lam=lam, flags=flags)
    return [dict(s, lam=lam, flags=flags) for s in specs]


def _time_call(A, nu, terms, n_results, specs, reps: int) -> float:
    out = lattice_sums(A, nu, terms, n_results, specs)        # warm: plan, workspace
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        s.record()
        lattice_sums(A, nu, terms, n_results, specs, out=out)
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e))
    return statistics.median(ts)


def tune(A, nu: Sequence[float], terms: Iterable, n_results: int, specs, lams=DEFAULT_LAMS,
         schedules=DEFAULT_SCHEDULES, reps: int = 3, verbose: bool = False, wave_shapes=(),
         cache_file: str | None = None) -> dict:
    """Time every lam with the first schedule, then the other schedules at the best
    lam, then the wave-block shapes (if given) at the best (lam, schedule), on the
    sample batch A with its specs, and return {"lam", "flags", "schedule", "wave",
    "ms", "table": [(lam, schedule, wave, ms), ...]}.  With cache_file, a result
    stored there for the same device, runtime, library and problem is reused."""
    A = torch.as_tensor(A, dtype=torch.float64, device="cuda").contiguous()
    terms = list(terms)
    key = (A.shape, tuple(nu), repr(terms), n_results, repr(specs), tuple(lams), tuple(schedules),
           tuple(wave_shapes))
    if key in _cache:
        return _cache[key]
    fkey = _file_key() + "|" + repr(key)
    stored = {}
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as fh:
            stored = json.load(fh)
        if fkey in stored:
            res = stored[fkey]
            res["table"] = [tuple(r) for r in res["table"]]
            _cache[key] = res
            return res
    res = _tune(A, nu, terms, n_results, specs, lams, schedules, reps, verbose, wave_shapes)
    _cache[key] = res
    if cache_file:
        stored[fkey] = res
        d = os.path.dirname(os.path.abspath(cache_file))
        os.makedirs(d, exist_ok=True)
        tmp = cache_file + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(stored, fh, indent=1)
        os.replace(tmp, cache_file)
    return res


def _tune(A, nu, terms, n_results, specs, lams, schedules, reps, verbose, wave_shapes) -> dict:
    table = []
    # lam first with the default schedule, then the schedule at the best lam
    auto = wave_shapes[0][0] if wave_shapes else "auto"
    for lam in lams:
        ms = _time_call(A, nu, terms, n_results, apply(specs, lam, schedules[0][1]), reps)
        table.append((lam, schedules[0][0], auto, ms))
        if verbose:
            print(f"lam {lam:.2f} {schedules[0][0]}: {ms:.3f} ms", flush=True)
    best_lam = min(table, key=lambda r: r[3])[0]
    for name, flags in schedules[1:]:
        ms = _time_call(A, nu, terms, n_results, apply(specs, best_lam, flags), reps)
        table.append((best_lam, name, auto, ms))
        if verbose:
            print(f"lam {best_lam:.2f} {name}: {ms:.3f} ms", flush=True)
    lam, sched, _, _ = min(table, key=lambda r: r[3])
    sflags = dict(schedules)[sched]
    for wname, wflags in wave_shapes[1:]:
        ms = _time_call(A, nu, terms, n_results, apply(specs, lam, sflags | wflags), reps)
        table.append((lam, sched, wname, ms))
        if verbose:
            print(f"lam {lam:.2f} {sched} wave {wname}: {ms:.3f} ms", flush=True)
    lam, sched, wave, ms = min(table, key=lambda r: r[3])
    flags = dict(schedules)[sched] | (dict(wave_shapes)[wave] if wave_shapes else 0)
    return {"lam": lam, "flags": flags, "schedule": sched, "wave": wave, "ms": ms, "table": table}
