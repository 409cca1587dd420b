"""Autotuner for the lattice-sum launches.

What it chooses, by timing candidate configurations on a sample of the workload:

* lam, the Ewald split parameter (in units of V^{1/d}).  The result does not
  depend on it beyond rounding, but the work per node does: the reciprocal table
  shrinks like lam^-d and the real-space table grows like lam^d, and the two cost
  differently per entry (an incomplete-gamma evaluation against one complex
  rotation).
* the node-kernel schedule: one workgroup per 256-node tile, or a persistent grid
  of k workgroups per CU taking tiles from a work queue costliest-first
  (spec flags EZ_SPEC_PERSISTENT | EZ_SPEC_BPC(k)).

Timing uses CUDA/HIP events on the current stream around whole calls (median of
`reps`).  Results are cached per (d, exponent set, sample shape) in-process.
"""
from __future__ import annotations

import statistics
from typing import Iterable, Sequence

import torch

from . import lattice_sums
from ._native import SPEC_PERSISTENT, spec_bpc

__all__ = ["tune", "apply", "DEFAULT_LAMS", "DEFAULT_SCHEDULES"]

DEFAULT_LAMS = (1.0, 1.15, 1.3, 1.45, 1.6)
# (name, flags)
DEFAULT_SCHEDULES = (("tile-per-workgroup", 0),
                     ("persistent, fit", SPEC_PERSISTENT),
                     ("persistent, 2/CU", SPEC_PERSISTENT | spec_bpc(2)),
                     ("persistent, 4/CU", SPEC_PERSISTENT | spec_bpc(4)))

_cache: dict = {}


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
         schedules=DEFAULT_SCHEDULES, reps: int = 3, verbose: bool = False) -> dict:
    """Time every (lam, schedule) pair on the sample batch A with its specs and
    return {"lam", "flags", "schedule", "ms", "table": [(lam, schedule, ms), ...]}."""
    A = torch.as_tensor(A, dtype=torch.float64, device="cuda").contiguous()
    terms = list(terms)
    key = (A.shape, tuple(nu), repr(terms), n_results, repr(specs), tuple(lams), tuple(schedules))
    if key in _cache:
        return _cache[key]
    table = []
    # lam first with the default schedule, then the schedule at the best lam
    for lam in lams:
        ms = _time_call(A, nu, terms, n_results, apply(specs, lam, 0), reps)
        table.append((lam, schedules[0][0], ms))
        if verbose:
            print(f"lam {lam:.2f} {schedules[0][0]}: {ms:.3f} ms", flush=True)
    best_lam = min(table, key=lambda r: r[2])[0]
    for name, flags in schedules[1:]:
        ms = _time_call(A, nu, terms, n_results, apply(specs, best_lam, flags), reps)
        table.append((best_lam, name, ms))
        if verbose:
            print(f"lam {best_lam:.2f} {name}: {ms:.3f} ms", flush=True)
    lam, sched, ms = min(table, key=lambda r: r[2])
    flags = dict(schedules)[sched]
    res = {"lam": lam, "flags": flags, "schedule": sched, "ms": ms, "table": table}
    _cache[key] = res
    return res
