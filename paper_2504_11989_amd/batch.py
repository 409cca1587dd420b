"""Batched lattice sums: the 4096-lattice bct scan program and replay of a captured HIP graph.

A scan evaluates many lattices with uneven quadrature plans in one call of the
library (one launch sequence: setup, the node kernel over every node tile of the
batch, the Taylor/Hadamard branch on a second stream, the fixed-order reduction).
`GraphedLatticeSums` captures that call once into a HIP graph (torch's graph API
drives the capture on its stream; the library's kernels and event edges are
recorded) and replays it; new lattices are copied into its input buffer first.
"""
from __future__ import annotations

from typing import Iterable, Sequence

import torch

from . import lattice_sums
from ._native import workspace_generation

__all__ = ["SCAN_NU", "SCAN_TERMS", "SCAN_RESULTS", "scan_sums", "GraphedLatticeSums"]

# three-body product sums zeta^(3)(nu, nu, nu) for nu in {3, 6, 9, 12} and the ATM
# energy (Sec. 2, Proposition) on one node set: exponents {-1, 1, 3, 5, 6, 9, 12}
SCAN_NU = [-1.0, 1.0, 3.0, 5.0, 6.0, 9.0, 12.0]
SCAN_RESULTS = ["E_ATM", "zeta3(3,3,3)", "zeta3(6,6,6)", "zeta3(9,9,9)", "zeta3(12,12,12)"]
SCAN_TERMS = [
    (0, 1.0 / 24.0, [(2, 3)]),
    (0, -3.0 / 16.0, [(0, 1), (3, 2)]),
    (0, 3.0 / 8.0, [(1, 1), (2, 1), (3, 1)]),
    (1, 1.0, [(2, 3)]),
    (2, 1.0, [(4, 3)]),
    (3, 1.0, [(5, 3)]),
    (4, 1.0, [(6, 3)]),
]


def scan_sums(A, specs, **kw):
    """The scan program on a batch of 3 x 3 generator matrices, one spec per lattice
    (or one shared): float64 (batch, 5) in the order of SCAN_RESULTS."""
    return lattice_sums(A, SCAN_NU, SCAN_TERMS, len(SCAN_RESULTS), specs, **kw)


class GraphedLatticeSums:
    """One lattice_sums call captured into a HIP graph and replayed.

    The captured call reads its lattices from `self.A` and writes `self.out` /
    `self.status`; to evaluate other lattices of the same batch shape and plans,
    copy them into `self.A` (on the current stream) before `replay()`.  The graph
    holds the library's device pointers (workspace, cached plan): it stays valid
    while the library frees none of them (no ez_finalize, no call with a larger
    problem that grows the workspace, no eviction of the plan), which is checked
    against the library's workspace generation before every replay."""

    def __init__(self, A, nu: Sequence[float], terms: Iterable, n_results: int, specs=None, warmup: int = 1):
        self.A = torch.as_tensor(A, dtype=torch.float64, device="cuda").clone().contiguous()
        b = self.A.shape[0]
        self.nu, self.terms, self.n_results, self.specs = list(nu), list(terms), int(n_results), specs
        self.out = torch.empty((b, self.n_results), dtype=torch.float64, device=self.A.device)
        self.status = torch.zeros(b, dtype=torch.int32, device=self.A.device)
        self.stream = torch.cuda.Stream(self.A.device)           # default priority
        self.stream.wait_stream(torch.cuda.current_stream(self.A.device))
        with torch.cuda.stream(self.stream):
            # plans, rule tables and workspace are created by the eager calls
            for _ in range(max(1, warmup)):
                self._call()
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._call()
        self.generation = workspace_generation()
        torch.cuda.current_stream(self.A.device).wait_stream(self.stream)

    def _call(self):
        lattice_sums(self.A, self.nu, self.terms, self.n_results, self.specs, out=self.out, status=self.status)

    def replay(self):
        if workspace_generation() != self.generation:
            raise RuntimeError("the library has freed or moved device memory this graph uses "
                               "(workspace grown, plan evicted or ez_finalize): capture it again")
        self.graph.replay()
        return self.out
