"""torch.autograd.Function wrappers over the adjoint kernels.

The forward call runs the lattice sums together with their derivatives with
respect to the generator matrix (one launch sequence; the adjoint pass is fused
into the node kernel), saves the derivative tensor, and the backward pass is a
contraction with the incoming gradient.  The derivative is that of the
quadrature value on the given plan (nodes fixed in fractional coordinates).
"""
from __future__ import annotations

from typing import Iterable, Sequence

import torch

from . import atm_energy, lattice_sums

__all__ = ["atm_energy_t", "lattice_sums_t", "AtmEnergyFunction", "LatticeSumsFunction"]


class AtmEnergyFunction(torch.autograd.Function):
    """E_ATM(A) for a batch of generator matrices (batch, d, d) -> (batch,)."""

    @staticmethod
    def forward(ctx, A, spec):
        E, g = atm_energy(A.detach(), spec, grad=True)
        ctx.save_for_backward(g)
        return E

    @staticmethod
    def backward(ctx, gE):
        (g,) = ctx.saved_tensors
        return gE[:, None, None] * g, None


class LatticeSumsFunction(torch.autograd.Function):
    """(batch, d, d) -> (batch, n_results) for a term program (n_results <= 2)."""

    @staticmethod
    def forward(ctx, A, nu, terms, n_results, specs):
        out, g = lattice_sums(A.detach(), nu, terms, n_results, specs, grad=True)
        ctx.save_for_backward(g)
        return out

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return torch.einsum("br,brij->bij", gout, g), None, None, None, None


def _batched(A):
    A = torch.as_tensor(A, dtype=torch.float64)
    if A.device.type != "cuda":
        raise ValueError("A must be a CUDA tensor")
    return (A.unsqueeze(0), True) if A.dim() == 2 else (A, False)


def atm_energy_t(A, spec=None):
    """Differentiable ATM energy per particle; A (d, d) or (batch, d, d) on the GPU."""
    A, single = _batched(A)
    E = AtmEnergyFunction.apply(A, spec)
    return E[0] if single else E


def lattice_sums_t(A, nu: Sequence[float], terms: Iterable, n_results: int, specs=None):
    """Differentiable form of lattice_sums (n_results <= 2)."""
    A, single = _batched(A)
    out = LatticeSumsFunction.apply(A, list(nu), list(terms), int(n_results), specs)
    return out[0] if single else out
