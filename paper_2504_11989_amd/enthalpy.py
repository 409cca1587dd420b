"""Enthalpy per particle of a Bravais lattice with Lennard-Jones pair and
Axilrod-Teller-Muto three-body interactions, its gradient with respect to the
generator matrix, and batched minimisation over lattices (paper, Sec. 5).

    H(A) = E_LJ(A) + c E_ATM(A) + p V(A),   V = |det A|,

with the pair potential U(r) = r^-12 - 2 r^-6 (well depth 1 at r = 1), so
E_LJ = Z_12(0)/2 - Z_6(0).  Both Epstein values at the origin are two-body
zeta functions (Sec. 2, Corollary: zeta^(2)(nu1, nu2) = Z_{nu1+nu2}(0)), so
E_LJ and E_ATM come out of one lattice-sum program on the exponent set
{-1, 1, 3, 5, 7}: Z_12 = zeta^(2)(5, 7) and Z_6 = zeta^(2)(3, 3).  Every
value and derivative is computed by the HIP kernels; this module only
assembles H and runs the optimiser's small linear algebra on the host.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lattice_sums

__all__ = ["LJ_ATM_NU", "LJ_ATM_TERMS", "energies", "enthalpy", "minimise", "classify", "phase_scan"]

LJ_ATM_NU = [-1.0, 1.0, 3.0, 5.0, 7.0]
# (result, coefficient, [(index into LJ_ATM_NU, multiplicity), ...])
LJ_ATM_TERMS = [
    (0, 0.5, [(3, 1), (4, 1)]),                 # Z_12(0)/2 = zeta^(2)(5, 7)/2
    (0, -1.0, [(2, 2)]),                        # -Z_6(0)   = -zeta^(2)(3, 3)
    (1, 1.0 / 24.0, [(2, 3)]),                  # ATM (Sec. 2, Proposition)
    (1, -3.0 / 16.0, [(0, 1), (3, 2)]),
    (1, 3.0 / 8.0, [(1, 1), (2, 1), (3, 1)]),
]


def energies(A, spec=None, grad=False):
    """E_LJ and E_ATM per particle: (batch, 2) [and their d/dA, (batch, 2, 3, 3)]."""
    return lattice_sums(A, LJ_ATM_NU, LJ_ATM_TERMS, 2, spec, grad=grad)


def enthalpy(A, c, p, spec=None):
    """H per particle and dH/dA for a batch of 3 x 3 generator matrices.

    A: (batch, 3, 3) float64 CUDA tensor; c, p: scalars or (batch,) tensors.
    Returns (H (batch,), dH/dA (batch, 3, 3), E (batch, 2) = [E_LJ, E_ATM], V (batch,))."""
    A = torch.as_tensor(A, dtype=torch.float64, device="cuda").contiguous()
    c = torch.as_tensor(c, dtype=torch.float64, device=A.device).expand(A.shape[0])
    p = torch.as_tensor(p, dtype=torch.float64, device=A.device).expand(A.shape[0])
    E, g = energies(A, spec, grad=True)
    det = torch.linalg.det(A)
    V = det.abs()
    dV = V[:, None, None] * torch.linalg.inv(A).transpose(1, 2)     # d|det A|/dA = |det A| A^{-T}
    H = E[:, 0] + c * E[:, 1] + p * V
    dH = g[:, 0] + c[:, None, None] * g[:, 1] + p[:, None, None] * dV
    return H, dH, E, V


def minimise(A0, c, p, spec=None, max_iter: int = 200, gtol: float = 1e-9, verbose: bool = False):
    """Minimise H over the generator matrix for every problem of the batch at once
    (BFGS with Armijo backtracking, one batched GPU evaluation per trial step).

    Returns dict(A, H, grad_norm, iterations, converged, E, V)."""
    A = torch.as_tensor(A0, dtype=torch.float64, device="cuda").clone()
    B = A.shape[0]
    x = A.reshape(B, 9).cpu().numpy()
    c_t = torch.as_tensor(c, dtype=torch.float64).expand(B).cuda()
    p_t = torch.as_tensor(p, dtype=torch.float64).expand(B).cuda()

    def f(xv):
        Ht, gt, Et, Vt = enthalpy(torch.from_numpy(xv.reshape(B, 3, 3)).cuda(), c_t, p_t, spec)
        return Ht.cpu().numpy(), gt.reshape(B, 9).cpu().numpy(), Et.cpu().numpy(), Vt.cpu().numpy()

    H, g, E, V = f(x)
    gn = np.linalg.norm(g, axis=1)
    Hinv = np.repeat(np.eye(9)[None], B, axis=0) * np.minimum(1.0, 0.05 / np.maximum(gn, 1e-30))[:, None, None]
    done = gn < gtol
    it = 0
    for it in range(1, max_iter + 1):
        if done.all():
            break
        d = -np.einsum("bij,bj->bi", Hinv, g)
        slope = np.einsum("bi,bi->b", g, d)
        reset = slope >= 0
        d[reset] = -g[reset]
        slope[reset] = -np.einsum("bi,bi->b", g[reset], g[reset])
        alpha = np.ones(B)
        acc = done.copy()
        xn, Hn, gn_, En, Vn = x.copy(), H.copy(), g.copy(), E.copy(), V.copy()
        for _ in range(40):
            xt = np.where(acc[:, None], x, x + alpha[:, None] * d)
            Ht, gt, Et, Vt = f(xt)
            ok = np.isfinite(Ht) & (Ht <= H + 1e-4 * alpha * slope) & ~acc
            xn[ok], Hn[ok], gn_[ok], En[ok], Vn[ok] = xt[ok], Ht[ok], gt[ok], Et[ok], Vt[ok]
            acc |= ok
            if acc.all():
                break
            alpha[~acc] *= 0.5
        s = xn - x
        y = gn_ - g
        sy = np.einsum("bi,bi->b", s, y)
        upd = (sy > 1e-14) & ~done
        if upd.any():
            # BFGS update of the inverse Hessians, all updated problems at once:
            # H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, rho = 1 / (y.s)
            su, yu = s[upd], y[upd]
            rho = 1.0 / sy[upd]
            Vb = np.eye(9)[None] - rho[:, None, None] * su[:, :, None] * yu[:, None, :]
            Hinv[upd] = Vb @ Hinv[upd] @ Vb.transpose(0, 2, 1) + rho[:, None, None] * su[:, :, None] * su[:, None, :]
        stalled = ~acc                      # no acceptable step: keep the point, restart the metric
        Hinv[stalled] = np.eye(9) * 1e-3
        x, H, g, E, V = xn, Hn, gn_, En, Vn
        gnorm = np.linalg.norm(g, axis=1)
        done |= gnorm < gtol
        if verbose:
            print(f"iter {it}: H range [{H.min():.6f}, {H.max():.6f}], max |g| {gnorm.max():.3e}, "
                  f"converged {int(done.sum())}/{B}", flush=True)
    return dict(A=x.reshape(B, 3, 3), H=H, grad_norm=np.linalg.norm(g, axis=1), iterations=it, converged=done,
                E=E, V=V)


def classify(A, tol: float = 0.03) -> str:
    """Name of the Bravais lattice a generator matrix spans, from its nearest-
    neighbour shells: 'fcc' (12 at r1), 'bcc' (8 at r1, 6 at 2 r1/sqrt 3), 'sc' (6),
    'hcp-like/other' otherwise."""
    A = np.asarray(A, dtype=np.float64)
    rng = np.arange(-3, 4)
    n = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3)
    n = n[np.any(n != 0, axis=1)]
    r = np.sort(np.linalg.norm(n @ A.T, axis=1))
    r1 = r[0]
    n1 = int(np.sum(r <= r1 * (1 + tol)))
    if n1 == 12:
        return "fcc"
    if n1 == 8:
        n2 = int(np.sum((r > r1 * (1 + tol)) & (r <= r1 * 2 / np.sqrt(3) * (1 + tol))))
        return "bcc" if n2 == 6 else "other"
    if n1 == 6:
        return "sc"
    return "other"


def phase_scan(cs, ps, starts, spec=None, max_iter: int = 300, gtol: float = 1e-8, verbose: bool = False):
    """Stable Bravais lattice over a grid of ATM couplings c and pressures p
    (paper, Sec. 5): H = E_LJ + c E_ATM + p V is minimised from every start
    matrix at every (c, p), all len(cs) len(ps) len(starts) problems in one
    batched minimisation; at each grid point the lowest minimum wins.

    starts: (n_starts, 3, 3) generator matrices (e.g. perturbed fcc and bcc).
    Returns dict(H (nc, np, ns), A (nc, np, ns, 3, 3), converged (nc, np, ns),
    grad_norm, iterations, winner (nc, np) start index, phase (nc, np) lattice
    names of the winning minima, V (nc, np) their volume per particle)."""
    cs = np.asarray(cs, dtype=np.float64)
    ps = np.asarray(ps, dtype=np.float64)
    starts = np.asarray(starts, dtype=np.float64)
    nc, npp, ns = len(cs), len(ps), len(starts)
    C, P, S = np.meshgrid(cs, ps, np.arange(ns), indexing="ij")
    A0 = starts[S.reshape(-1)]
    res = minimise(A0, C.reshape(-1), P.reshape(-1), spec, max_iter=max_iter, gtol=gtol, verbose=verbose)
    H = res["H"].reshape(nc, npp, ns)
    A = res["A"].reshape(nc, npp, ns, 3, 3)
    win = np.argmin(np.where(np.isfinite(H), H, np.inf), axis=2)
    phase = np.empty((nc, npp), dtype=object)
    V = np.zeros((nc, npp))
    for i in range(nc):
        for j in range(npp):
            Aw = A[i, j, win[i, j]]
            phase[i, j] = classify(Aw)
            V[i, j] = abs(np.linalg.det(Aw))
    return dict(H=H, A=A, converged=res["converged"].reshape(nc, npp, ns),
                grad_norm=res["grad_norm"].reshape(nc, npp, ns), iterations=res["iterations"],
                winner=win, phase=phase, V=V)
