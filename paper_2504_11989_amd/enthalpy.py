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

import sys

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


# Parametrisations of the generator matrix for the minimisation: theta -> A(theta)
# and the chain rule dH/dtheta = sum_ij dH/dA_ij dA_ij/dtheta (dH/dA from the
# adjoint kernels).
#   "general": theta = the 9 entries of A
#   "scale"  : A = R S for the start's shape S (theta = R, the paper's scan over
#              the nearest-neighbour distance of a fixed lattice, Sec. 5)
#   "bct"    : A = [[a, 0, a/2], [0, a, a/2], [0, 0, c/2]] (theta = (a, c)): the
#              body-centred tetragonal family, bcc at c = a, fcc at c = sqrt(2) a,
#              which joins them along the Bain path
def _param_init(param, A0):
    B = A0.shape[0]
    if param == "general":
        return A0.reshape(B, 9).copy(), None
    if param == "scale":
        return np.ones((B, 1)), A0.copy()
    if param == "bct":
        return np.stack([A0[:, 0, 0], 2.0 * A0[:, 2, 2]], axis=1), None
    raise ValueError("param must be 'general', 'scale' or 'bct'")


def _param_A(param, x, shape):
    B = x.shape[0]
    if param == "general":
        return x.reshape(B, 3, 3)
    if param == "scale":
        return x[:, 0, None, None] * shape
    A = np.zeros((B, 3, 3))
    A[:, 0, 0] = A[:, 1, 1] = x[:, 0]
    A[:, 0, 2] = A[:, 1, 2] = 0.5 * x[:, 0]
    A[:, 2, 2] = 0.5 * x[:, 1]
    return A


def _param_grad(param, gA, shape):
    B = gA.shape[0]
    if param == "general":
        return gA.reshape(B, 9)
    if param == "scale":
        return np.einsum("bij,bij->b", gA, shape)[:, None]
    return np.stack([gA[:, 0, 0] + gA[:, 1, 1] + 0.5 * (gA[:, 0, 2] + gA[:, 1, 2]), 0.5 * gA[:, 2, 2]], axis=1)


def minimise(A0, c, p, spec=None, max_iter: int = 200, gtol: float = 1e-9, verbose: bool = False,
             param: str = "general", cond_max: float = 25.0):
    """Minimise H over the generator matrix for every problem of the batch at once
    (BFGS with Armijo backtracking in the parameters of `param`, one batched GPU
    evaluation of H and dH/dA per trial step).  A problem stops when its gradient
    norm (in the parameters) drops below gtol, or as degenerate when its matrix
    becomes singular or skewed beyond cond(A) > cond_max, or its lattice tables
    overflow: a lattice that flattens into chains or layers has no minimum among
    Bravais lattices.

    Returns dict(A, H, grad_norm, iterations, converged, degenerate, E, V)."""
    A0 = np.asarray(A0, dtype=np.float64)
    B = A0.shape[0]
    x, shape = _param_init(param, A0)
    n = x.shape[1]
    c_t = torch.as_tensor(np.broadcast_to(np.asarray(c, dtype=np.float64), (B,)).copy()).cuda()
    p_t = torch.as_tensor(np.broadcast_to(np.asarray(p, dtype=np.float64), (B,)).copy()).cuda()

    def f(xv, idx=None):
        # H and its gradient for the problems idx (all when None), one batched call
        if idx is None:
            idx = np.arange(B)
        sh = None if shape is None else shape[idx]
        A = _param_A(param, xv[idx], sh)
        Ht, gt, Et, Vt = enthalpy(torch.from_numpy(np.ascontiguousarray(A)).cuda(), c_t[idx], p_t[idx], spec)
        Hn = Ht.cpu().numpy()
        cond = np.linalg.cond(A)
        Hn = np.where(np.isfinite(cond) & (cond <= cond_max), Hn, np.nan)
        return Hn, _param_grad(param, gt.cpu().numpy(), sh), Et.cpu().numpy(), Vt.cpu().numpy()

    H, g, E, V = f(x)
    gn = np.linalg.norm(g, axis=1)
    Hinv = np.repeat(np.eye(n)[None], B, axis=0) * np.minimum(1.0, 0.05 / np.maximum(gn, 1e-30))[:, None, None]
    degenerate = ~np.isfinite(H)
    done = (gn < gtol) | degenerate
    fails = np.zeros(B, dtype=int)
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
            # trial steps of the problems still searching, evaluated together
            idx = np.nonzero(~acc)[0]
            xt = x[idx] + alpha[idx, None] * d[idx]
            xfull = x.copy()
            xfull[idx] = xt
            Ht, gt, Et, Vt = f(xfull, idx)
            # Armijo condition, with an allowance for the rounding of H near the minimum
            ok = np.isfinite(Ht) & (Ht <= H[idx] + 1e-4 * alpha[idx] * slope[idx] + 4e-15 * np.abs(H[idx]))
            ii = idx[ok]
            xn[ii], Hn[ii], gn_[ii], En[ii], Vn[ii] = xt[ok], Ht[ok], gt[ok], Et[ok], Vt[ok]
            acc[ii] = True
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
            Vb = np.eye(n)[None] - rho[:, None, None] * su[:, :, None] * yu[:, None, :]
            Hinv[upd] = Vb @ Hinv[upd] @ Vb.transpose(0, 2, 1) + rho[:, None, None] * su[:, :, None] * su[:, None, :]
        stalled = ~acc                      # no acceptable step: keep the point, restart the metric
        Hinv[stalled] = np.eye(n) * 1e-3
        fails = np.where(stalled, fails + 1, 0)
        x, H, g, E, V = xn, Hn, gn_, En, Vn
        gnorm = np.linalg.norm(g, axis=1)
        # no finite acceptable step in three iterations in a row: the problem sits at the
        # edge of the admissible (non-degenerate) matrices
        degenerate |= (fails >= 3) & ~done & (gnorm >= gtol)
        done |= (gnorm < gtol) | degenerate
        if verbose:
            print(f"iter {it}: H range [{np.nanmin(H):.6f}, {np.nanmax(H):.6f}], max |g| {gnorm.max():.3e}, "
                  f"converged {int((done & ~degenerate).sum())}/{B}, degenerate {int(degenerate.sum())}",
                  file=sys.stderr, flush=True)
    A = _param_A(param, x, shape)
    gnorm = np.linalg.norm(g, axis=1)
    return dict(A=A.copy(), H=H, grad_norm=gnorm, iterations=it, converged=(gnorm < gtol) & ~degenerate,
                degenerate=degenerate, E=E, V=V)


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


def phase_scan(cs, ps, spec=None, max_iter: int = 100, gtol: float = 1e-7, stability: bool = True,
               stability_iter: int = 150, stability_stride: int = 1, seed: int = 5, verbose: bool = False):
    """Stable lattice over a grid of ATM couplings c and pressures p (paper,
    Sec. 5, Fig. 11): H = E_LJ + c E_ATM + p V per particle.

    1. As in the paper, H of the fcc and of the bcc lattice is minimised over the
       lattice scale R (A = R A_0) at every (c, p), all problems in one batched
       minimisation driven by the adjoint gradient (dH/dR = <dH/dA, A_0>); the
       lower enthalpy wins.
    2. (stability=True) The winner of every stability_stride-th point in c and p,
       its entries perturbed by up to 10% (seeded), is minimised over the general
       3 x 3 generator matrix: it
       returns to a lattice of the same kind (named by its neighbour shells), or
       degenerates: strong ATM coupling at low pressure favours collinear
       triples, the lattice flattens into chains, and H has no minimum among
       Bravais lattices there.

    Returns dict(H (nc, np, 2) [fcc, bcc], R (nc, np, 2) nearest-neighbour distance
    of the minima, converged (nc, np, 2), phase (nc, np) 'fcc' / 'bcc', V (nc, np)
    volume per particle of the winner, A (nc, np, 3, 3), iterations, and with
    stability: general (nc, np) outcome names, general_H, general_converged,
    general_degenerate, general_iterations)."""
    cs = np.asarray(cs, dtype=np.float64)
    ps = np.asarray(ps, dtype=np.float64)
    nc, npp = len(cs), len(ps)
    # unit nearest-neighbour distance (paper, Sec. 5)
    nn1 = [np.array([[1.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 1.0]]) / np.sqrt(2.0),
           np.array([[1.0, 1.0, 0.0], [np.sqrt(2.0), 0.0, np.sqrt(2.0)], [0.0, np.sqrt(2.0), np.sqrt(2.0)]])
           / np.sqrt(3.0)]
    starts = np.stack(nn1)
    C, P, S = np.meshgrid(cs, ps, np.arange(2), indexing="ij")
    res = minimise(starts[S.reshape(-1)], C.reshape(-1), P.reshape(-1), spec, max_iter=max_iter, gtol=gtol,
                   verbose=verbose, param="scale")
    H = res["H"].reshape(nc, npp, 2)
    A = res["A"].reshape(nc, npp, 2, 3, 3)
    R = np.abs(np.linalg.det(A)) ** (1.0 / 3.0) / np.abs(np.linalg.det(starts)) ** (1.0 / 3.0)
    win = np.argmin(np.where(np.isfinite(H), H, np.inf), axis=2)
    phase = np.where(win == 0, "fcc", "bcc").astype(object)
    Aw = np.take_along_axis(A, win[:, :, None, None, None], axis=2)[:, :, 0]
    V = np.abs(np.linalg.det(Aw))
    out = dict(H=H, R=R, converged=res["converged"].reshape(nc, npp, 2), phase=phase, V=V, A=Aw,
               iterations=res["iterations"])
    if stability:
        # every stride-th point in c and in p
        si = np.arange(0, nc, stability_stride)
        sj = np.arange(0, npp, stability_stride)
        rng = np.random.default_rng(seed)
        Aw_s = Aw[np.ix_(si, sj)].reshape(-1, 3, 3)
        A0 = Aw_s * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, size=Aw_s.shape))
        Cg, Pg = np.meshgrid(cs[si], ps[sj], indexing="ij")
        rg = minimise(A0, Cg.reshape(-1), Pg.reshape(-1), spec, max_iter=stability_iter, gtol=1e-6,
                      verbose=verbose, param="general")
        gen = np.empty((len(si), len(sj)), dtype=object)
        for k in range(len(si) * len(sj)):
            i, j = divmod(k, len(sj))
            if rg["degenerate"][k]:
                gen[i, j] = "degenerate"
            elif not rg["converged"][k]:
                gen[i, j] = "unconverged"
            else:
                gen[i, j] = classify(rg["A"][k])
        shp = (len(si), len(sj))
        out.update(general=gen, general_c=cs[si], general_p=ps[sj], general_H=rg["H"].reshape(shp),
                   general_converged=rg["converged"].reshape(shp), general_degenerate=rg["degenerate"].reshape(shp),
                   general_iterations=rg["iterations"])
    return out


def _bct_unit(c_over_a):
    """body-centred tetragonal generator matrix at unit density (volume 1)"""
    a = (2.0 / c_over_a) ** (1.0 / 3.0)
    return np.array([[a, 0.0, a / 2.0], [0.0, a, a / 2.0], [0.0, 0.0, c_over_a * a / 2.0]])
