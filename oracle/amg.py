"""Aggregation AMG hierarchy, V-cycle and PCG (oracle, test infrastructure only).

* Galerkin coarse operators A_{l+1} = P_l^T A_l P_l (Section 2, first display).
* Piecewise-constant P from fixed box aggregates of the structured grid,
  2x2x2 by default, e x e x e for an aggregate edge e (entries 1.0; a
  dimension of extent 1 is not coarsened, a ragged extent leaves a last
  aggregate narrower than e).  Problems stacked along z (``nbatch`` > 1) are
  aggregated separately.
* Optionally the smoothed prolongator of Section 4, P = (I - omega D^{-1} A) P_hat
  with D the diagonal of A and omega = 4 / (3 lambda), lambda an estimate of
  the largest eigenvalue of D^{-1} A; the estimate used is the Gershgorin bound
  ||D^{-1} A||_inf, taken per stacked problem.
* Coarsening continues while a level has more than ``max_coarse`` rows per
  problem; the coarsest level is solved by dense Cholesky (scipy cho_factor /
  cho_solve), one factor per stacked problem, or, as in the paper's runs
  (Section 4), by a fixed number of l1-Jacobi sweeps from zero.
* V-cycle of eq. (amg): pre-smoothing with p_k(M^{-1}A) from zero, residual
  restriction, recursion, prolongation, post-smoothing with the same
  polynomial (M is diagonal and p_k(M^{-1}A) is A-self-adjoint, so the
  M^{-T} of eq. (amg) is the same operator and the V-cycle is symmetric).
* Preconditioned CG with x0 = 0 and the stopping test ||r_k||_2 <= rtol ||b||_2
  on the recursively updated residual; an optional flexible (Polak-Ribiere)
  beta for preconditioners that are not exactly fixed (the paper's runs use
  a flexible CG, Section 4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import polynomials as P
from .smoothers import OPTCHEB1, OPTCHEB4, l1_diagonal, smooth, smooth_l1jacobi


@dataclass
class Level:
    A: sp.csr_matrix
    Minv: np.ndarray
    grid: tuple  # per-problem (nx, ny, nz)
    nbatch: int
    P: sp.csr_matrix | None = None  # prolongation to this level from the next one


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    chol: list = field(default_factory=list)  # cho_factor per stacked problem on the coarsest level
    coarse_sweeps: int = 0  # > 0: the coarsest solve is this many l1-Jacobi sweeps from zero

    @property
    def L(self):
        return len(self.levels) - 1


def box_aggregates(grid, nbatch=1, edge=2):
    """Aggregate index of every fine row and the coarse per-problem grid.

    Fine row (i, j, k) of problem p belongs to coarse cell (i//e, j//e, k//e)
    of problem p (a dimension of extent 1 is kept); coarse rows are ordered
    problem-major, then lexicographically.
    """
    nx, ny, nz = grid
    e = edge
    cx = nx if nx == 1 else (nx + e - 1) // e
    cy = ny if ny == 1 else (ny + e - 1) // e
    cz = nz if nz == 1 else (nz + e - 1) // e
    i = np.arange(nx) if nx == 1 else np.arange(nx) // e
    j = np.arange(ny) if ny == 1 else np.arange(ny) // e
    k = np.arange(nz) if nz == 1 else np.arange(nz) // e
    agg1 = (i[None, None, :] + cx * j[None, :, None] + cx * cy * k[:, None, None]).ravel()
    nc1 = cx * cy * cz
    agg = np.concatenate([agg1 + p * nc1 for p in range(nbatch)])
    return agg.astype(np.int64), (cx, cy, cz)


def prolongator(agg, nc):
    n = agg.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))


def jacobi_weight(A, nbatch=1):
    """omega = 4 / (3 lambda) of the smoothed prolongator, one value per stacked problem, with
    lambda = ||D^{-1} A||_inf (max over the problem's rows of sum_j |a_ij| / a_ii), an upper
    bound of the largest eigenvalue of D^{-1} A (Gershgorin)."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    rows = np.asarray(abs(A).sum(axis=1)).ravel() / d
    per = A.shape[0] // nbatch
    return np.array([4.0 / (3.0 * rows[p * per:(p + 1) * per].max()) for p in range(nbatch)])


DROP_TAU = 2.0**-46


def drop_small(M, tau=DROP_TAU):
    """Remove the entries of a computed product whose magnitude is at most tau times the largest
    of their row: with the smoothed prolongator, entries that cancel exactly in exact arithmetic
    come out of the products as rounding residue (~1e-17) in an order-dependent way."""
    M = sp.csr_matrix(M)
    rowmax = np.zeros(M.shape[0])
    np.maximum.at(rowmax, np.repeat(np.arange(M.shape[0]), np.diff(M.indptr)), np.abs(M.data))
    keep = np.abs(M.data) > tau * np.repeat(rowmax, np.diff(M.indptr))
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))[keep]
    out = sp.csr_matrix((M.data[keep], (rows, M.indices[keep])), shape=M.shape)
    out.sort_indices()
    return out


def smoothed_prolongator(A, Phat, nbatch=1):
    """P = (I - omega D^{-1} A) P_hat (Section 4), omega from jacobi_weight per stacked problem."""
    A = sp.csr_matrix(A)
    omega = np.repeat(jacobi_weight(A, nbatch), A.shape[0] // nbatch)
    S = sp.diags(omega / A.diagonal())
    return (Phat - S @ (A @ Phat)).tocsr()


def build_hierarchy(A, grid, nbatch=1, max_coarse=4096, agg_edge=2, smoothed=False, coarse_sweeps=0,
                    aggregation="box", match_steps=3, vbm_theta=0.08):
    """Levels A_0 = A, A_{l+1} = P_l^T A_l P_l while rows per problem > max_coarse
    (and while the aggregation reduces the level).

    ``agg_edge``: edge of the box aggregates; ``smoothed``: use the smoothed
    prolongator; ``coarse_sweeps`` > 0: solve the coarsest level by that many
    l1-Jacobi sweeps from zero instead of the dense Cholesky factorisation.
    Outside the default (2x2x2 boxes, plain P) the smoothed P and the Galerkin
    operators pass through drop_small.  ``aggregation="matching"``: aggregates
    from ``match_steps`` compatible weighted matchings (oracle.matching) instead
    of boxes (one problem only).  ``aggregation="vbm"``: the classical smoothed
    aggregation aggregates (oracle.vbm) with strength threshold ``vbm_theta``
    on level 0, halved on each coarser level (one problem only).
    """
    from .matching import matching_prolongator
    from .vbm import vbm_tentative
    if aggregation not in ("box", "matching", "vbm"):
        raise ValueError(aggregation)
    if aggregation != "box" and nbatch != 1:
        raise ValueError("graph aggregation takes one problem")
    A = sp.csr_matrix(A)
    A.sort_indices()
    H = Hierarchy(coarse_sweeps=int(coarse_sweeps))
    g = tuple(grid)
    if nbatch > 1:
        g = (g[0], g[1], g[2] // nbatch)
    H.levels.append(Level(A=A, Minv=l1_diagonal(A), grid=g, nbatch=nbatch))
    wsmooth = np.ones(A.shape[0])
    while A.shape[0] // nbatch > max_coarse:
        if aggregation == "matching":
            Pm, wsmooth = matching_prolongator(A, wsmooth, match_steps)
            nc = Pm.shape[1]
            gc = (nc, 1, 1)
        elif aggregation == "vbm":
            Pm = vbm_tentative(A, vbm_theta * 0.5 ** (len(H.levels) - 1))
            nc = Pm.shape[1]
            gc = (nc, 1, 1)
        else:
            agg, gc = box_aggregates(g, nbatch, agg_edge)
            nc = int(np.prod(gc)) * nbatch
            Pm = prolongator(agg, nc)
        if nc >= A.shape[0]:
            break  # aggregation no longer reduces the level: this one is the coarsest
        general = smoothed or agg_edge != 2 or aggregation != "box"
        if smoothed:
            Pm = drop_small(smoothed_prolongator(A, Pm, nbatch))
        Pm.sort_indices()
        Ac = (Pm.T @ A @ Pm).tocsr()
        if general:
            Ac = drop_small(Ac)
        Ac.sort_indices()
        H.levels[-1].P = Pm
        A, g = Ac, gc
        H.levels.append(Level(A=A, Minv=l1_diagonal(A), grid=g, nbatch=nbatch))
    if H.coarse_sweeps > 0:
        return H
    nL = A.shape[0] // nbatch
    dense = A.toarray()
    for p in range(nbatch):
        blk = dense[p * nL:(p + 1) * nL, p * nL:(p + 1) * nL]
        H.chol.append(sla.cho_factor(blk, lower=True))
    return H


def coarse_solve(H, b):
    lv = H.levels[-1]
    if H.coarse_sweeps > 0:
        return smooth_l1jacobi(lv.A, lv.Minv, b, None, H.coarse_sweeps)
    nb = lv.nbatch
    nL = b.size // nb
    out = np.empty_like(b)
    for p in range(nb):
        out[p * nL:(p + 1) * nL] = sla.cho_solve(H.chol[p], b[p * nL:(p + 1) * nL])
    return out


def smoother_params(kind, k, beta=None):
    """Default constants: the optimal beta table (OPTCHEB4) and a*_k (OPTCHEB1)."""
    if kind == OPTCHEB4 and beta is None:
        beta = P.optimal_beta(k)[0]
    a = P.a_star(k) if kind == OPTCHEB1 else None
    return beta, a


def vcycle(H, r, kind, k, beta=None, level=0, betas_by_level=None):
    """z = B r for the multiplicative V-cycle of eq. (amg).

    ``beta`` is used on every level unless ``betas_by_level[l]`` is given
    (per-level weights, used by the learned-beta variant).
    """
    if level == H.L:
        return coarse_solve(H, r)
    lv = H.levels[level]
    bl = beta if betas_by_level is None else betas_by_level[level]
    bl, a = smoother_params(kind, k, bl)
    x = smooth(lv.A, lv.Minv, r, None, kind, k, bl, a)
    res = r - lv.A @ x
    rc = lv.P.T @ res
    xc = vcycle(H, rc, kind, k, beta, level + 1, betas_by_level)
    x = x + lv.P @ xc
    x = smooth(lv.A, lv.Minv, r, x, kind, k, bl, a)
    return x


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float
    history: list
    converged: bool


def pcg(A, b, precond, rtol=1e-8, maxit=1000, flexible=False):
    """Preconditioned CG from x0 = 0; stops when ||r_k|| <= rtol ||b|| (recursive residual).

    ``precond(r)`` returns z = B r.  Standard beta = (r_{k+1}, z_{k+1})/(r_k, z_k);
    flexible beta = (z_{k+1}, r_{k+1} - r_k)/(r_k, z_k).
    """
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.sqrt(np.dot(b, b))
    if nb == 0.0:
        return PCGResult(x, 0, 0.0, [0.0], True)
    hist = [1.0]
    z = precond(r)
    p = z.copy()
    rz = np.dot(r, z)
    for it in range(1, maxit + 1):
        q = A @ p
        pq = np.dot(p, q)
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        rel = np.sqrt(np.dot(r, r)) / nb
        hist.append(rel)
        if rel <= rtol:
            return PCGResult(x, it, rel, hist, True)
        z = precond(r)
        if flexible:
            rz_new = np.dot(r, z)
            beta = np.dot(z, r - r_old) / rz
        else:
            rz_new = np.dot(r, z)
            beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return PCGResult(x, maxit, hist[-1], hist, False)


def amg_pcg(A, b, grid, kind, k, nbatch=1, max_coarse=4096, rtol=1e-8, maxit=1000, H=None,
            flexible=False, beta=None, **hierarchy_opts):
    """Set up the hierarchy (unless given) and solve A x = b with the V-cycle-preconditioned CG."""
    if H is None:
        H = build_hierarchy(A, grid, nbatch, max_coarse, **hierarchy_opts)
    res = pcg(H.levels[0].A, b, lambda r: vcycle(H, r, kind, k, beta), rtol, maxit, flexible)
    return res, H
