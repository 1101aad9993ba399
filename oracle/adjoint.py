"""Derivatives of the V-cycle with respect to the smoother weights (oracle, test infrastructure only).

The optimal 4th-kind smoother (eq. polsmootheropt) is linear in its weights
beta_j, and the V-cycle of eq. (amg) is a polynomial in them, hence an
analytic function: its derivative is obtained exactly (to rounding) by the
complex-step rule d f/d beta = Im f(beta + i h) / h, h = 1e-30, running the
plain oracle V-cycle in complex arithmetic.  Norms are written as
sqrt(sum r_i^2) without conjugation so that they stay analytic.

Stacked problems are independent (block-diagonal A, per-problem weights), so
the oracle treats each one with its own hierarchy.
"""
from __future__ import annotations

import numpy as np

from . import amg
from .smoothers import OPTCHEB4


def _norm_analytic(v):
    return np.sqrt(np.sum(v * v))


def vcycle_beta(H, r, k, betas):
    """z = B(beta) r with betas[l] (length k) on level l (optimal 4th kind)."""
    return amg.vcycle(H, r, OPTCHEB4, k, betas_by_level=list(betas) + [None])


def two_cycle_ratio(H, b, k, betas):
    """||r_2|| / ||r_0|| with r_0 = b, r_{m+1} = r_m - A B(beta) r_m (two stationary V-cycle steps from x = 0)."""
    A = H.levels[0].A
    r0 = b
    r1 = r0 - A @ vcycle_beta(H, r0, k, betas)
    r2 = r1 - A @ vcycle_beta(H, r1, k, betas)
    return _norm_analytic(r2) / _norm_analytic(r0)


def loss(Hs, bs, k, betas_p):
    """Mean over problems of the two-cycle residual ratio; betas_p[p][l] = weights of problem p on level l."""
    return sum(two_cycle_ratio(H, b, k, bp) for H, b, bp in zip(Hs, bs, betas_p)) / len(Hs)


def grad_complex_step(Hs, bs, k, betas_p, h=1e-30):
    """d loss / d beta[p][l][j] by the complex step, array of shape (P, nsmooth_levels, k)."""
    P = len(Hs)
    nl = len(betas_p[0])
    g = np.zeros((P, nl, k))
    for p in range(P):
        for l in range(nl):
            for j in range(k):
                bc = [np.array(v, dtype=complex) for v in betas_p[p]]
                bc[l][j] += 1j * h
                g[p, l, j] = two_cycle_ratio(Hs[p], bs[p], k, bc).imag / h / P
    return g


def grad_central_fd(Hs, bs, k, betas_p, h=1e-6):
    """The same derivative by central differences (an independent check of the complex step)."""
    P = len(Hs)
    nl = len(betas_p[0])
    g = np.zeros((P, nl, k))
    for p in range(P):
        for l in range(nl):
            for j in range(k):
                bp = [np.array(v, dtype=float) for v in betas_p[p]]
                bm = [np.array(v, dtype=float) for v in betas_p[p]]
                bp[l][j] += h
                bm[l][j] -= h
                g[p, l, j] = (two_cycle_ratio(Hs[p], bs[p], k, bp) - two_cycle_ratio(Hs[p], bs[p], k, bm)) / (2 * h) / P
    return g


def linear_functional_grad(H, r, c, k, betas, h=1e-30):
    """d <c, B(beta) r> / d beta[l][j] by the complex step, shape (nsmooth_levels, k)."""
    nl = len(betas)
    g = np.zeros((nl, k))
    for l in range(nl):
        for j in range(k):
            bc = [np.array(v, dtype=complex) for v in betas]
            bc[l][j] += 1j * h
            g[l, j] = np.sum(c * vcycle_beta(H, r, k, bc)).imag / h
    return g
