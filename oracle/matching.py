"""Compatible weighted-matching aggregation (oracle, test infrastructure only).

Section 4 builds one of its two hierarchies from aggregates given by repeated
approximate weighted matchings of the graph of A (aggregates of size up to 8
after three matching steps), with the resulting prolongator optionally used as
the tentative prolongator of the smoothed prolongator.  The paper defers the
construction to the compatible-matching literature it cites; the published
method restated here:

* Edge weights of the graph of A for a smooth vector w (w = 1 on the first
  level): w_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2).  An edge is an
  off-diagonal stored entry; a_ij is taken from the row with the smaller index,
  so that the weight of an edge does not depend on the rounding of a Galerkin
  product that is symmetric only up to rounding.
* The weights are rounded to a grid of 2^-30 before they are compared, so that
  rounding noise of the coarse operators cannot reorder edges whose weights are
  equal in exact arithmetic.
* Matching: the greedy matching in decreasing edge order (a half-approximation
  of the maximum-weight matching), with ties of the rounded weight broken by a
  hash of the edge (SplitMix64 of (min << 32 | max), larger first) and then by
  (min, max) ascending.  It equals the matching of locally dominant edges
  found in parallel rounds, which is what the GPU computes.
* A matched pair {i, j} forms an aggregate, an unmatched vertex a singleton.
  Aggregates are numbered by their smallest vertex.  The tentative prolongator
  column of aggregate J holds w_i / nu_J on its vertices, nu_J = ||w|_J||, so
  P_hat has orthonormal columns and P_hat nu = w; the next step uses P_hat^T A P_hat
  and the smooth vector nu.
* ``steps`` matching steps are composed: P_hat = P_1 P_2 ... P_steps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

QUANT = 2.0**30
MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea and Flood; constants as published by Vigna)."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & MASK64
    return x ^ (x >> 31)


def edge_hash(i: int, j: int) -> int:
    lo, hi = (i, j) if i < j else (j, i)
    return splitmix64((lo << 32) | hi)


def edge_weights(A, w):
    """Rounded weights of the edges i < j: (rows, cols, keys) with keys = rint(w_ij * 2^30) (int64)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    d = A.diagonal()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    upper = cols > rows
    i, j, a = rows[upper], cols[upper], A.data[upper]
    num = (2.0 * a) * (w[i] * w[j])
    den = (d[i] * w[i]) * w[i] + (d[j] * w[j]) * w[j]
    wij = 1.0 - num / den
    keys = np.rint(wij * QUANT).astype(np.int64)
    return i, j, keys


def greedy_matching(n, i, j, keys):
    """mate[v] (-1 when unmatched) of the greedy matching over the edges in decreasing order of
    (key, hash, -min, -max)."""
    order = sorted(range(len(i)), key=lambda e: (-int(keys[e]), -edge_hash(int(i[e]), int(j[e])),
                                                 int(i[e]), int(j[e])))
    mate = np.full(n, -1, dtype=np.int64)
    for e in order:
        a, b = int(i[e]), int(j[e])
        if mate[a] < 0 and mate[b] < 0:
            mate[a] = b
            mate[b] = a
    return mate


def pair_aggregates(mate):
    """Aggregate index of every vertex (numbered by the aggregate's smallest vertex) and their count."""
    n = mate.size
    v = np.arange(n)
    leader = np.where(mate < 0, v, np.minimum(v, mate))
    is_leader = leader == v
    rank = np.cumsum(is_leader) - 1
    return rank[leader], int(is_leader.sum())


def matching_step(A, w):
    """One matching step: (P_hat, A_c = P_hat^T A P_hat with the drop rule, nu)."""
    from .amg import drop_small
    A = sp.csr_matrix(A)
    n = A.shape[0]
    i, j, keys = edge_weights(A, w)
    mate = greedy_matching(n, i, j, keys)
    agg, nc = pair_aggregates(mate)
    v = np.arange(n)
    lo = np.where(mate < 0, v, np.minimum(v, mate))
    hi = np.where(mate < 0, v, np.maximum(v, mate))
    nu_v = np.where(mate < 0, np.abs(w), np.sqrt(w[lo] * w[lo] + w[hi] * w[hi]))
    nu = np.zeros(nc)
    nu[agg] = nu_v
    P = sp.csr_matrix((w / nu_v, (v, agg)), shape=(n, nc))
    Ac = drop_small((P.T @ A @ P).tocsr())
    return P, Ac, nu, mate


def matching_prolongator(A, w=None, steps=3):
    """Composite tentative prolongator of ``steps`` matching steps and the coarse smooth vector."""
    A = sp.csr_matrix(A)
    w = np.ones(A.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    P = None
    Acur = A
    for _ in range(steps):
        Ps, Acur, w, _ = matching_step(Acur, w)
        P = Ps if P is None else (P @ Ps).tocsr()
        if Acur.shape[0] <= 1:
            break
    P.sort_indices()
    return P, w
