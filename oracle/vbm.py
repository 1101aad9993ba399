"""Classical smoothed-aggregation (VBM) aggregates (oracle, test infrastructure only).

Section 4 names, besides compatible matching, the smoothed aggregation of Vanek,
Mandel and Brezina, determined on each process's local rows ("decoupled").  On
one device every row is local, so decoupled and coupled coincide.  The paper
defers the construction to that reference; restated here, with the points it
leaves open fixed as follows.

* Strength of connection on level l with threshold theta_l = theta / 2^l (the
  threshold of the cited method is halved on each coarser level): the edge
  {i, j}, i != j, is strong when a_ij != 0 and a_ij^2 >= theta_l^2 |a_ii a_jj|
  (the squared form of |a_ij| >= theta_l sqrt(|a_ii a_jj|)), with a_ij read from
  the row of the smaller index so that both ends see one decision.  N_i is i
  with its strong neighbours.
* Phase 1 (root neighbourhoods): the vertices are visited in decreasing order of
  the SplitMix64 hash of their index; a vertex whose neighbourhood N_i meets no
  aggregate formed so far becomes a root and N_i its aggregate.  N_i and N_r are
  disjoint exactly when i and r are at least three strong edges apart, so the
  roots are the greedy maximal independent set of the square of the strength
  graph in that order, and the result does not depend on how the visit is
  scheduled (it equals the rounds of locally first vertices that the GPU runs).
* Phase 2 (enlargement): a vertex outside every phase-1 aggregate joins the
  phase-1 aggregate of its strong neighbour j with the largest |a_ij| (ties: the
  smallest j).  By maximality every such vertex has one.
* Phase 3 (remainder): whatever is still unassigned forms a singleton (never
  reached when phase 1 is maximal; kept so that every row has an aggregate).
* Aggregates are numbered in increasing order of their root; the tentative
  prolongator is piecewise constant with entries 1.0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .matching import splitmix64


def strength_graph(A, theta):
    """Symmetric boolean strength graph (CSR, no diagonal) and the |a_ij| of its edges."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    d = A.diagonal()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    upper = cols > rows
    i, j, a = rows[upper], cols[upper], A.data[upper]
    t2 = float(theta) * float(theta)
    strong = (a != 0.0) & (a * a >= t2 * np.abs(d[i] * d[j]))
    i, j, a = i[strong], j[strong], np.abs(a[strong])
    S = sp.csr_matrix((np.concatenate([a, a]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n))
    S.sort_indices()
    return S


def vbm_aggregates(A, theta):
    """Aggregate index of every row (numbered by increasing root) and the number of aggregates."""
    S = strength_graph(A, theta)
    n = S.shape[0]
    ptr, nbr, mag = S.indptr, S.indices, S.data

    def neigh(v):
        return nbr[ptr[v]:ptr[v + 1]]

    # phase 1 in decreasing hash order
    order = sorted(range(n), key=lambda v: -splitmix64(v))
    owner = np.full(n, -1, dtype=np.int64)  # root of the phase-1 aggregate holding the vertex
    is_root = np.zeros(n, dtype=bool)
    for v in order:
        hood = [v] + [int(u) for u in neigh(v)]
        if all(owner[u] < 0 for u in hood):
            is_root[v] = True
            for u in hood:
                owner[u] = v
    # phase 2 reads the phase-1 owners only
    final = owner.copy()
    for v in range(n):
        if owner[v] >= 0:
            continue
        best = -1
        for p in range(ptr[v], ptr[v + 1]):
            u = int(nbr[p])
            if owner[u] < 0:
                continue
            if best < 0 or mag[p] > mag[best] or (mag[p] == mag[best] and u < int(nbr[best])):
                best = p
        if best >= 0:
            final[v] = owner[int(nbr[best])]
    # phase 3: singletons
    left = final < 0
    is_root |= left
    final[left] = np.flatnonzero(left)
    rank = np.cumsum(is_root) - 1
    return rank[final], int(is_root.sum())


def vbm_tentative(A, theta):
    """Piecewise-constant tentative prolongator (entries 1.0) of the VBM aggregates."""
    agg, nc = vbm_aggregates(A, theta)
    n = agg.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))
