"""Classical smoothed-aggregation (VBM) aggregates (oracle, test infrastructure only).

Section 4 names, besides compatible matching, the smoothed aggregation of Vanek,
Mandel and Brezina, determined on each process's local rows ("decoupled").  On
one device every row is local, so decoupled and coupled coincide.  The paper
defers the construction to that reference; restated here, with the points it
leaves open fixed as follows.

* Strength of connection on level l with threshold theta_l = theta / 2^l (the
  threshold of the cited method is halved on each coarser level): the coupling
  of the edge {i, j}, i != j, is s_ij = a_ij^2 / |a_ii a_jj| (the square of
  |a_ij| / sqrt(|a_ii a_jj|)), with a_ij read from the row of the smaller index
  so that both ends see one value.  It is rounded to a grid of 2^-30,
  q_ij = rint(2^30 s_ij), so that couplings equal in exact arithmetic compare
  equal although the Galerkin products that made them differ in rounding.  The
  edge is strong when a_ij != 0 and q_ij >= rint(2^30 theta_l^2).  N_i is i with
  its strong neighbours.
* Phase 1 (root neighbourhoods): the vertices are visited in decreasing order of
  the SplitMix64 hash of their index; a vertex whose neighbourhood N_i meets no
  aggregate formed so far becomes a root and N_i its aggregate.  N_i and N_r are
  disjoint exactly when i and r are at least three strong edges apart, so the
  roots are the greedy maximal independent set of the square of the strength
  graph in that order, and the result does not depend on how the visit is
  scheduled (it equals the rounds of locally first vertices that the GPU runs).
* Phase 2 (enlargement): a vertex outside every phase-1 aggregate joins the
  phase-1 aggregate of its strong neighbour j with the largest q_ij (ties: the
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

QUANT = 2.0**30


def strength_graph(A, theta):
    """Symmetric strength graph (CSR, no diagonal) holding q_ij + 1 for each edge (never zero)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    d = A.diagonal()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    upper = cols > rows
    i, j, a = rows[upper], cols[upper], A.data[upper]
    q = np.rint((a * a) / np.abs(d[i] * d[j]) * QUANT)
    qt = np.rint(float(theta) * float(theta) * QUANT)
    strong = (a != 0.0) & (q >= qt)
    i, j, q = i[strong], j[strong], q[strong] + 1.0
    S = sp.csr_matrix((np.concatenate([q, q]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n))
    S.sort_indices()
    return S


def vbm_aggregates(A, theta):
    """Aggregate index of every row (numbered by increasing root) and the number of aggregates."""
    S = strength_graph(A, theta)
    n = S.shape[0]
    ptr, nbr, key = S.indptr, S.indices, S.data

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
            if best < 0 or key[p] > key[best] or (key[p] == key[best] and u < int(nbr[best])):
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
