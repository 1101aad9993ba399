"""Pins of the oracle's compatible weighted-matching aggregation (Section 4, "Compatible Matching").

* The greedy matching in decreasing edge order equals the matching found by parallel rounds of
  locally dominant edges (an independent formulation, written out here), on graphs with many ties.
* It is a maximal matching whose weight is at least half the maximum (brute force on tiny graphs).
* Edge weights reduce to closed forms on the Laplacians; SplitMix64 reproduces published outputs.
* The tentative prolongator has orthonormal columns and reproduces the smooth vector; three steps
  give aggregates of at most eight vertices; the V-cycle built on it is symmetric with spec(BA) in (0, 1].
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import amg
from oracle import matching as M
from oracle import smoothers as S


def test_splitmix64_published_outputs():
    # the generator seeded with 1234567 (state advanced by the golden gamma before each output)
    state = 1234567
    outs = []
    for _ in range(3):
        outs.append(M.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) & M.MASK64
    assert outs == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def _parallel_locally_dominant(n, i, j, keys):
    """Rounds: every free vertex points at its best free neighbour; mutual pointers are matched."""
    nbrs = [[] for _ in range(n)]
    for e in range(len(i)):
        k = (int(keys[e]), M.edge_hash(int(i[e]), int(j[e])), -int(i[e]), -int(j[e]))
        nbrs[int(i[e])].append((k, int(j[e])))
        nbrs[int(j[e])].append((k, int(i[e])))
    mate = [-1] * n
    while True:
        cand = [-1] * n
        for v in range(n):
            if mate[v] >= 0:
                continue
            free = [(k, u) for k, u in nbrs[v] if mate[u] < 0]
            if free:
                cand[v] = max(free)[1]
        new = [(v, cand[v]) for v in range(n) if cand[v] >= 0 and cand[cand[v]] == v]
        if not new:
            return np.array(mate)
        for v, u in new:
            mate[v] = u


@pytest.mark.parametrize("seed", range(6))
def test_greedy_equals_parallel_locally_dominant(seed):
    rng = np.random.default_rng(seed)
    n = 60
    G = sp.random(n, n, density=0.12, random_state=seed, format="coo")
    edges = {(min(a, b), max(a, b)) for a, b in zip(G.row, G.col) if a != b}
    i = np.array([e[0] for e in sorted(edges)])
    j = np.array([e[1] for e in sorted(edges)])
    keys = rng.integers(0, 4, i.size).astype(np.int64)  # heavy ties
    assert np.array_equal(M.greedy_matching(n, i, j, keys), _parallel_locally_dominant(n, i, j, keys))


def _max_matching_weight(n, edges, wts):
    best = 0
    for r in range(len(edges) + 1):
        for sub in itertools.combinations(range(len(edges)), r):
            used = set()
            ok = True
            for e in sub:
                a, b = edges[e]
                if a in used or b in used:
                    ok = False
                    break
                used.update((a, b))
            if ok:
                best = max(best, sum(wts[e] for e in sub))
    return best


@pytest.mark.parametrize("seed", range(4))
def test_greedy_is_maximal_and_half_optimal(seed):
    rng = np.random.default_rng(10 + seed)
    n = 8
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < 0.4]
    i = np.array([e[0] for e in edges])
    j = np.array([e[1] for e in edges])
    keys = rng.integers(1, 100, len(edges)).astype(np.int64)
    mate = M.greedy_matching(n, i, j, keys)
    for a in range(n):
        if mate[a] >= 0:
            assert mate[mate[a]] == a
    for a, b in edges:  # maximal: no edge with both ends free
        assert mate[a] >= 0 or mate[b] >= 0
    got = sum(int(keys[e]) for e, (a, b) in enumerate(edges) if mate[a] == b)
    assert 2 * got >= _max_matching_weight(n, edges, [int(k) for k in keys])


def test_edge_weight_closed_forms():
    # 2D 5-point Laplacian, w = 1: 1 - 2 (-1) / (4 + 4) = 5/4 on every edge
    A = W.poisson2d_5pt(6, 5).to_scipy()
    i, j, keys = M.edge_weights(A, np.ones(A.shape[0]))
    assert np.all(keys == int(1.25 * 2**30)) and i.size == (A.nnz - A.shape[0]) // 2
    # scaling w by a constant and A by a positive factor changes nothing
    i2, j2, keys2 = M.edge_weights(3.0 * A, 2.0 * np.ones(A.shape[0]))
    assert np.array_equal(keys, keys2)
    # 27-point Q1: an exactly zero face entry has weight 1, an edge entry 1 + 2 (1/6) / (16/3)
    Q = W.q1_27pt(4).to_scipy()
    i, j, keys = M.edge_weights(Q, np.ones(Q.shape[0]))
    vals = {int(k) for k in keys}
    assert int(2**30) in vals and int(np.rint((1 + (1 / 3) / (16 / 3)) * 2**30)) in vals


def test_aggregates_and_tentative_prolongator():
    A = W.fv_diffusion(np.exp(2.0 * W.gaussian_random_field((10, 9, 8), 3.0, 4))).to_scipy()
    w0 = np.ones(A.shape[0])
    P, w = M.matching_prolongator(A, w0, steps=3)
    sizes = np.bincount(P.indices, minlength=P.shape[1])
    assert sizes.min() >= 1 and sizes.max() <= 8 and sizes.sum() == A.shape[0]
    assert np.all(np.diff(P.indptr) == 1)  # one aggregate per vertex
    assert np.abs((P.T @ P).toarray() - np.eye(P.shape[1])).max() <= 1e-15
    assert np.abs(P @ w - w0).max() <= 1e-15
    # aggregates are numbered by their smallest vertex
    first = np.array([P.indices.tolist().index(c) for c in range(P.shape[1])])
    assert np.all(np.diff(first) > 0)
    # one step: pairs of neighbours only
    P1, Ac, nu, mate = M.matching_step(A, w0)
    for v in np.nonzero(mate >= 0)[0]:
        assert A[v, mate[v]] != 0
    assert abs(Ac - Ac.T).max() <= 1e-14 * abs(Ac).max()


@pytest.mark.parametrize("smoothed", [False, True])
@pytest.mark.parametrize("kind", [S.L1JAC, S.OPTCHEB4, S.OPTCHEB1])
def test_matching_vcycle_symmetric_and_spectrum(smoothed, kind):
    M_ = W.fv_diffusion(np.exp(W.gaussian_random_field((9, 9, 9), 3.0, 2)))
    A = M_.to_scipy()
    H = amg.build_hierarchy(A, M_.grid, max_coarse=30, aggregation="matching", smoothed=smoothed)
    assert H.L >= 1
    n = A.shape[0]
    I = np.eye(n)
    B = np.column_stack([amg.vcycle(H, I[:, c], kind, 3) for c in range(n)])
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    lam, V = np.linalg.eigh(A.toarray())
    Ah = V @ np.diag(np.sqrt(lam)) @ V.T
    mu = np.linalg.eigvalsh(Ah @ B @ Ah)
    assert mu.min() > 0 and mu.max() <= 1.0 + 1e-12


def test_matching_needs_one_problem():
    big = W.stack_block_diagonal([W.poisson3d_7pt(4), W.poisson3d_7pt(4)])
    with pytest.raises(ValueError):
        amg.build_hierarchy(big.to_scipy(), big.grid, nbatch=2, max_coarse=8, aggregation="matching")
