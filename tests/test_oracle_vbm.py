"""Pins of the oracle's classical smoothed-aggregation (VBM) aggregates (Section 4, "VBM").

* The roots of phase 1, taken greedily in decreasing hash order, equal the roots found by parallel
  rounds of locally first vertices of the squared strength graph (an independent formulation,
  written out here with sparse boolean products).
* Brute force on small graphs: the roots are pairwise at least three strong edges apart and every
  vertex is within two of a root; the phase-1 aggregates are exactly the roots' neighbourhoods;
  every other vertex sits with the phase-1 aggregate of its strongest aggregated neighbour.
* The threshold: equality counts as strong (a chain with diagonal 4 at theta = 1/4), one step of
  the 2^-30 grid above it nothing is strong, exact zeros are never strong, the decision reads a_ij
  from the smaller row, and couplings within rounding of each other compare equal.
* Closed forms: on the 1D Laplacian the aggregates are intervals of 2 to 5 vertices, and a vertex
  halfway between two roots four apart joins the left one (equal strengths, smaller index); on the
  anisotropic 5-point operator the aggregates stay inside grid lines of the strong direction.
* The V-cycle built on the aggregates is symmetric with spec(BA) in (0, 1].
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import amg
from oracle import matching as M
from oracle import smoothers as S
from oracle import vbm as V


def _roots_parallel(Sg):
    """Rounds: an undecided vertex whose hash is the largest among the undecided vertices within
    two strong edges becomes a root; the undecided vertices within two edges of a root drop out."""
    n = Sg.shape[0]
    C = (Sg + sp.identity(n, format="csr")).astype(bool).astype(np.int8).tocsr()  # closed neighbourhoods
    h = np.array([M.splitmix64(v) for v in range(n)], dtype=object)
    state = np.zeros(n, dtype=np.int8)  # 0 undecided, 1 root, 2 out
    while (state == 0).any():
        und = np.flatnonzero(state == 0)
        m1 = [max((h[u] for u in C.indices[C.indptr[j]:C.indptr[j + 1]] if state[u] == 0), default=-1)
              for j in range(n)]
        for i in und:
            m2 = max(m1[j] for j in C.indices[C.indptr[i]:C.indptr[i + 1]])
            if m2 == h[i]:
                state[i] = 1
        roots = (state == 1).astype(np.int8)
        near = (C @ (C @ roots)) > 0
        state[(state == 0) & near] = 2
    return np.flatnonzero(state == 1)


def _graphs():
    yield "poisson2d", W.poisson2d_5pt(9, 7).to_scipy(), 0.08
    yield "q1_27pt", W.q1_27pt(5).to_scipy(), 0.0
    yield "aniso_q1", W.anisotropy2d_q1(12)[0].to_scipy(), 0.08
    yield "fv", W.fv_diffusion(np.exp(2.0 * W.gaussian_random_field((7, 6, 5), 3.0, 1))).to_scipy(), 0.25
    rng = np.random.default_rng(5)
    R = sp.random(70, 70, density=0.06, random_state=5, format="csr")
    R = abs(R + R.T)
    R.setdiag(0)
    R.eliminate_zeros()
    Ar = sp.diags(np.asarray(R.sum(axis=1)).ravel() + rng.uniform(0.1, 1.0, 70)) - R
    yield "random", sp.csr_matrix(Ar), 0.1


@pytest.mark.parametrize("name,A,theta", list(_graphs()), ids=[g[0] for g in _graphs()])
def test_phase1_roots_equal_parallel_rounds_and_phases_hold(name, A, theta):
    agg, nc = V.vbm_aggregates(A, theta)
    Sg = V.strength_graph(A, theta)
    n = A.shape[0]
    roots = _roots_parallel(Sg)
    C = (Sg + sp.identity(n, format="csr")).astype(bool).toarray()
    C2 = (C.astype(np.int64) @ C.astype(np.int64)) > 0
    # independence and maximality in the squared graph
    Rm = np.zeros(n, dtype=bool)
    Rm[roots] = True
    sub = C2[np.ix_(roots, roots)]
    assert np.array_equal(sub, np.eye(roots.size, dtype=bool))
    assert C2[:, Rm].any(axis=1).all()
    # aggregates numbered by increasing root; one aggregate per root
    assert nc == roots.size
    assert np.array_equal(agg[roots], np.arange(nc))
    # phase 1: the neighbourhood of each root is its aggregate
    owner = np.full(n, -1)
    for r in roots:
        owner[C[r]] = agg[r]
    in1 = owner >= 0
    assert np.array_equal(agg[in1], owner[in1])
    # phase 2: strongest aggregated neighbour, ties to the smaller index
    Sd = Sg.toarray()
    for v in np.flatnonzero(~in1):
        cand = [u for u in np.flatnonzero(Sd[v]) if owner[u] >= 0]
        assert cand, (name, v)
        best = max(cand, key=lambda u: (Sd[v, u], -u))
        assert agg[v] == owner[best]


def test_threshold_equality_zeros_and_row_choice():
    # the 5-point operator on a 12 x 1 grid: a chain with diagonal 4 and off-diagonal -1 (the
    # y-couplings go to eliminated boundary nodes): a^2 / (a_ii a_jj) = 1/16 = theta^2 at 1/4
    L1 = W.poisson2d_5pt(12, 1).to_scipy()
    assert np.all(L1.diagonal() == 4.0)
    S1 = V.strength_graph(L1, 0.25)
    assert S1.nnz == 2 * (L1.shape[0] - 1) and np.all(S1.data == 2.0**26 + 1)
    t_up = np.sqrt((2.0**26 + 1) / 2.0**30)  # the next point of the grid
    assert np.rint(t_up * t_up * 2.0**30) == 2.0**26 + 1
    assert V.strength_graph(L1, t_up).nnz == 0
    agg, nc = V.vbm_aggregates(L1, 0.3)
    assert nc == L1.shape[0] and np.array_equal(agg, np.arange(nc))
    H = amg.build_hierarchy(L1, (12, 1, 1), max_coarse=2, aggregation="vbm", vbm_theta=0.3)
    assert H.L == 0  # nothing to aggregate: the fine level is the coarsest
    # explicit zeros (the 27-point face entries) are never strong, even at theta = 0
    Q = W.q1_27pt(4).to_scipy()
    nonzero_off = int(((Q != 0).sum()) - Q.shape[0])
    assert V.strength_graph(Q, 0.0).nnz == nonzero_off
    # a_ij and a_ji that differ beyond the grid: the smaller row decides for both ends
    B = sp.lil_matrix(np.array([[2.0, -1.0, 0.0], [-1.0, 2.0, -1.0], [0.0, -1.0, 2.0]]))
    low = -0.5 * (1.0 - 2.0**-20)
    B[0, 1], B[1, 0] = -0.5, low
    Sb = V.strength_graph(sp.csr_matrix(B), 0.25).toarray()
    assert Sb[0, 1] and Sb[1, 0]  # 0.25 / 4 = theta^2 from row 0
    B[0, 1], B[1, 0] = low, -0.5
    Sb = V.strength_graph(sp.csr_matrix(B), 0.25).toarray()
    assert not Sb[0, 1] and not Sb[1, 0]
    assert np.array_equal(Sb, Sb.T)
    # couplings one ulp apart fall on one grid point: phase 2 then breaks the tie by index
    C = sp.lil_matrix((3, 3))
    C.setdiag([2.0, 2.0, 2.0])
    C[0, 1] = C[1, 0] = -1.0
    C[1, 2] = C[2, 1] = np.nextafter(-1.0, -2.0)
    Sc = V.strength_graph(sp.csr_matrix(C), 0.0).toarray()
    assert Sc[1, 0] == Sc[1, 2]


@pytest.mark.parametrize("n", [10, 31, 64, 257])
def test_1d_intervals_and_tie_rule(n):
    T = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    agg, nc = V.vbm_aggregates(T, 0.08)
    assert np.all(np.diff(agg) >= 0)  # contiguous intervals in vertex order
    sizes = np.bincount(agg)
    assert sizes.min() >= 2 and sizes.max() <= 5
    assert np.all(sizes[1:-1] >= 3)
    rts = _roots_parallel(V.strength_graph(T, 0.08))
    assert np.array_equal(agg[rts], np.arange(nc))
    for r0, r1 in zip(rts[:-1], rts[1:]):
        assert 3 <= r1 - r0 <= 5
        if r1 - r0 == 4:
            assert agg[r0 + 2] == agg[r0]  # equal strengths: the smaller neighbour index wins
        if r1 - r0 == 5:
            assert agg[r0 + 2] == agg[r0] and agg[r0 + 3] == agg[r1]


def test_anisotropic_aggregates_follow_the_strong_direction():
    nx, ny, eps = 16, 12, 0.01
    A = W.stencil_csr((nx, ny, 1), [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0)],
                      [2.0 + 2.0 * eps, -1.0, -1.0, -eps, -eps]).to_scipy()
    # |a_x| / a_ii = 1 / 2.02 is strong at theta 0.08; eps / 2.02 is not
    agg, nc = V.vbm_aggregates(A, 0.08)
    y = np.arange(A.shape[0]) // nx
    for c in range(nc):
        assert np.unique(y[agg == c]).size == 1
    agg0, nc0 = V.vbm_aggregates(A, 0.0)
    assert nc0 < nc and max(np.unique(y[agg0 == c]).size for c in range(nc0)) > 1


@pytest.mark.parametrize("smoothed", [False, True])
@pytest.mark.parametrize("kind", [S.L1JAC, S.OPTCHEB4, S.OPTCHEB1])
def test_vbm_vcycle_symmetric_and_spectrum(smoothed, kind):
    M_ = W.fv_diffusion(np.exp(W.gaussian_random_field((9, 9, 9), 3.0, 2)))
    A = M_.to_scipy()
    H = amg.build_hierarchy(A, M_.grid, max_coarse=30, aggregation="vbm", smoothed=smoothed)
    assert H.L >= 1
    n = A.shape[0]
    I = np.eye(n)
    B = np.column_stack([amg.vcycle(H, I[:, c], kind, 3) for c in range(n)])
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    lam, Vv = np.linalg.eigh(A.toarray())
    Ah = Vv @ np.diag(np.sqrt(lam)) @ Vv.T
    mu = np.linalg.eigvalsh(Ah @ B @ Ah)
    assert mu.min() > 0 and mu.max() <= 1.0 + 1e-12


def test_vbm_pcg_converges_and_needs_one_problem():
    M_ = W.poisson3d_7pt(14)
    A = M_.to_scipy()
    b = W.rhs_uniform(A.shape[0], 9)
    r, H = amg.amg_pcg(A, b, M_.grid, S.OPTCHEB4, 2, max_coarse=64, aggregation="vbm", smoothed=True)
    assert H.L >= 2 and r.iters < 30
    assert np.linalg.norm(b - A @ r.x) <= 1.0001e-8 * np.linalg.norm(b)
    big = W.stack_block_diagonal([W.poisson3d_7pt(4), W.poisson3d_7pt(4)])
    with pytest.raises(ValueError):
        amg.build_hierarchy(big.to_scipy(), big.grid, nbatch=2, max_coarse=8, aggregation="vbm")


def test_aggregates_stable_under_rounding_of_coarse_operators():
    """Smoothed Galerkin levels hold couplings that are equal in exact arithmetic but differ in
    rounding; a relative perturbation of one ulp in any entry leaves the aggregates unchanged."""
    M_ = W.poisson3d_7pt(16)
    H = amg.build_hierarchy(M_.to_scipy(), M_.grid, max_coarse=40, aggregation="vbm", smoothed=True)
    assert H.L >= 2
    rng = np.random.default_rng(0)
    for l in range(1, H.L + 1):
        A1 = H.levels[l].A
        ref = V.vbm_aggregates(A1, 0.08 * 0.5**l)
        for _ in range(3):
            B = A1.copy()
            B.data = B.data * (1.0 + rng.choice([-1.0, 0.0, 1.0], B.data.size) * 2.0**-52)
            agg, nc = V.vbm_aggregates(B, 0.08 * 0.5**l)
            assert nc == ref[1] and np.array_equal(agg, ref[0])
