"""Pins of the oracle's smoothed-aggregation ingredients (Section 4): the smoothed prolongator
P = (I - omega D^{-1} A) P_hat with omega = 4 / (3 ||D^{-1} A||_inf), box aggregates of any edge,
the coarsest solve by l1-Jacobi sweeps and the V-cycle built from them."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import amg
from oracle import smoothers as S

KINDS = [S.L1JAC, S.CHEB4, S.OPTCHEB4, S.OPTCHEB1]


def _lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


@pytest.mark.parametrize("edge,column", [(3, [1, 2, 3, 2, 1]), (2, [1, 2, 2, 1])])
def test_1d_smoothed_prolongator_is_the_textbook_hat(edge, column):
    """1D Laplacian: D^{-1} A = tridiag(-1/2, 1, -1/2), ||.||_inf = 2, omega = 2/3, so
    I - omega D^{-1} A = tridiag(1/3, 1/3, 1/3) and an interior column of P is the
    aggregate's indicator averaged with its two neighbours: (1, 2, 3, 2, 1)/3 for
    aggregates of 3, (1, 2, 2, 1)/3 for aggregates of 2."""
    n = 24
    A = _lap1d(n)
    agg, gc = amg.box_aggregates((n, 1, 1), 1, edge)
    assert amg.jacobi_weight(A)[0] == pytest.approx(2.0 / 3.0, rel=1e-15)
    P = amg.smoothed_prolongator(A, amg.prolongator(agg, gc[0])).toarray()
    J = 3
    col = P[:, J]
    nz = np.nonzero(np.abs(col) > 1e-15)[0]
    assert list(nz) == list(range(edge * J - 1, edge * J + edge + 1))
    assert np.allclose(col[nz] * 3.0, column, rtol=0, atol=1e-14)


def test_jacobi_weight_is_a_gershgorin_bound():
    M = W.fv_diffusion(np.exp(2.0 * W.gaussian_random_field((6, 7, 5), 3.0, 9)))
    A = M.to_scipy()
    d = A.diagonal()
    lam_max = np.linalg.eigvals(np.diag(1 / d) @ A.toarray()).real.max()
    lam = 4.0 / (3.0 * amg.jacobi_weight(A)[0])
    assert lam >= lam_max * (1 - 1e-12)
    # 7-point Poisson: sum |a_ij| / a_ii = 12 / 6 on interior rows
    assert amg.jacobi_weight(W.poisson3d_7pt(6).to_scipy())[0] == pytest.approx(2.0 / 3.0, rel=1e-15)


def test_jacobi_weight_per_stacked_problem():
    mats = [W.poisson3d_7pt(4), W.fv_diffusion(np.exp(3.0 * W.gaussian_random_field((4, 4, 4), 2.0, 3)))]
    big = W.stack_block_diagonal(mats).to_scipy()
    w = amg.jacobi_weight(big, nbatch=2)
    assert w[0] == pytest.approx(amg.jacobi_weight(mats[0].to_scipy())[0], rel=1e-15)
    assert w[1] == pytest.approx(amg.jacobi_weight(mats[1].to_scipy())[0], rel=1e-15)


def test_smoothed_prolongator_keeps_constants_where_a_annihilates_them():
    """P 1 = (I - omega D^{-1} A) 1: equal to 1 on rows whose row sum is zero (the rows of the
    anisotropic problem away from the Dirichlet face)."""
    A2, _ = W.anisotropy2d_q1(12)
    A = A2.to_scipy()
    agg, gc = amg.box_aggregates(A2.grid, 1, 2)
    P = amg.smoothed_prolongator(A, amg.prolongator(agg, int(np.prod(gc))))
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    free = np.abs(rowsum) <= 1e-13 * A.diagonal()
    assert free.sum() > A.shape[0] // 2
    assert np.allclose((P @ np.ones(P.shape[1]))[free], 1.0, rtol=0, atol=1e-13)
    assert np.all((P @ np.ones(P.shape[1]))[~free] < 1.0)


def test_smoothed_galerkin_brute_force():
    """A_c = P^T A P against explicit loops: P[i, J] = [agg(i) = J] - omega / a_ii sum_{j in J} a_ij."""
    M = W.fv_diffusion(np.exp(W.gaussian_random_field((5, 4, 6), 2.0, 4)))
    A = M.to_scipy()
    Ad = A.toarray()
    H = amg.build_hierarchy(A, M.grid, max_coarse=A.shape[0] - 1, smoothed=True)
    agg, gc = amg.box_aggregates(M.grid)
    nc = int(np.prod(gc))
    n = A.shape[0]
    lam = max(sum(abs(Ad[i, j]) for j in range(n)) / Ad[i, i] for i in range(n))
    omega = 4.0 / (3.0 * lam)
    Pd = np.zeros((n, nc))
    for i in range(n):
        Pd[i, agg[i]] += 1.0
        for j in range(n):
            Pd[i, agg[j]] -= omega / Ad[i, i] * Ad[i, j]
    assert np.allclose(H.levels[0].P.toarray(), Pd, rtol=0, atol=1e-14)
    Ac = np.zeros((nc, nc))
    for I in range(nc):
        for J in range(nc):
            Ac[I, J] = sum(Pd[i, I] * sum(Ad[i, j] * Pd[j, J] for j in range(n) if Ad[i, j] != 0)
                           for i in range(n) if Pd[i, I] != 0)
    assert np.allclose(H.levels[1].A.toarray(), Ac, rtol=1e-13, atol=1e-13 * np.abs(Ac).max())


def test_box_aggregates_edge3():
    agg, gc = amg.box_aggregates((7, 4, 1), 1, 3)
    assert gc == (3, 2, 1)
    sizes = np.bincount(agg)
    assert sorted(set(sizes)) == [1, 3, 9] and sizes.sum() == 28
    assert agg[6 + 7 * 3] == 2 + 3 * 1


def test_drop_small_removes_only_rounding_residue():
    M = sp.csr_matrix(np.array([[4.0, 1e-17, -1.0], [3e-14, 2.0, 0.0], [-1.0, 0.0, 4.0]]))
    D = amg.drop_small(M).toarray()
    assert D[0, 1] == 0.0 and D[1, 0] == 3e-14 and D[1, 2] == 0.0
    assert amg.drop_small(M).nnz == 6  # the explicit zeros go too


@pytest.mark.parametrize("edge", [2, 3])
def test_smoothed_products_have_no_cancellations_on_the_workloads(edge):
    """On the stencil workloads the smoothed P and P^T A P keep their full structural pattern,
    so the drop rule changes nothing there."""
    for M in (W.q1_27pt(12), W.anisotropy2d_q1(16)[0], W.poisson3d_7pt(16)):
        A = M.to_scipy()
        agg, gc = amg.box_aggregates(M.grid, 1, edge)
        P = amg.smoothed_prolongator(A, amg.prolongator(agg, int(np.prod(gc))))
        structural = (abs(P).T @ abs(A) @ abs(P)).tocsr()
        Ac = amg.drop_small((P.T @ A @ P).tocsr())
        assert amg.drop_small(P).nnz == P.nnz == (abs(A) @ amg.prolongator(agg, P.shape[1])).nnz
        assert Ac.nnz == structural.nnz


def test_coarse_sweeps_closed_form():
    """s l1-Jacobi sweeps from zero give x = (I - (I - M^{-1} A)^s) A^{-1} b."""
    M = W.fv_diffusion(np.exp(W.gaussian_random_field((6, 6, 6), 2.0, 5)))
    A = M.to_scipy()
    H = amg.build_hierarchy(A, M.grid, coarse_sweeps=30)
    assert H.L == 0 and H.chol == []
    b = W.rhs_uniform(A.shape[0], 3)
    Ad = A.toarray()
    G = np.eye(A.shape[0]) - np.diag(S.l1_diagonal(A)) @ Ad
    x = (np.eye(A.shape[0]) - np.linalg.matrix_power(G, 30)) @ np.linalg.solve(Ad, b)
    assert np.allclose(amg.coarse_solve(H, b), x, rtol=1e-11, atol=1e-13 * np.abs(x).max())


@pytest.mark.parametrize("opts", [dict(smoothed=True), dict(smoothed=True, agg_edge=3, coarse_sweeps=30),
                                  dict(agg_edge=3)])
@pytest.mark.parametrize("kind", [S.L1JAC, S.OPTCHEB4, S.OPTCHEB1])
def test_vcycle_symmetric_and_spectrum(opts, kind):
    M = W.fv_diffusion(np.exp(W.gaussian_random_field((9, 9, 9), 3.0, 2)))
    A = M.to_scipy()
    H = amg.build_hierarchy(A, M.grid, max_coarse=30, **opts)
    assert H.L >= 1
    n = A.shape[0]
    I = np.eye(n)
    B = np.column_stack([amg.vcycle(H, I[:, i], kind, 3) for i in range(n)])
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    lam, V = np.linalg.eigh(A.toarray())
    Ah = V @ np.diag(np.sqrt(lam)) @ V.T
    mu = np.linalg.eigvalsh(Ah @ B @ Ah)
    assert mu.min() > 0 and mu.max() <= 1.0 + 1e-12


def test_smoothed_aggregation_reduces_iterations():
    """The smoothed prolongator is a better coarse space than the plain one (fewer PCG steps)."""
    A, b, _ = W.config_problem(2, size=24)
    As = A.to_scipy()
    plain, _ = amg.amg_pcg(As, b, A.grid, S.OPTCHEB4, 2, max_coarse=100)
    smooth, _ = amg.amg_pcg(As, b, A.grid, S.OPTCHEB4, 2, max_coarse=100, smoothed=True)
    assert smooth.converged and smooth.iters < plain.iters
