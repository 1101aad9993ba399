"""Pins of the oracle's hierarchy, V-cycle and PCG.

* Galerkin product A_c = P^T A P (Section 2): for 2x2x2 (2x2) boxes and a
  piecewise-constant P the coarse 7-point (5-point) Laplacian is exactly
  4x (2x) the Laplacian of the half-size grid; other stencils against an
  explicit double loop over aggregates.
* V-cycle (eq. amg): symmetric, spectrum of BA in (0, 1], two-level bound of
  Prop. 1 with the approximation constant C of eq. (approxC) read in the M^{-1} norm.
* PCG: with B = I it is plain CG and reproduces scipy's iteration count; a
  one-level hierarchy solves in one iteration.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import amg
from oracle import polynomials as P
from oracle import smoothers as S

KINDS = [S.L1JAC, S.CHEB4, S.OPTCHEB4, S.OPTCHEB1]


def test_galerkin_7pt_is_scaled_laplacian():
    A = W.poisson3d_7pt(16).to_scipy()
    H = amg.build_hierarchy(A, (16, 16, 16), max_coarse=512)
    assert [l.A.shape[0] for l in H.levels] == [4096, 512]
    D = H.levels[1].A - 4.0 * W.poisson3d_7pt(8).to_scipy()
    assert abs(D).max() == 0.0


def test_galerkin_5pt_is_scaled_laplacian():
    A = W.poisson2d_5pt(32, 32).to_scipy()
    H = amg.build_hierarchy(A, (32, 32, 1), max_coarse=256)
    assert [l.A.shape[0] for l in H.levels] == [1024, 256]
    assert abs(H.levels[1].A - 2.0 * W.poisson2d_5pt(16, 16).to_scipy()).max() == 0.0


@pytest.mark.parametrize("which", ["q1", "fv", "odd"])
def test_galerkin_brute_force(which):
    if which == "q1":
        M = W.q1_27pt(6)
    elif which == "fv":
        M = W.fv_diffusion(np.exp(W.gaussian_random_field((6, 6, 6), 2.0, 3)))
    else:
        M = W.poisson3d_7pt(5, 3, 7)
    A = M.to_scipy()
    H = amg.build_hierarchy(A, M.grid, max_coarse=A.shape[0] - 1)
    Ad = A.toarray()
    agg, gc = amg.box_aggregates(M.grid)
    nc = int(np.prod(gc))
    Ac = np.zeros((nc, nc))
    for i in range(A.shape[0]):
        for j in range(A.shape[0]):
            Ac[agg[i], agg[j]] += Ad[i, j]
    assert np.allclose(H.levels[1].A.toarray(), Ac, rtol=1e-14, atol=1e-14)


def test_box_aggregates_geometry_and_batch():
    agg, gc = amg.box_aggregates((5, 4, 3))
    assert gc == (3, 2, 2)
    # row (i, j, k) -> (i//2, j//2, k//2)
    i, j, k = 4, 3, 2
    assert agg[i + 5 * j + 20 * k] == 2 + 3 * 1 + 6 * 1
    sizes = np.bincount(agg)
    assert sizes.max() == 8 and sizes.min() == 2 and sizes.sum() == 60  # (1 wide in x) x 2 x (1 wide in z)
    aggb, gcb = amg.box_aggregates((4, 4, 4), nbatch=3)
    assert aggb.size == 192 and aggb.max() == 3 * 8 - 1
    assert np.all(aggb[64:128] == aggb[:64] + 8)


def test_batched_hierarchy_is_blockwise():
    mats = [W.fv_diffusion(np.exp(s * W.gaussian_random_field((8, 8, 8), 2.0, 20 + p)))
            for p, s in enumerate((0.5, 1.0, 2.0))]
    big = W.stack_block_diagonal(mats)
    Hb = amg.build_hierarchy(big.to_scipy(), big.grid, nbatch=3, max_coarse=64)
    for p, m in enumerate(mats):
        Hs = amg.build_hierarchy(m.to_scipy(), m.grid, max_coarse=64)
        assert len(Hs.levels) == len(Hb.levels)
        for ls, lb in zip(Hs.levels, Hb.levels):
            n = ls.A.shape[0]
            blk = lb.A[p * n:(p + 1) * n, p * n:(p + 1) * n]
            assert abs(blk - ls.A).max() <= 1e-14 * abs(ls.A).max()


def test_coarse_solve_residual():
    A = W.fv_diffusion(np.exp(2.0 * W.gaussian_random_field((16, 16, 16), 8.0, 1))).to_scipy()
    H = amg.build_hierarchy(A, (16, 16, 16))
    assert H.L == 0
    b = W.rhs_uniform(A.shape[0], 4)
    x = amg.coarse_solve(H, b)
    assert np.linalg.norm(A @ x - b) <= 1e-13 * np.linalg.norm(b)
    # special case: cho_solve is the LAPACK Cholesky solve
    assert np.allclose(x, sla.solve(A.toarray(), b, assume_a="pos"), rtol=1e-12, atol=1e-14)


def _dense_B(H, kind, k):
    n = H.levels[0].A.shape[0]
    I = np.eye(n)
    return np.column_stack([amg.vcycle(H, I[:, i], kind, k) for i in range(n)])


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [1, 3, 6])
def test_vcycle_symmetric_and_spectrum(kind, k):
    M = W.fv_diffusion(np.exp(W.gaussian_random_field((8, 8, 8), 3.0, 2)))
    A = M.to_scipy()
    H = amg.build_hierarchy(A, M.grid, max_coarse=8)
    assert H.L == 2
    B = _dense_B(H, kind, k)
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    # spec(BA) in (0, 1]: eigenvalues of A^{1/2} B A^{1/2}
    Ad = A.toarray()
    lam, V = np.linalg.eigh(Ad)
    Ah = V @ np.diag(np.sqrt(lam)) @ V.T
    mu = np.linalg.eigvalsh(Ah @ B @ Ah)
    assert mu.min() > 0 and mu.max() <= 1.0 + 1e-12


def _gamma(kind, k):
    if kind == S.L1JAC:
        import mpmath as mp
        return P.gamma_of(lambda x: (1 - x) ** k, ngrid=1000)
    if kind == S.CHEB4:
        return P.gamma_cheb4_closed(k)
    if kind == S.OPTCHEB4:
        return P.optimal_beta(k)[1]
    return P.Lambda(k)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_two_level_bound_prop1(kind, k):
    """||E||_A <= C/(C + 1/gamma), E = I - B A, C = lambda_max(M^{1/2}(A^{-1} - P A_c^{-1} P^T) M^{1/2})."""
    A = W.poisson2d_5pt(12, 12).to_scipy()
    H = amg.build_hierarchy(A, (12, 12, 1), max_coarse=36)
    assert H.L == 1
    Ad = A.toarray()
    n = Ad.shape[0]
    B = _dense_B(H, kind, k)
    E = np.eye(n) - B @ Ad
    lam, V = np.linalg.eigh(Ad)
    Ah = V @ np.diag(np.sqrt(lam)) @ V.T
    Aih = V @ np.diag(1 / np.sqrt(lam)) @ V.T
    normE = np.linalg.norm(Ah @ E @ Aih, 2)
    Pm = H.levels[0].P.toarray()
    Ac = Pm.T @ Ad @ Pm
    Q = np.linalg.inv(Ad) - Pm @ np.linalg.solve(Ac, Pm.T)
    m12 = 1.0 / np.sqrt(H.levels[0].Minv)
    C = np.linalg.eigvalsh(m12[:, None] * Q * m12[None, :]).max()
    g = _gamma(kind, k)
    assert normE <= C / (C + 1.0 / g) + 1e-12


@pytest.mark.parametrize("kind", [S.CHEB4])
def test_bound_monotone_in_degree_for_4th_kind(kind):
    A = W.poisson2d_5pt(12, 12).to_scipy()
    H = amg.build_hierarchy(A, (12, 12, 1), max_coarse=36)
    Ad = A.toarray()
    lam, V = np.linalg.eigh(Ad)
    Ah = V @ np.diag(np.sqrt(lam)) @ V.T
    Aih = V @ np.diag(1 / np.sqrt(lam)) @ V.T
    norms = []
    for k in range(1, 7):
        E = np.eye(Ad.shape[0]) - _dense_B(H, kind, k) @ Ad
        norms.append(np.linalg.norm(Ah @ E @ Aih, 2))
    assert all(b < a for a, b in zip(norms, norms[1:]))


def test_pcg_identity_is_cg():
    A = W.poisson3d_7pt(12).to_scipy()
    b = W.rhs_uniform(A.shape[0], 8)
    res = amg.pcg(A, b, lambda r: r.copy(), rtol=1e-8, maxit=500)
    count = [0]
    def cb(xk):
        count[0] += 1
    x, info = spla.cg(A, b, rtol=1e-8, atol=0.0, maxiter=500, callback=cb)
    assert info == 0 and res.converged
    assert res.iters == count[0]
    assert np.allclose(res.x, x, rtol=1e-10, atol=1e-12)
    assert np.linalg.norm(b - A @ res.x) <= 1.01e-8 * np.linalg.norm(b)


def test_one_level_pcg_converges_in_one_iteration():
    A, b, _ = W.config_problem(1)
    res, H = amg.amg_pcg(A.to_scipy(), b, A.grid, S.OPTCHEB4, 4)
    assert H.L == 0 and res.iters == 1 and res.relres < 1e-12


def test_zero_rhs():
    A = W.poisson3d_7pt(6).to_scipy()
    res = amg.pcg(A, np.zeros(A.shape[0]), lambda r: r)
    assert res.iters == 0 and np.all(res.x == 0)


@pytest.mark.parametrize("kind", KINDS)
def test_amg_pcg_converges_and_true_residual(kind):
    A, b, _ = W.config_problem(2, size=24)
    res, H = amg.amg_pcg(A.to_scipy(), b, A.grid, kind, 3, max_coarse=512)
    assert res.converged and H.L == 2  # 24^3 -> 12^3 -> 6^3
    assert np.linalg.norm(b - A.to_scipy() @ res.x) <= 2e-8 * np.linalg.norm(b)
    # iteration counts drop (weakly) with degree
    res6, _ = amg.amg_pcg(A.to_scipy(), b, A.grid, kind, 6, max_coarse=512, H=H)
    assert res6.iters <= res.iters


def test_flexible_cg_reduces_to_cg_and_to_pcg():
    """The flexible (Polak-Ribiere) beta equals the standard one whenever the preconditioner is
    fixed, because consecutive residuals are then B-orthogonal: with B = I it is scipy's CG, and
    with the fixed V-cycle it takes the standard PCG's iterations to the same solution."""
    A = W.poisson3d_7pt(12).to_scipy()
    b = W.rhs_uniform(A.shape[0], 8)
    res = amg.pcg(A, b, lambda r: r.copy(), rtol=1e-8, maxit=500, flexible=True)
    count = [0]

    def cb(xk):
        count[0] += 1
    x, info = spla.cg(A, b, rtol=1e-8, atol=0.0, maxiter=500, callback=cb)
    assert info == 0 and res.converged and res.iters == count[0]
    assert np.allclose(res.x, x, rtol=1e-9, atol=1e-11)
    A2, b2, _ = W.config_problem(2, size=20)
    A2 = A2.to_scipy()
    H = amg.build_hierarchy(A2, (20, 20, 20), max_coarse=200)
    std, _ = amg.amg_pcg(A2, b2, (20, 20, 20), S.OPTCHEB4, 3, H=H)
    flx, _ = amg.amg_pcg(A2, b2, (20, 20, 20), S.OPTCHEB4, 3, H=H, flexible=True)
    assert std.iters == flx.iters
    assert np.linalg.norm(flx.x - std.x) <= 1e-9 * np.linalg.norm(std.x)


@pytest.mark.parametrize("seed", range(3))
def test_flexible_cg_survives_a_varying_preconditioner(seed):
    """A preconditioner that changes at every application (a random positive rescaling of the
    Jacobi diagonal) breaks the standard beta, which assumes a fixed one: it does not reach 1e-8
    in 2000 iterations.  The flexible beta keeps consecutive directions A-orthogonal for any
    preconditioner and converges."""
    A = W.poisson3d_7pt(16).to_scipy()
    b = W.rhs_uniform(A.shape[0], 3)
    Minv = 1.0 / A.diagonal()
    out = {}
    for flexible in (False, True):
        rng = np.random.default_rng(seed)
        res = amg.pcg(A, b, lambda r: Minv * rng.uniform(0.3, 1.7, r.size) * r, rtol=1e-8, maxit=2000,
                      flexible=flexible)
        out[flexible] = res
    assert not out[False].converged
    assert out[True].converged and out[True].iters < 400
    assert np.linalg.norm(b - A @ out[True].x) <= 1.01e-8 * np.linalg.norm(b)
