"""Pins of the oracle's smoother recurrences.

Each recurrence (Section 2: eqs. polsmoother, polsmootheropt, polsmootheropt1kind,
Algorithm 1, and plain l1-Jacobi) is checked against the error polynomial it
must realise, evaluated from closed forms on the eigenpairs of M^{-1}A:
  * brute-force dense matrix polynomials on n <= 64;
  * the sine eigenvectors of the 2D 5-point Laplacian (analytic eigenpairs,
    uniform M = 8 I) over 10 consecutive applications, 64x64 grid;
  * the generalized eigenpairs of (A, M) with the true l1 diagonal, n = 4096.
Plus the p(0) = 1 fixed point, the k = 1 special cases and the smoothing
property equivalent to the definition of gamma in Prop. 1.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import polynomials as P
from oracle import smoothers as S

KINDS = [S.L1JAC, S.CHEB4, S.OPTCHEB4, S.OPTCHEB1]


def _params(kind, k):
    beta = P.optimal_beta(k)[0] if kind == S.OPTCHEB4 else None
    a = P.a_star(k) if kind == S.OPTCHEB1 else None
    return beta, a


def _dense_poly(A, Minv, p):
    """p(M^{-1}A) from the eigendecomposition of M^{-1/2} A M^{-1/2}."""
    Ad = A.toarray() if sp.issparse(A) else A
    s = np.sqrt(Minv)
    lam, V = np.linalg.eigh(s[:, None] * Ad * s[None, :])
    return (s[:, None] * V) @ np.diag(p(lam)) @ (V.T / s[None, :])


def test_l1_diagonal_brute_force():
    A = W.fv_diffusion(np.exp(W.gaussian_random_field((3, 4, 5), 2.0, 7))).to_scipy().toarray()
    M = np.array([A[i, i] + sum(abs(A[i, j]) for j in range(A.shape[0]) if j != i) for i in range(A.shape[0])])
    assert np.allclose(S.l1_diagonal(sp.csr_matrix(A)), 1.0 / M, rtol=1e-15, atol=0)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("prob", ["lap2d", "fv3d"])
def test_recurrence_equals_dense_polynomial(kind, k, prob):
    if prob == "lap2d":
        A = W.poisson2d_5pt(8, 8).to_scipy()
    else:
        A = W.fv_diffusion(np.exp(1.5 * W.gaussian_random_field((4, 4, 4), 2.0, 11))).to_scipy()
    n = A.shape[0]
    Minv = S.l1_diagonal(A)
    rng = np.random.default_rng(5)
    b = rng.uniform(-1, 1, n)
    x0 = rng.uniform(-1, 1, n)
    beta, a = _params(kind, k)
    G = _dense_poly(A, Minv, S.error_polynomial(kind, k, beta, a))
    xs = np.linalg.solve(A.toarray(), b)
    for start in (None, x0):
        e0 = -xs if start is None else start - xs
        x = S.smooth(A, Minv, b, start, kind, k, beta, a)
        expect = xs + G @ e0
        assert np.linalg.norm(x - expect) <= 1e-12 * np.linalg.norm(expect)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [1, 3, 6])
def test_sine_closed_form_2d_uniform_M(kind, k):
    """x_t = sum_v (1 - p(lambda_v/8)^t) (v.b)/(lambda_v v.v) v after t applications from 0, M = 8I."""
    m = 64
    A = W.poisson2d_5pt(m, m).to_scipy()
    b = W.rhs_uniform(m * m, W.SEED_RHS + 1)
    Minv = np.full(m * m, 1.0 / 8.0)
    beta, a = _params(kind, k)
    p = S.error_polynomial(kind, k, beta, a)
    h = 1.0 / (m + 1)
    idx = np.arange(1, m + 1)
    Sx = np.sin(np.pi * h * np.outer(idx, idx))  # Sx[p-1, i-1] = sin(p pi i h)
    lam = 4 - 2 * np.cos(np.pi * h * idx)[:, None] - 2 * np.cos(np.pi * h * idx)[None, :]
    B = b.reshape(m, m)  # B[j, i]
    coef = Sx @ B.T @ Sx.T  # coef[p, q] = sum_ij sin(p pi i h) sin(q pi j h) b_ij
    vv = (m + 1) / 2.0
    x = None
    for t in range(1, 11):
        x = S.smooth(A, Minv, b, x, kind, k, beta, a)
        fac = (1 - p(lam / 8.0) ** t) / lam * coef / (vv * vv)
        xt = (Sx.T @ fac @ Sx).T.ravel()  # back to (j, i) lexicographic order
        assert np.linalg.norm(x - xt) <= 1e-12 * np.linalg.norm(xt)


@pytest.mark.parametrize("kind", KINDS)
def test_eigh_closed_form_true_l1(kind):
    """C1 workload (64x64, true l1 M): 10 applications vs the generalized eigenpairs of (A, M)."""
    k = 4
    A, b, _ = W.config_problem(1)
    As = A.to_scipy()
    Minv = S.l1_diagonal(As)
    beta, a = _params(kind, k)
    p = S.error_polynomial(kind, k, beta, a)
    lam, V = sla.eigh(As.toarray(), np.diag(1.0 / Minv))  # A v = lam M v, V^T M V = I
    assert lam.min() > 0 and lam.max() <= 1.0 + 1e-12
    mu = lam / 1.0
    c = V.T @ b  # A^{-1} b = V diag(1/lam) V^T b  (M-orthonormal V)
    x = None
    for t in range(1, 11):
        x = S.smooth(As, Minv, b, x, kind, k, beta, a)
        xt = V @ ((1 - p(mu) ** t) / lam * c)
        assert np.linalg.norm(x - xt) <= 1e-11 * np.linalg.norm(xt)


def test_k1_special_cases():
    A = W.poisson3d_7pt(6).to_scipy()
    Minv = S.l1_diagonal(A)
    b = W.rhs_uniform(A.shape[0], 3)
    x4 = S.smooth(A, Minv, b, None, S.CHEB4, 1)
    assert np.allclose(x4, 4.0 / 3.0 * Minv * b, rtol=1e-15, atol=0)
    xo = S.smooth(A, Minv, b, None, S.OPTCHEB4, 1, P.optimal_beta(1)[0])
    x1 = S.smooth(A, Minv, b, None, S.OPTCHEB1, 1, None, P.a_star(1))
    assert np.allclose(xo, 1.5 * Minv * b, rtol=1e-15, atol=0)
    assert np.allclose(x1, 1.5 * Minv * b, rtol=1e-15, atol=0)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [1, 2, 5])
def test_exact_solution_is_fixed(kind, k):
    A = W.poisson3d_7pt(5).to_scipy()
    Minv = S.l1_diagonal(A)
    xs = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    b = A @ xs
    beta, a = _params(kind, k)
    x = S.smooth(A, Minv, b, xs, kind, k, beta, a)
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)


@pytest.mark.parametrize("kind", [S.CHEB4, S.OPTCHEB4, S.OPTCHEB1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_smoothing_property(kind, k, paper_constants):
    """||G e||_A^2 + gamma^{-1} ||A G e||_{M^{-1}}^2 <= ||e||_A^2 with the printed gamma (Prop. 1)."""
    g = {S.CHEB4: paper_constants["gamma_cheb4"], S.OPTCHEB4: paper_constants["gamma_optcheb4"],
         S.OPTCHEB1: paper_constants["lambda_cheb1"]}[kind][k - 1]
    A = W.fv_diffusion(np.exp(W.gaussian_random_field((8, 8, 8), 3.0, 4))).to_scipy()
    Minv = S.l1_diagonal(A)
    beta, a = _params(kind, k)
    zero = np.zeros(A.shape[0])
    rng = np.random.default_rng(9)
    worst = 0.0
    for _ in range(20):
        e = rng.standard_normal(A.shape[0])
        Ge = S.smooth(A, Minv, zero, e, kind, k, beta, a)  # b = 0: x_out = G e
        AGe = A @ Ge
        lhs = Ge @ AGe + (AGe @ (Minv * AGe)) / g
        worst = max(worst, lhs / (e @ (A @ e)))
    assert worst <= 1.0 + 1e-12
