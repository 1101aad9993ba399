"""Pins of the oracle's derivatives and of its network.

* d <c, B(beta) r> / d beta_{l,j}: as a function of one weight the V-cycle
  output is a polynomial of degree <= 2 (the weight enters one pre- and one
  post-smoother on its level), so a central difference with a large step is
  exact: the complex-step derivative must equal it to rounding.
* The two-cycle residual-ratio loss: complex step vs central differences.
* The MLP: backward vs torch-CPU float64 autograd and finite differences;
  Adam vs torch.optim.Adam.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as AD
from oracle import amg
from oracle import mlp as M
from oracle import polynomials as P


def _problems(n=8, P_=2):
    Hs, bs = [], []
    for p in range(P_):
        A = W.fv_diffusion(np.exp((0.5, 1.0, 2.0)[p % 3] * W.gaussian_random_field((n, n, n), 3.0, 40 + p)))
        Hs.append(amg.build_hierarchy(A.to_scipy(), A.grid, max_coarse=8))
        bs.append(W.rhs_uniform(A.n, 50 + p))
    return Hs, bs


def _betas(k, nl, P_, seed=0):
    rng = np.random.default_rng(seed)
    base = np.array(P.optimal_beta(k)[0])
    return [[base * (1 + 0.05 * rng.standard_normal(k)) for _ in range(nl)] for _ in range(P_)]


@pytest.mark.parametrize("k", [2, 3])
def test_complex_step_equals_exact_quadratic_difference(k):
    Hs, _ = _problems(8, 1)
    H = Hs[0]
    nl = len(H.levels) - 1
    assert nl == 2
    betas = _betas(k, nl, 1)[0]
    rng = np.random.default_rng(3)
    r = rng.uniform(-1, 1, H.levels[0].A.shape[0])
    c = rng.uniform(-1, 1, r.size)
    g = AD.linear_functional_grad(H, r, c, k, betas)
    step = 0.25
    for l in range(nl):
        for j in range(k):
            bp = [v.copy() for v in betas]
            bm = [v.copy() for v in betas]
            bp[l][j] += step
            bm[l][j] -= step
            fd = (c @ AD.vcycle_beta(H, r, k, bp) - c @ AD.vcycle_beta(H, r, k, bm)) / (2 * step)
            assert g[l, j] == pytest.approx(fd, rel=1e-9, abs=1e-12)


def test_loss_gradient_complex_step_vs_central_fd():
    k = 3
    Hs, bs = _problems(8, 2)
    betas = _betas(k, 2, 2, seed=1)
    gc = AD.grad_complex_step(Hs, bs, k, betas)
    gf = AD.grad_central_fd(Hs, bs, k, betas)
    assert np.allclose(gc, gf, rtol=1e-6, atol=1e-9)
    assert np.abs(gc).max() > 1e-4


def test_loss_matches_direct_stationary_iteration():
    """loss = ||b - A x_2|| / ||b|| with x_{m+1} = x_m + B(b - A x_m), x_0 = 0."""
    k = 4
    Hs, bs = _problems(8, 1)
    H, b = Hs[0], bs[0]
    betas = _betas(k, 2, 1, seed=2)[0]
    A = H.levels[0].A
    x = np.zeros_like(b)
    for _ in range(2):
        x = x + AD.vcycle_beta(H, b - A @ x, k, betas)
    assert AD.two_cycle_ratio(H, b, k, betas) == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b),
                                                                 rel=1e-12)


def test_mlp_against_torch_autograd_and_fd():
    torch = pytest.importorskip("torch")
    theta = W.mlp_init(W.SEED_MLP)
    assert theta.size == M.NPARAM == 5126
    rng = np.random.default_rng(1)
    X = rng.standard_normal((12, M.NI))
    dY = rng.standard_normal((12, M.NO))
    y, cache = M.forward(theta, X)
    g = M.backward(theta, cache, dY)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    p, o = {}, 0
    for name, shp in M.SIZES:
        m = int(np.prod(shp))
        p[name] = th[o:o + m].reshape(shp)
        o += m
    Xt = torch.tensor(X)
    yt = M.OUT_SCALE * (torch.tanh(torch.tanh(Xt @ p["W1"].T + p["b1"]) @ p["W2"].T + p["b2"]) @ p["W3"].T + p["b3"])
    assert np.allclose(yt.detach().numpy(), y, rtol=1e-13, atol=1e-15)
    (yt * torch.tensor(dY)).sum().backward()
    assert np.allclose(th.grad.numpy(), g, rtol=1e-12, atol=1e-14)
    # finite differences on a few coordinates
    for idx in (0, 100, 700, 4700, 5000, 5125):
        e = np.zeros_like(theta)
        e[idx] = 1e-6
        fd = (np.sum(dY * M.forward(theta + e, X)[0]) - np.sum(dY * M.forward(theta - e, X)[0])) / 2e-6
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    t = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 4):
        g = rng.standard_normal(50)
        theta, m, v = M.adam_step(theta, g, m, v, step, lr=1e-2)
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(t.detach().numpy(), theta, rtol=1e-12, atol=1e-14)
