"""GPU tests of the differentiable V-cycle, the network kernels and the learned weights.

Gradients are compared with the oracle's complex-step derivatives (exact to
rounding); the FP64 bar is 1e-9 relative for gradients (they combine many
dot products) and 1e-12 for forward values.  The network kernels run in FP32
and are compared with the FP64 oracle network at FP32 tolerance.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import dev, hierarchy, host, nan_vec, relerr, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402
from oracle import adjoint as AD  # noqa: E402
from oracle import amg as OA  # noqa: E402
from oracle import mlp as OM  # noqa: E402
from oracle import polynomials as P  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


def _stack(n, P_, seed0=60):
    mats = [W.fv_diffusion(np.exp(W.config4_sigmas(P_)[p] * W.gaussian_random_field((n, n, n), 4.0, seed0 + p)))
            for p in range(P_)]
    return mats, W.stack_block_diagonal(mats)


def _beta_table(k, P_, nlevels, seed):
    rng = np.random.default_rng(seed)
    base = np.array(P.optimal_beta(k)[0])
    t = np.tile(base, (P_, nlevels, 1))
    t[:, :-1, :] *= 1 + 0.05 * rng.standard_normal((P_, nlevels - 1, k))
    return t


def test_fwd_ckpt_and_bwd_match_oracle(amg):
    torch = torch_cuda()
    k, P_, n = 3, 3, 12
    mats, big = _stack(n, P_)
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=27) for m in mats]
    rng = np.random.default_rng(1)
    r = rng.uniform(-1, 1, big.n)
    c = rng.uniform(-1, 1, big.n)
    with hierarchy(big, nbatch=P_, max_coarse=27) as h:
        L = amg.amg_num_levels(h)
        assert L == 3 == len(Hs[0].levels)
        tab = _beta_table(k, P_, L, 2)
        beta = dev(tab.ravel())
        ck = torch.empty(amg.amg_ckpt_bytes(h), dtype=torch.uint8, device="cuda")
        z = nan_vec(big.n)
        amg.vcycle_fwd_ckpt(h, k, beta, dev(r), z, ck)
        gr = nan_vec(big.n)
        gb = torch.zeros_like(beta)
        amg.vcycle_bwd(h, k, beta, ck, dev(c), gr, gb)
        torch.cuda.synchronize()
        zh, grh, gbh = host(z), host(gr), host(gb).reshape(P_, L, k)
    m0 = mats[0].n
    for p in range(P_):
        sl = slice(p * m0, (p + 1) * m0)
        betas = [tab[p, l] for l in range(L - 1)]
        assert relerr(zh[sl], AD.vcycle_beta(Hs[p], r[sl], k, betas)) <= 1e-12
        # the V-cycle is symmetric: dL/dr = B(beta) c
        assert relerr(grh[sl], AD.vcycle_beta(Hs[p], c[sl], k, betas)) <= 1e-12
        g = AD.linear_functional_grad(Hs[p], r[sl], c[sl], k, betas)
        assert np.allclose(gbh[p, :L - 1], g, rtol=1e-9, atol=1e-12 * np.abs(g).max())
        assert np.all(gbh[p, L - 1] == 0)


def test_train_loss_grad_matches_oracle(amg):
    torch = torch_cuda()
    k, P_, n = 4, 3, 12
    mats, big = _stack(n, P_, seed0=70)
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=27) for m in mats]
    b = W.rhs_uniform(big.n, 5)
    m0 = mats[0].n
    bs = [b[p * m0:(p + 1) * m0] for p in range(P_)]
    with hierarchy(big, nbatch=P_, max_coarse=27) as h:
        L = amg.amg_num_levels(h)
        tab = _beta_table(k, P_, L, 3)
        beta = dev(tab.ravel())
        g = torch.empty_like(beta)
        loss, ratios = amg.amg_train_loss_grad(h, k, beta, dev(b), g, P_)
        torch.cuda.synchronize()
        gh = host(g).reshape(P_, L, k)
    betas = [[tab[p, l] for l in range(L - 1)] for p in range(P_)]
    for p in range(P_):
        assert ratios[p] == pytest.approx(AD.two_cycle_ratio(Hs[p], bs[p], k, betas[p]), rel=1e-12)
    assert loss == pytest.approx(AD.loss(Hs, bs, k, betas), rel=1e-12)
    go = AD.grad_complex_step(Hs, bs, k, betas)
    assert np.allclose(gh[:, :L - 1], go, rtol=1e-9, atol=1e-12 * np.abs(go).max())


def test_train_loss_grad_degree6_matches_oracle(amg):
    """FP64 at the learned-weights degree (k = 6) on a stack with that workload's three-level
    structure (fine, one box level, dense coarsest): loss and every gradient entry against the
    complex-step oracle."""
    torch = torch_cuda()
    k, P_, n = 6, 3, 16
    mats, big = _stack(n, P_, seed0=75)
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=64) for m in mats]
    assert len(Hs[0].levels) == 3
    b = W.rhs_uniform(big.n, 9)
    m0 = mats[0].n
    bs = [b[p * m0:(p + 1) * m0] for p in range(P_)]
    with hierarchy(big, nbatch=P_, max_coarse=64) as h:
        L = amg.amg_num_levels(h)
        assert L == 3
        tab = _beta_table(k, P_, L, 13)
        beta = dev(tab.ravel())
        g = torch.empty_like(beta)
        loss, ratios = amg.amg_train_loss_grad(h, k, beta, dev(b), g, P_)
        torch.cuda.synchronize()
        gh = host(g).reshape(P_, L, k)
    betas = [[tab[p, l] for l in range(L - 1)] for p in range(P_)]
    for p in range(P_):
        assert ratios[p] == pytest.approx(AD.two_cycle_ratio(Hs[p], bs[p], k, betas[p]), rel=1e-12)
    assert loss == pytest.approx(AD.loss(Hs, bs, k, betas), rel=1e-12)
    go = AD.grad_complex_step(Hs, bs, k, betas)
    assert np.allclose(gh[:, :L - 1], go, rtol=1e-9, atol=1e-12 * np.abs(go).max())
    assert np.all(gh[:, L - 1] == 0)


def test_learned_beta_composition_and_gradient_handover(amg):
    """amg_learned_beta: table + network output on the smoothing rows, the plain table on the
    coarsest row, fallback to the table where the polynomial leaves Pi_k (the oracle's polynomial
    on the same grid decides); amg_learned_beta_grad: dL/dbeta on the kept rows, zero elsewhere."""
    torch = torch_cuda()
    k, P_, n = 6, 4, 12
    mats, big = _stack(n, P_, seed0=140)
    base = np.array(P.optimal_beta(k)[0])
    xs = np.arange(1, 4097) / 4096.0
    with hierarchy(big, nbatch=P_, max_coarse=27) as h:
        L = amg.amg_num_levels(h)
        rows = P_ * (L - 1)
        scales = [1.0, 0.9, 1.05, 1.3, 1.6, 2.0, 0.97, 1.1]
        y = np.zeros((rows, 6), dtype=np.float32)
        rng = np.random.default_rng(21)
        for q in range(rows):
            y[q, :k] = (base * (scales[q % len(scales)] - 1.0) + 1e-3 * rng.standard_normal(k)).astype(np.float32)
        beta, valid = amg.amg_learned_beta(h, k, dev(y), P_)
        plain, pvalid = amg.amg_learned_beta(h, k, None, P_)
        gb = rng.standard_normal((P_, L, k))
        gy = torch.full((rows, 6), float("nan"), dtype=torch.float32, device="cuda")
        amg.amg_learned_beta_grad(h, k, dev(gb.ravel()), valid, gy)
        torch.cuda.synchronize()
        bh, vh, ph, pvh, gyh = host(beta), host(valid), host(plain), host(pvalid), host(gy)
    assert np.all(pvh == 1) and np.all(ph == np.tile(base, (P_, L, 1)))
    expect_valid = []
    for p in range(P_):
        for l in range(L):
            if l == L - 1:
                assert np.all(bh[p, l] == base)
                continue
            q = p * (L - 1) + l
            cand = base + y[q, :k].astype(np.float64)
            ok = int(np.abs(P.p_optcheb4(cand, xs)).max() < 1.0)
            expect_valid.append(ok)
            assert np.all(bh[p, l] == (cand if ok else base)), (p, l)
    assert list(vh) == expect_valid and 0 in expect_valid and 1 in expect_valid
    for q in range(rows):
        p, l = divmod(q, L - 1)
        want = gb[p, l].astype(np.float32) if vh[q] else np.zeros(k, dtype=np.float32)
        assert np.all(gyh[q, :k] == want) and np.all(gyh[q, k:] == 0), q


def test_train_loss_grad_fp32(amg):
    """FP32 hierarchy: loss and gradient within FP32 rounding of the FP64 oracle (parity unpinned for FP32)."""
    torch = torch_cuda()
    k, P_, n = 6, 2, 16
    mats, big = _stack(n, P_, seed0=80)
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=64) for m in mats]
    b = W.rhs_uniform(big.n, 6)
    m0 = mats[0].n
    bs = [b[p * m0:(p + 1) * m0] for p in range(P_)]
    with hierarchy(big, nbatch=P_, max_coarse=64, precision=amg.AMG_FP32) as h:
        L = amg.amg_num_levels(h)
        tab = _beta_table(k, P_, L, 4)
        beta = dev(tab.ravel())
        g = torch.empty_like(beta)
        loss, _ = amg.amg_train_loss_grad(h, k, beta, dev(b), g, P_)
        torch.cuda.synchronize()
        gh = host(g).reshape(P_, L, k)
    betas = [[tab[p, l] for l in range(L - 1)] for p in range(P_)]
    assert loss == pytest.approx(AD.loss(Hs, bs, k, betas), rel=1e-4)
    go = AD.grad_complex_step(Hs, bs, k, betas)
    assert np.abs(gh[:, :L - 1] - go).max() <= 2e-3 * np.abs(go).max()


def test_autograd_function(amg):
    """z = B(beta) r through torch.autograd: beta.grad and r.grad equal the oracle's."""
    torch = torch_cuda()
    k, P_, n = 3, 2, 8
    mats, big = _stack(n, P_, seed0=90)
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=8) for m in mats]
    rng = np.random.default_rng(4)
    r = rng.uniform(-1, 1, big.n)
    c = rng.uniform(-1, 1, big.n)
    with hierarchy(big, nbatch=P_, max_coarse=8) as h:
        L = amg.amg_num_levels(h)
        tab = _beta_table(k, P_, L, 5)
        beta = dev(tab.ravel()).requires_grad_(True)
        rt = dev(r).requires_grad_(True)
        z = amg.VCycleFunction.apply(beta, rt, h, k)
        (z * dev(c)).sum().backward()
        torch.cuda.synchronize()
        gb = host(beta.grad).reshape(P_, L, k)
        grr = host(rt.grad)
    m0 = mats[0].n
    for p in range(P_):
        sl = slice(p * m0, (p + 1) * m0)
        betas = [tab[p, l] for l in range(L - 1)]
        g = AD.linear_functional_grad(Hs[p], r[sl], c[sl], k, betas)
        assert np.allclose(gb[p, :L - 1], g, rtol=1e-9, atol=1e-12 * np.abs(g).max())
        assert relerr(grr[sl], AD.vcycle_beta(Hs[p], c[sl], k, betas)) <= 1e-12


def test_mlp_kernels_match_oracle(amg):
    torch = torch_cuda()
    theta = W.mlp_init(W.SEED_MLP)
    rng = np.random.default_rng(5)
    for Bn in (1, 7, 64):
        X = rng.standard_normal((Bn, 8)).astype(np.float32)
        dY = rng.standard_normal((Bn, 6)).astype(np.float32)
        params = dev(theta.astype(np.float32))
        y = torch.empty((Bn, 6), dtype=torch.float32, device="cuda")
        cache = torch.empty((Bn, 128), dtype=torch.float32, device="cuda")
        amg.mlp_fwd(params, dev(X), y, cache)
        g = torch.empty_like(params)
        work = torch.empty(2 * Bn * 64, dtype=torch.float32, device="cuda")
        amg.mlp_bwd(params, dev(X), cache, dev(dY), g, work)
        torch.cuda.synchronize()
        yo, co = OM.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float64))
        go = OM.backward(theta.astype(np.float32).astype(np.float64), co, dY.astype(np.float64))
        assert np.abs(host(y) - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())
        assert np.abs(host(g) - go).max() <= 1e-4 * np.abs(go).max()
    # Adam: three steps against the oracle update (float32 state)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    th = theta.astype(np.float32).astype(np.float64)
    mo = np.zeros_like(th)
    vo = np.zeros_like(th)
    for step in range(1, 4):
        gg = rng.standard_normal(th.size).astype(np.float32)
        amg.mlp_adam(params, dev(gg), m, v, step, 1e-3)
        th, mo, vo = OM.adam_step(th, gg.astype(np.float64), mo, vo, step, lr=1e-3)
    torch.cuda.synchronize()
    assert np.abs(host(params) - th).max() <= 1e-6


def test_beta_validity_check(amg):
    torch = torch_cuda()
    rows, ks = [], 6
    base = np.array(P.optimal_beta(ks)[0])
    for s in (1.0, 0.9, 1.05, 1.3, 1.6, 2.0):
        rows.append(base * s)
    rows.append(np.array([1.0] * ks))  # plain 4th kind
    tab = np.array(rows)
    valid = host(amg.amg_beta_valid(dev(tab.ravel()), ks, 4096))
    xs = np.arange(1, 4097) / 4096.0
    expect = [int(np.abs(P.p_optcheb4(rw, xs)).max() < 1.0) for rw in tab]
    assert list(valid) == expect
    assert valid[0] == 1 and valid[-1] == 1 and 0 in expect


def test_level_features(amg):
    torch = torch_cuda()
    k, P_, n = 6, 3, 16
    mats, big = _stack(n, P_, seed0=100)
    sig = W.config4_sigmas(P_)
    with hierarchy(big, nbatch=P_, max_coarse=64) as h:
        L = amg.amg_num_levels(h)
        f = host(amg.amg_level_features(h, k, sig)).reshape(P_, L - 1, 8)
    for p, m in enumerate(mats):
        H = OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=64)
        for l in range(L - 1):
            A = H.levels[l].A
            Minv = H.levels[l].Minv
            v = np.ones(A.shape[0])
            for _ in range(19):
                v = Minv * (A @ v)
            w = Minv * (A @ v)
            lam = np.linalg.norm(w) / np.linalg.norm(v)
            d = A.diagonal()
            ratio = np.mean((1.0 / Minv - d) / d)
            expect = [k / 6, l / (L - 1), 1 - lam, A.nnz / A.shape[0] / 27, np.log2(A.shape[0]) / 24, sig[p],
                      H.levels[l + 1].A.shape[0] / A.shape[0], ratio]
            assert np.allclose(f[p, l], expect, rtol=1e-5, atol=1e-6), (p, l, f[p, l], expect)


def test_learned_beta_gains_over_plain(amg):
    """Train the network (FP32, hand-written kernels) on stacked diffusion problems; the learned weights
    must lower the two-cycle residual ratio on the training problems and, by at least 5%, on
    held-out problems of the same family (other random fields and right-hand side)."""
    torch = torch_cuda()
    from paper_2407_09848_amd import learned
    k, P_, n = 6, 6, 24
    mats, big = _stack(n, P_, seed0=200)
    b = W.rhs_uniform(big.n, 7)
    sig = W.config4_sigmas(P_)
    with hierarchy(big, nbatch=P_, max_coarse=512, precision=amg.AMG_FP32) as h:
        res = learned.train(h, dev(b), sig, degree=k, steps=60, lr=3e-3, init_params=W.mlp_init(W.SEED_MLP))
        feats = amg.amg_level_features(h, k, sig)
        beta, _, _ = learned.predict_beta(h, res.params, feats, k, P_)
        train_loss, _ = learned.evaluate(h, beta, dev(b), k, P_)
    gain_train = 1 - train_loss / res.plain_loss
    print(f"training set: plain {res.plain_loss:.6f} learned {train_loss:.6f} gain {100 * gain_train:.2f}%")
    assert train_loss < res.plain_loss
    # held-out problems (other random fields and right-hand side)
    mats2, big2 = _stack(n, P_, seed0=300)
    b2 = W.rhs_uniform(big2.n, 8)
    with hierarchy(big2, nbatch=P_, max_coarse=512, precision=amg.AMG_FP32) as h2:
        feats2 = amg.amg_level_features(h2, k, sig)
        beta2, _, _ = learned.predict_beta(h2, res.params, feats2, k, P_)
        plain = learned.plain_beta(h2, k, P_)
        l_learned, _ = learned.evaluate(h2, beta2, dev(b2), k, P_)
        l_plain, _ = learned.evaluate(h2, plain, dev(b2), k, P_)
    gain = 1 - l_learned / l_plain
    print(f"held out: plain {l_plain:.6f} learned {l_learned:.6f} gain {100 * gain:.2f}%")
    # the network, trained on other random fields, lowers the loss on problems it has not seen
    assert gain >= 0.05
