"""GPU vs oracle for the preconditioner ingredients of the paper's own runs (Section 4): the
smoothed prolongator P = (I - omega D^{-1} A) P_hat, box aggregates of edge 3, and the
coarsest solve by l1-Jacobi sweeps, with flexible CG.

Bar (FP64): Galerkin sparsity bit-exact, values and transfers within 1e-13 of the largest
entry, V-cycles within 1e-12, exact PCG iteration counts, adjoint gradients within 1e-9.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import KINDS, dev, hierarchy, host, nan_vec, oracle_params, relerr, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402
from oracle import adjoint as AD  # noqa: E402
from oracle import amg as OA  # noqa: E402
from oracle import polynomials as P  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


def _fv(shape, sigma, seed):
    return W.fv_diffusion(np.exp(sigma * W.gaussian_random_field(shape, 4.0, seed)))


def _case(name):
    """(matrix, nbatch, max_coarse, hierarchy options)"""
    if name == "poisson_sa2":
        return W.poisson3d_7pt(24), 1, 100, dict(smoothed=True)
    if name == "fv_odd_sa2":
        return _fv((14, 18, 20), 2.0, 3), 1, 60, dict(smoothed=True)
    if name == "q1_sa3":
        return W.q1_27pt(20), 1, 100, dict(smoothed=True, agg_edge=3)
    if name == "aniso_sa2":
        return W.anisotropy2d_q1(40)[0], 1, 60, dict(smoothed=True, coarse_sweeps=30)
    if name == "box3":
        return W.poisson3d_7pt(20, 17, 13), 1, 50, dict(agg_edge=3)
    mats = [_fv((8, 8, 8), s, 10 + p) for p, s in enumerate((0.5, 1.0, 2.0))]
    return W.stack_block_diagonal(mats), 3, 8, dict(smoothed=True)


CASES = ["poisson_sa2", "fv_odd_sa2", "q1_sa3", "aniso_sa2", "box3", "batch_sa2"]


@pytest.mark.parametrize("case", CASES)
def test_hierarchy_and_transfers_match_oracle(amg, case):
    torch = torch_cuda()
    A, nbatch, mc, opts = _case(case)
    H = OA.build_hierarchy(A.to_scipy(), A.grid, nbatch=nbatch, max_coarse=mc, **opts)
    assert len(H.levels) >= 2
    with hierarchy(A, nbatch=nbatch, max_coarse=mc, **opts) as h:
        assert amg.amg_num_levels(h) == len(H.levels)
        for l, lv in enumerate(H.levels):
            rp, cl, vl, mi = amg.amg_level_export(h, l)
            torch.cuda.synchronize()
            assert np.array_equal(host(rp), lv.A.indptr), (case, l)
            assert np.array_equal(host(cl), lv.A.indices), (case, l)
            scale = np.abs(lv.A.data).max()
            assert np.abs(host(vl) - lv.A.data).max() <= 1e-13 * scale, (case, l)
            assert np.allclose(host(mi), lv.Minv, rtol=1e-13, atol=0)
        for l in range(len(H.levels) - 1):
            lv = H.levels[l]
            n, nc = lv.A.shape[0], H.levels[l + 1].A.shape[0]
            rng = np.random.default_rng(7 + l)
            b, x, xc = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, nc)
            bc = nan_vec(nc)
            amg.amg_restrict_residual(h, l, dev(b), dev(x), bc)
            xd = dev(x)
            amg.amg_prolong_add(h, l, dev(xc), xd)
            torch.cuda.synchronize()
            assert relerr(host(bc), lv.P.T @ (b - lv.A @ x)) <= 1e-13, (case, l)
            assert relerr(host(xd), x + lv.P @ xc) <= 1e-14, (case, l)


@pytest.mark.parametrize("case", ["poisson_sa2", "q1_sa3", "aniso_sa2", "box3", "batch_sa2"])
def test_vcycle_matches_oracle(amg, case):
    torch = torch_cuda()
    A, nbatch, mc, opts = _case(case)
    H = OA.build_hierarchy(A.to_scipy(), A.grid, nbatch=nbatch, max_coarse=mc, **opts)
    r = np.random.default_rng(4).uniform(-1, 1, A.n)
    rd = dev(r)
    with hierarchy(A, nbatch=nbatch, max_coarse=mc, **opts) as h:
        for kind in KINDS:
            for k in (1, 2, 4):
                z = nan_vec(A.n)
                amg.vcycle_apply(h, kind, k, rd, z)
                torch.cuda.synchronize()
                beta, _ = oracle_params(kind, k)
                assert relerr(host(z), OA.vcycle(H, r, kind, k, beta)) <= 1e-12, (case, kind, k)
        assert np.array_equal(host(rd), r)


def test_paper_configuration_pcg_iterations(amg):
    """The paper's ingredients on the 3D Poisson problem at 32^3: smoothed prolongator,
    30 l1-Jacobi sweeps on the coarsest level, flexible CG to 1e-8; every kind, k = 1..4."""
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=32)
    As = A.to_scipy()
    opts = dict(smoothed=True, coarse_sweeps=30)
    H = OA.build_hierarchy(As, A.grid, max_coarse=512, **opts)
    with hierarchy(A, max_coarse=512, **opts) as h:
        for kind in KINDS:
            for k in range(1, 5):
                x = nan_vec(A.n)
                rc, it, rel, hist = amg.pcg_solve(h, kind, k, dev(b), x, True, 1e-8, 1000, True, True)
                torch.cuda.synchronize()
                beta, _ = oracle_params(kind, k)
                ro, _ = OA.amg_pcg(As, b, A.grid, kind, k, H=H, beta=beta, flexible=True)
                assert rc == amg.AMG_OK and it == ro.iters, (kind, k, it, ro.iters)
                assert np.allclose(hist, ro.history, rtol=1e-6, atol=0)
                assert relerr(host(x), ro.x) <= 1e-10


def test_fp32_smoothed_hierarchy(amg):
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=32)
    opts = dict(smoothed=True, agg_edge=3, coarse_sweeps=30)
    its = {}
    for prec in (amg.AMG_FP64, amg.AMG_FP32):
        with hierarchy(A, max_coarse=512, precision=prec, **opts) as h:
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve(h, 2, 4, dev(b), x, True, 1e-8, 1000, True)
            torch.cuda.synchronize()
            assert rc == amg.AMG_OK
            assert np.linalg.norm(b - A.to_scipy() @ host(x)) <= 1.05e-8 * np.linalg.norm(b)
            its[prec] = it
    assert abs(its[amg.AMG_FP32] - its[amg.AMG_FP64]) <= 1


def test_adjoint_through_smoothed_transfers(amg):
    """The differentiable V-cycle on stacked problems with smoothed prolongators (one omega per
    problem) and a swept coarsest level, against the oracle's complex-step gradient."""
    torch = torch_cuda()
    k, P_, n = 3, 3, 12
    sig = W.config4_sigmas(P_)
    mats = [_fv((n, n, n), sig[p], 60 + p) for p in range(P_)]
    big = W.stack_block_diagonal(mats)
    opts = dict(smoothed=True, coarse_sweeps=20)
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid, max_coarse=27, **opts) for m in mats]
    b = W.rhs_uniform(big.n, 5)
    m0 = mats[0].n
    bs = [b[p * m0:(p + 1) * m0] for p in range(P_)]
    with hierarchy(big, nbatch=P_, max_coarse=27, **opts) as h:
        L = amg.amg_num_levels(h)
        assert L == len(Hs[0].levels) >= 3
        rng = np.random.default_rng(3)
        tab = np.tile(np.array(P.optimal_beta(k)[0]), (P_, L, 1))
        tab[:, :-1, :] *= 1 + 0.05 * rng.standard_normal((P_, L - 1, k))
        beta = dev(tab.ravel())
        g = torch.empty_like(beta)
        loss, ratios = amg.amg_train_loss_grad(h, k, beta, dev(b), g, P_)
        torch.cuda.synchronize()
        gh = host(g).reshape(P_, L, k)
    betas = [[tab[p, l] for l in range(L - 1)] for p in range(P_)]
    assert loss == pytest.approx(AD.loss(Hs, bs, k, betas), rel=1e-12)
    go = AD.grad_complex_step(Hs, bs, k, betas)
    assert np.allclose(gh[:, :L - 1], go, rtol=1e-9, atol=1e-12 * np.abs(go).max())


def test_option_validation(amg):
    torch_cuda()
    A = W.poisson3d_7pt(8)
    for bad in (dict(agg_edge=1), dict(agg_edge=5), dict(coarse_sweeps=-1), dict(coarse_sweeps=1001)):
        with pytest.raises(amg.AmgError) as e:
            with hierarchy(A, max_coarse=64, **bad):
                pass
        assert e.value.code == amg.AMG_EINVAL


def test_product_capacity_error(amg):
    """A Galerkin product row with more distinct columns than the LDS table holds is reported as
    AMG_ECAPACITY, not computed wrongly: the dense 8000 x 8000 SPD matrix, aggregated in pairs and
    smoothed, gives rows of A P_hat with 4000 distinct columns."""
    torch_cuda()
    n = 8000
    rng = np.random.default_rng(2)
    Bm = rng.uniform(-1, 1, (n, 8))
    dense = Bm @ Bm.T / 8.0 + n * np.eye(n)
    A = W.CSR(n=n, row_ptr=(np.arange(n + 1) * n).astype(np.int32), col=np.tile(np.arange(n, dtype=np.int32), n),
              val=dense.ravel(), grid=(n, 1, 1))
    with pytest.raises(amg.AmgError) as e:
        with hierarchy(A, max_coarse=100, smoothed=True):
            pass
    assert e.value.code == amg.AMG_ECAPACITY
