"""GPU vs oracle for the compatible weighted-matching aggregation (Section 4, "Compatible Matching"):
aggregates of up to eight rows from three matching steps, plain or smoothed prolongator.

Bar: the matching itself is integer data, so the level sizes and the Galerkin sparsity must be
bit-exact; values and transfers within 1e-13 of the largest entry; V-cycles within 1e-12; exact
PCG iteration counts.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import KINDS, dev, hierarchy, host, nan_vec, oracle_aggregates, oracle_params, relerr, torch_cuda  # noqa: E402,E501

import workloads as W  # noqa: E402
from oracle import amg as OA  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


def _fv(shape, sigma, seed):
    return W.fv_diffusion(np.exp(sigma * W.gaussian_random_field(shape, 4.0, seed)))


def _case(name):
    if name == "poisson":
        return W.poisson3d_7pt(20), 40
    if name == "fv_odd":
        return _fv((14, 18, 20), 2.0, 3), 40
    if name == "q1":
        return W.q1_27pt(12), 30
    return W.anisotropy2d_q1(40)[0], 30


@pytest.mark.parametrize("smoothed", [False, True])
@pytest.mark.parametrize("case", ["poisson", "fv_odd", "q1", "aniso"])
def test_matching_hierarchy_matches_oracle(amg, case, smoothed):
    torch = torch_cuda()
    A, mc = _case(case)
    opts = dict(aggregation=amg.AMG_AGG_MATCHING, smoothed=smoothed)
    H = OA.build_hierarchy(A.to_scipy(), A.grid, max_coarse=mc, aggregation="matching", smoothed=smoothed)
    assert len(H.levels) >= 3
    with hierarchy(A, max_coarse=mc, **opts) as h:
        sizes = [amg.amg_level_info(h, l)[0] for l in range(amg.amg_num_levels(h))]
        assert sizes == [lv.A.shape[0] for lv in H.levels], (case, sizes)
        for l, oagg in enumerate(oracle_aggregates(H, "matching", {})):
            assert np.array_equal(host(amg.amg_level_aggregates(h, l)).astype(np.int64), oagg), (case, l)
        for l, lv in enumerate(H.levels):
            rp, cl, vl, mi = amg.amg_level_export(h, l)
            torch.cuda.synchronize()
            assert np.array_equal(host(rp), lv.A.indptr), (case, l)
            assert np.array_equal(host(cl), lv.A.indices), (case, l)
            assert np.abs(host(vl) - lv.A.data).max() <= 1e-13 * np.abs(lv.A.data).max(), (case, l)
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


@pytest.mark.parametrize("smoothed", [False, True])
def test_matching_vcycle_matches_oracle(amg, smoothed):
    torch = torch_cuda()
    A = _fv((16, 15, 14), 2.0, 8)
    opts = dict(aggregation=amg.AMG_AGG_MATCHING, smoothed=smoothed, coarse_sweeps=30)
    H = OA.build_hierarchy(A.to_scipy(), A.grid, max_coarse=50, aggregation="matching", smoothed=smoothed,
                           coarse_sweeps=30)
    r = np.random.default_rng(4).uniform(-1, 1, A.n)
    with hierarchy(A, max_coarse=50, **opts) as h:
        for kind in KINDS:
            for k in (1, 2, 4):
                z = nan_vec(A.n)
                amg.vcycle_apply(h, kind, k, dev(r), z)
                torch.cuda.synchronize()
                beta, _ = oracle_params(kind, k)
                assert relerr(host(z), OA.vcycle(H, r, kind, k, beta)) <= 1e-12, (kind, k)


def test_matching_paper_configuration_pcg(amg):
    """The paper's Poisson configuration at 32^3: compatible matching (aggregates up to 8), smoothed
    prolongator, 30 coarse l1-Jacobi sweeps, flexible CG to 1e-8; every kind, k = 1..4."""
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=32)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=200, aggregation="matching", smoothed=True, coarse_sweeps=30)
    with hierarchy(A, max_coarse=200, aggregation=amg.AMG_AGG_MATCHING, smoothed=True, coarse_sweeps=30) as h:
        assert [amg.amg_level_info(h, l)[0] for l in range(amg.amg_num_levels(h))] == \
            [lv.A.shape[0] for lv in H.levels]
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


def test_matching_option_validation(amg):
    torch_cuda()
    big = W.stack_block_diagonal([W.poisson3d_7pt(4), W.poisson3d_7pt(4)])
    with pytest.raises(amg.AmgError) as e:
        with hierarchy(big, nbatch=2, max_coarse=8, aggregation=amg.AMG_AGG_MATCHING):
            pass
    assert e.value.code == amg.AMG_EINVAL
    for bad in (dict(aggregation=3), dict(aggregation=amg.AMG_AGG_MATCHING, match_steps=4)):
        with pytest.raises(amg.AmgError) as e:
            with hierarchy(W.poisson3d_7pt(6), max_coarse=8, **bad):
                pass
        assert e.value.code == amg.AMG_EINVAL
