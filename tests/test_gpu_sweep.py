"""Randomised GPU-vs-oracle sweep over the setup options: problem family and ragged size, box /
matching / VBM aggregates, plain or smoothed prolongator, box edge, matching steps, strength
threshold, Cholesky or swept coarsest level, polynomial kind and degree 1..12.

Each seeded case checks, at the bars of the dedicated tests: the aggregate of every row, the
level sizes and the Galerkin sparsity bit-exact, the coarse values within 1e-13 of the largest
entry, two V-cycles within 1e-12, and the PCG iteration count exactly (a count one apart is accepted only when the oracle's residual
at the stopping test lies within 1e-6 of the tolerance, the borderline reading of the stopping rule),
with the residual history within 1e-6 relative or 1e-12 absolute.
"""
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import dev, hierarchy, host, nan_vec, oracle_aggregates, oracle_params, relerr, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402
from oracle import amg as OA  # noqa: E402

pytestmark = pytest.mark.gpu

# 160 seeded cases by default; AMGP_SWEEP_FIRST / AMGP_SWEEP_CASES select another range of seeds
FIRST = int(os.environ.get("AMGP_SWEEP_FIRST", "0"))
NCASES = int(os.environ.get("AMGP_SWEEP_CASES", "160"))


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


def _graph_spd(n, rng):
    """Weighted graph Laplacian of a random sparse graph plus a positive diagonal (one row per
    vertex, structurally symmetric, sorted columns, diagonal stored)."""
    R = sp.random(n, n, density=min(1.0, 6.0 / n), random_state=int(rng.integers(1 << 30)), format="csr")
    R = abs(R + R.T)
    R.setdiag(0)
    R.eliminate_zeros()
    A = sp.diags(np.asarray(R.sum(axis=1)).ravel() + rng.uniform(0.1, 1.0, n)) - R
    A = sp.csr_matrix(A)
    A.sort_indices()
    return W.CSR(n=n, row_ptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32), val=A.data.copy(),
                 grid=(n, 1, 1))


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    fam = ["p2d", "p3d", "q1", "fv", "aniso", "graph"][seed % 6]
    if fam == "p2d":
        A = W.poisson2d_5pt(int(rng.integers(20, 70)), int(rng.integers(20, 70)))
    elif fam == "p3d":
        A = W.poisson3d_7pt(*[int(v) for v in rng.integers(7, 17, 3)])
    elif fam == "q1":
        A = W.q1_27pt(*[int(v) for v in rng.integers(6, 12, 3)])
    elif fam == "fv":
        shape = tuple(int(v) for v in rng.integers(7, 15, 3))
        A = W.fv_diffusion(np.exp(float(rng.uniform(0.5, 2.0)) * W.gaussian_random_field(shape, 3.0, seed)))
    elif fam == "aniso":
        A = W.anisotropy2d_q1(int(rng.integers(20, 50)))[0]
    else:
        A = _graph_spd(int(rng.integers(300, 2500)), rng)
    aggs = ["matching", "vbm"] if fam == "graph" else ["box", "matching", "vbm"]
    agg = aggs[int(rng.integers(len(aggs)))]
    opts = dict(smoothed=bool(rng.integers(2)), coarse_sweeps=int(rng.choice([0, 0, 7, 30])))
    if agg == "box":
        opts["agg_edge"] = int(rng.integers(2, 5))
    elif agg == "matching":
        opts["match_steps"] = int(rng.integers(1, 4))
    else:
        opts["vbm_theta"] = float(rng.choice([0.0, 0.05, 0.08, 0.12]))
    mc = int(rng.integers(8, 80))
    kinds = rng.integers(0, 4, 3)
    degs = rng.integers(1, 13, 3)
    return fam, A, agg, opts, mc, kinds, degs


def _lib_opts(amg, agg, opts):
    o = dict(opts)
    o["aggregation"] = {"box": amg.AMG_AGG_BOX, "matching": amg.AMG_AGG_MATCHING, "vbm": amg.AMG_AGG_VBM}[agg]
    return o


@pytest.mark.parametrize("seed", range(FIRST, FIRST + NCASES))
def test_sweep_case_matches_oracle(amg, seed):
    torch = torch_cuda()
    fam, A, agg, opts, mc, kinds, degs = _case(seed)
    tag = (seed, fam, A.n, agg, opts, mc)
    print("case", tag, flush=True)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=mc, aggregation=agg, **opts)
    flexible = opts["smoothed"] or opts["coarse_sweeps"] > 0
    with hierarchy(A, max_coarse=mc, **_lib_opts(amg, agg, opts)) as h:
        sizes = [amg.amg_level_info(h, l)[0] for l in range(amg.amg_num_levels(h))]
        assert sizes == [lv.A.shape[0] for lv in H.levels], tag
        for l, oagg in enumerate(oracle_aggregates(H, agg, opts)):
            assert np.array_equal(host(amg.amg_level_aggregates(h, l)).astype(np.int64), oagg), (tag, l)
        for l, lv in enumerate(H.levels):
            rp, cl, vl, _ = amg.amg_level_export(h, l)
            torch.cuda.synchronize()
            assert np.array_equal(host(rp), lv.A.indptr) and np.array_equal(host(cl), lv.A.indices), (tag, l)
            assert np.abs(host(vl) - lv.A.data).max() <= 1e-13 * np.abs(lv.A.data).max(), (tag, l)
        r = np.random.default_rng(seed).uniform(-1, 1, A.n)
        for kind, k in zip(kinds[:2], degs[:2]):
            z = nan_vec(A.n)
            amg.vcycle_apply(h, int(kind), int(k), dev(r), z)
            torch.cuda.synchronize()
            beta, _ = oracle_params(int(kind), int(k))
            assert relerr(host(z), OA.vcycle(H, r, int(kind), int(k), beta)) <= 1e-12, (tag, kind, k)
        kind, k = int(kinds[2]), int(degs[2])
        b = W.rhs_uniform(A.n, seed)
        x = nan_vec(A.n)
        rc, it, rel, hist = amg.pcg_solve(h, kind, k, dev(b), x, True, 1e-8, 1000, flexible, True)
        torch.cuda.synchronize()
        beta, _ = oracle_params(kind, k)
        ro, _ = OA.amg_pcg(As, b, A.grid, kind, k, H=H, beta=beta, flexible=flexible)
        assert rc == amg.AMG_OK, (tag, rc)
        if it != ro.iters:
            lo = min(it, ro.iters)
            assert abs(it - ro.iters) == 1 and abs(ro.history[lo] / 1e-8 - 1.0) <= 1e-6, (tag, kind, k, it, ro.iters)
        else:
            # relative residuals below 1e-12 are rounding noise (a one-level hierarchy solves exactly)
            assert np.allclose(hist, ro.history, rtol=1e-6, atol=1e-12), (tag, kind, k)
            assert relerr(host(x), ro.x) <= 1e-9, (tag, kind, k)
