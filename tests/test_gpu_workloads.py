"""The smoothers on the paper's other two test settings, GPU vs the CPU oracle through the C ABI.

* Polynomial preconditioning alone (the remark after Fig. boundcomparison,
  Fig. better-than-optimal): CG preconditioned by the degree-k smoother on the
  dense A = Q D Q^T, b = A 1, rtol 1e-5 (pcg_solve_smoother).
* Anisotropy 2D (Section 4): Q1 elements, eps = 100, theta = pi/6, Dirichlet on
  y = -1 only, AMG-PCG with 2x2 box aggregates (pcg_solve).

Bar: smoother applications within 1e-12 of the oracle; iteration counts equal
to the oracle's where its count is stable under a 1-ulp change of b (stored
with the counts); where rounding alone moves the oracle's count (the 'gap'
spectrum, eigenvalues from 1e-8 to 10), the GPU count must fall within that
spread widened by 25%, and the solve must reach the tolerance.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import KINDS, dev, hierarchy, host, nan_vec, oracle_params, relerr, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402
from oracle import amg as OA  # noqa: E402
from oracle import smoothers as S  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


def _qdq_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "qdq_pcg_iterations.txt")):
        if line.strip() and not line.startswith("#"):
            sp, N, kind, k, it, rel, lo, hi = line.split()
            rows.append((sp, int(N), int(kind), int(k), int(it), float(rel), int(lo), int(hi)))
    return rows


def _aniso_rows(size):
    rows = []
    for line in open(os.path.join(GOLDEN, f"aniso_pcg_iterations_{size}.txt")):
        if line.strip() and not line.startswith("#"):
            kind, k, it, rel = line.split()
            rows.append((int(kind), int(k), int(it), float(rel)))
    return rows


@pytest.mark.parametrize("spectrum", ["equispaced", "gap"])
def test_smoother_dense_qdq(amg, spectrum):
    """Smoother applications on a dense 256 x 256 operator (256-wide ELL rows), every kind, k = 1..8."""
    torch = torch_cuda()
    A, b, _ = W.qdq_dense(256, spectrum)
    As = A.to_scipy()
    Minv = S.l1_diagonal(As)
    r = np.random.default_rng(5).uniform(-1, 1, A.n)
    with hierarchy(A, max_coarse=4096) as h:
        assert amg.amg_num_levels(h) == 1
        for kind in KINDS:
            for k in range(1, 9):
                x = nan_vec(A.n)
                amg.smoother_apply(h, 0, kind, k, dev(r), x, True)
                torch.cuda.synchronize()
                beta, a = oracle_params(kind, k)
                xo = S.smooth(As, Minv, r, None, kind, k, beta, a)
                assert relerr(host(x), xo) <= 1e-12, (kind, k)


def test_poly_pcg_qdq_matches_oracle(amg):
    """Every (spectrum, N, kind, degree) of the stored table; all mismatches are reported together."""
    torch = torch_cuda()
    rows = _qdq_rows()
    assert len(rows) == 3 * 2 * 4 * 8
    cache = {}
    bad = []
    nexact = 0
    for sp, N, kind, k, it_o, rel_o, lo, hi in rows:
        if (sp, N) not in cache:
            cache.clear()
            cache[(sp, N)] = W.qdq_dense(N, sp)
        A, b, _ = cache[(sp, N)]
        with hierarchy(A, max_coarse=4096) as h:
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve_smoother(h, kind, k, dev(b), x, True, 1e-5, 5000)
            torch.cuda.synchronize()
        true_rel = np.linalg.norm(b - A.to_scipy() @ host(x)) / np.linalg.norm(b)
        case = (sp, N, kind, k, it, it_o, lo, hi, rel, rel_o)
        if rc != amg.AMG_OK or rel > 1e-5 or true_rel > 1.1e-5:
            bad.append(("not converged",) + case)
        elif lo == hi and it == it_o:
            nexact += 1
        elif not (0.75 * lo <= it <= 1.25 * hi):
            bad.append(("count",) + case)
        elif lo == hi and not (sp == "gap" and N == 256):
            # a count stable under 1-ulp changes of b must be reproduced, except on the
            # ill-conditioned gap spectrum at N = 256 (condition number 1e9)
            bad.append(("stable count differs",) + case)
    for row in bad:
        print(row)
    assert not bad
    assert nexact >= 150
def test_poly_pcg_history_matches_oracle(amg):
    """Residual histories of the smoother-preconditioned CG on the equispaced spectrum."""
    torch = torch_cuda()
    A, b, _ = W.qdq_dense(256, "equispaced")
    Ad = A.to_scipy().toarray()
    Minv = S.l1_diagonal(A.to_scipy())
    with hierarchy(A, max_coarse=4096) as h:
        for kind in KINDS:
            for k in (1, 3, 6):
                x = nan_vec(A.n)
                rc, it, rel, hist = amg.pcg_solve_smoother(h, kind, k, dev(b), x, True, 1e-5, 5000, False, True)
                torch.cuda.synchronize()
                beta, a = oracle_params(kind, k)
                ro = OA.pcg(Ad, b, lambda r: S.smooth(Ad, Minv, r, None, kind, k, beta, a), 1e-5, 5000)
                assert it == ro.iters
                assert np.allclose(hist, ro.history, rtol=1e-8, atol=0)
                assert relerr(host(x), ro.x) <= 1e-9


def test_poly_pcg_gap_history_matches_oracle(amg):
    """The ill-conditioned gap spectrum at N = 256 (condition number 1e9), where the iteration
    counts themselves depend on rounding: the first 20 residuals of the smoother-preconditioned CG
    match the oracle's to 1e-8 for every kind and degrees 1, 2, 4, 6 and 8.  Over those 20
    iterations the oracle moves by at most 6e-11 when b is perturbed by one ulp per entry; it
    departs from itself by more than 1e-8 only after 30 to 49 iterations."""
    torch = torch_cuda()
    A, b, _ = W.qdq_dense(256, "gap")
    Ad = A.to_scipy().toarray()
    Minv = S.l1_diagonal(A.to_scipy())
    m = 20
    with hierarchy(A, max_coarse=4096) as h:
        for kind in KINDS:
            for k in (1, 2, 4, 6, 8):
                x = nan_vec(A.n)
                rc, it, rel, hist = amg.pcg_solve_smoother(h, kind, k, dev(b), x, True, 1e-5, 5000, False, True)
                torch.cuda.synchronize()
                beta, a = oracle_params(kind, k)
                ro = OA.pcg(Ad, b, lambda r: S.smooth(Ad, Minv, r, None, kind, k, beta, a), 1e-5, 5000)
                assert rc == amg.AMG_OK and it > m and ro.iters > m, (kind, k, it, ro.iters)
                assert np.allclose(hist[:m + 1], ro.history[:m + 1], rtol=1e-8, atol=0), (kind, k)


def test_aniso_hierarchy_and_vcycle(amg):
    """Odd x extent (N + 1 nodes): the last aggregate of every grid line is one node wide."""
    torch = torch_cuda()
    A, _ = W.anisotropy2d_q1(32)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=60)
    assert len(H.levels) >= 3
    r = np.random.default_rng(6).uniform(-1, 1, A.n)
    with hierarchy(A, max_coarse=60) as h:
        assert amg.amg_num_levels(h) == len(H.levels)
        for l, lv in enumerate(H.levels):
            rp, cl, vl, mi = amg.amg_level_export(h, l)
            torch.cuda.synchronize()
            assert np.array_equal(host(rp), lv.A.indptr)
            assert np.array_equal(host(cl), lv.A.indices)
            assert np.allclose(host(vl), lv.A.data, rtol=1e-14, atol=1e-14 * np.abs(lv.A.data).max())
            assert np.allclose(host(mi), lv.Minv, rtol=1e-14, atol=0)
        for kind in KINDS:
            for k in (1, 2, 4):
                z = nan_vec(A.n)
                amg.vcycle_apply(h, kind, k, dev(r), z)
                torch.cuda.synchronize()
                beta, _ = oracle_params(kind, k)
                assert relerr(host(z), OA.vcycle(H, r, kind, k, beta)) <= 1e-12, (kind, k)


def test_aniso_pcg_iterations_256(amg):
    torch = torch_cuda()
    A, b = W.anisotropy2d_q1(256)
    bd = dev(b)
    rows = _aniso_rows(256)
    assert len(rows) == 16
    with hierarchy(A) as h:
        for kind, k, it_o, rel_o in rows:
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve(h, kind, k, bd, x, True, 1e-8, 1000)
            torch.cuda.synchronize()
            assert rc == amg.AMG_OK and it == it_o, (kind, k, it, it_o)
            assert rel == pytest.approx(rel_o, rel=1e-3)
            assert np.linalg.norm(b - A.to_scipy() @ host(x)) <= 1.05e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("n", [96, 164])
def test_q1_stored_zeros_leave_results_unchanged(amg, n):
    """The 27-point Q1 operator with its six zero face entries per row stored, and without them
    (the 21-point pattern a caller gets by eliminating stored zeros): the coarse levels are the
    same matrices, and the smoothers, the V-cycle and PCG return bitwise the same vectors, since
    a zero product leaves each row sum unchanged.  164^3 runs the streaming kernels."""
    torch = torch_cuda()
    A, B = W.q1_27pt(n), W.q1_27pt(n, store_zeros=False)
    assert B.nnz < A.nnz
    b = W.rhs_uniform(A.n, 41)
    x0 = W.rhs_uniform(A.n, 42)
    bd = dev(b)
    out = {}
    for name, M in (("stored", A), ("eliminated", B)):
        res = {}
        with hierarchy(M) as h:
            L = amg.amg_num_levels(h)
            res["levels"] = [amg.amg_level_info(h, l) for l in range(L)]
            res["layout0"] = amg.amg_level_layout(h, 0)
            res["export"] = [tuple(host(t) for t in amg.amg_level_export(h, l)) for l in range(L)]
            for kind in KINDS:
                x = nan_vec(A.n)
                amg.smoother_apply(h, 0, kind, 4, bd, x, True)
                res[("smooth0", kind)] = host(x)
                x = dev(x0)
                amg.smoother_apply(h, 0, kind, 3, bd, x, False)
                res[("smooth", kind)] = host(x)
            for kind in (2, 3):
                z = nan_vec(A.n)
                amg.vcycle_apply(h, kind, 4, bd, z)
                res[("vcycle", kind)] = host(z)
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve(h, 2, 4, bd, x, True, 1e-8, 1000)
            torch.cuda.synchronize()
            assert rc == amg.AMG_OK
            res["pcg"] = (it, rel, host(x))
        out[name] = res
    s, e = out["stored"], out["eliminated"]
    assert [lv[0] for lv in s["levels"]] == [lv[0] for lv in e["levels"]]
    assert s["levels"][0][1] == A.nnz and e["levels"][0][1] == B.nnz
    assert s["levels"][1:] == e["levels"][1:]
    assert e["layout0"][2] and e["layout0"][0] < s["layout0"][0]
    # level 0: same l1 diagonal; coarser levels: the same CSR matrices and diagonals, bitwise
    assert np.array_equal(s["export"][0][3], e["export"][0][3])
    for l in range(1, len(s["levels"])):
        for a_, b_ in zip(s["export"][l], e["export"][l]):
            assert np.array_equal(a_, b_), l
    for key in s:
        if isinstance(key, tuple):
            assert np.array_equal(s[key], e[key]), key
    assert s["pcg"][0] == e["pcg"][0] and s["pcg"][1] == e["pcg"][1]
    assert np.array_equal(s["pcg"][2], e["pcg"][2])
    print(f"Q1 {n}^3: {A.nnz} vs {B.nnz} stored entries, {s['pcg'][0]} iterations either way", flush=True)
