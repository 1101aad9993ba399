"""GPU path vs the CPU oracle, element by element, through the C ABI.

Bar (FP64): relative error <= 1e-12 per smoother application and per
V-cycle, exact PCG iteration counts; integer/index data (Galerkin sparsity,
aggregates) bit-exact.  Output buffers are NaN-filled before write-only calls
so an unwritten entry fails the comparison.
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

TOL = 1e-12


def _fv(shape, sigma, seed):
    g = W.gaussian_random_field(shape, 4.0, seed)
    return W.fv_diffusion(np.exp(sigma * g))


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


# ---------------------------------------------------------------------------
# smoother (one level), C1 workload: 10 consecutive applications per (kind, k)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", KINDS)
def test_smoother_c1_ten_applications(amg, kind):
    torch = torch_cuda()
    A, b, _ = W.config_problem(1)
    As = A.to_scipy()
    Minv = S.l1_diagonal(As)
    bd = dev(b)
    with hierarchy(A) as h:
        assert amg.amg_num_levels(h) == 1
        for k in range(1, 7):
            beta, a = oracle_params(kind, k)
            x = nan_vec(A.n)
            xo = None
            for t in range(10):
                amg.smoother_apply(h, 0, kind, k, bd, x, x_is_zero=(t == 0))
                xo = S.smooth(As, Minv, b, xo, kind, k, beta, a)
                torch.cuda.synchronize()
                e = relerr(host(x), xo)
                assert e <= TOL, (kind, k, t, e)


@pytest.mark.parametrize("shape", [(13, 11, 9), (64, 3, 5), (7, 1, 1)])
@pytest.mark.parametrize("kind", KINDS)
def test_smoother_ragged_fv(amg, shape, kind):
    """Several 64-row slices and a ragged tail; x0 = 0 and x0 random."""
    torch = torch_cuda()
    A = _fv(shape[::-1], 1.5, 5)
    As = A.to_scipy()
    Minv = S.l1_diagonal(As)
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, A.n)
    x0 = rng.uniform(-1, 1, A.n)
    with hierarchy(A, max_coarse=10**9) as h:
        for k in (1, 2, 3, 6):
            beta, a = oracle_params(kind, k)
            x = nan_vec(A.n)
            amg.smoother_apply(h, 0, kind, k, dev(b), x, x_is_zero=True)
            xd = dev(x0)
            amg.smoother_apply(h, 0, kind, k, dev(b), xd, x_is_zero=False)
            torch.cuda.synchronize()
            assert relerr(host(x), S.smooth(As, Minv, b, None, kind, k, beta, a)) <= TOL
            assert relerr(host(xd), S.smooth(As, Minv, b, x0, kind, k, beta, a)) <= TOL


def test_smoother_does_not_modify_b(amg):
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=16)
    bd = dev(b)
    with hierarchy(A) as h:
        for kind in KINDS:
            x = nan_vec(A.n)
            amg.smoother_apply(h, 0, kind, 5, bd, x, True)
            amg.smoother_apply(h, 0, kind, 5, bd, x, False)
    torch.cuda.synchronize()
    assert np.array_equal(host(bd), b)


# ---------------------------------------------------------------------------
# hierarchy: l1 diagonal, Galerkin operators, SpMV, transfers, coarse solve
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["poisson", "fv_odd", "q1", "q1_11x6x7", "q1_10x7x7", "batch"])
def test_hierarchy_matches_oracle(amg, case):
    """The two Q1 grids of odd extents leave aggregates one cell wide in two directions on level 1,
    coupled only through the stored zero face entries: the coarse patterns hold no such zeros."""
    torch = torch_cuda()
    nbatch = 1
    if case.startswith("q1_"):
        A = W.q1_27pt(*[int(v) for v in case[3:].split("x")])
        mc = 38 if case == "q1_11x6x7" else 14
    elif case == "poisson":
        A = W.poisson3d_7pt(32)
        mc = 4096
    elif case == "fv_odd":
        A = _fv((14, 18, 20), 2.0, 3)
        mc = 60
    elif case == "q1":
        A = W.q1_27pt(20)
        mc = 200
    else:
        A = W.stack_block_diagonal([_fv((8, 8, 8), s, 10 + p) for p, s in enumerate((0.5, 1.0, 2.0))])
        nbatch, mc = 3, 8
    H = OA.build_hierarchy(A.to_scipy(), A.grid, nbatch=nbatch, max_coarse=mc)
    with hierarchy(A, nbatch=nbatch, max_coarse=mc) as h:
        assert amg.amg_num_levels(h) == len(H.levels)
        for l, lv in enumerate(H.levels):
            rp, cl, vl, mi = amg.amg_level_export(h, l)
            torch.cuda.synchronize()
            assert np.array_equal(host(rp), lv.A.indptr)
            assert np.array_equal(host(cl), lv.A.indices)
            assert np.allclose(host(vl), lv.A.data, rtol=1e-14, atol=1e-14 * np.abs(lv.A.data).max())
            assert np.allclose(host(mi), lv.Minv, rtol=1e-14, atol=0)
            # SpMV
            x = np.random.default_rng(l).uniform(-1, 1, lv.A.shape[0])
            y = nan_vec(lv.A.shape[0])
            amg.amg_spmv(h, l, dev(x), y)
            torch.cuda.synchronize()
            assert relerr(host(y), lv.A @ x) <= 1e-14
        # transfers on every level
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
            assert relerr(host(bc), lv.P.T @ (b - lv.A @ x)) <= 1e-14
            assert np.array_equal(host(xd), x + lv.P @ xc)
        # coarse solve
        nL = H.levels[-1].A.shape[0]
        bl = np.random.default_rng(3).uniform(-1, 1, nL)
        xl = nan_vec(nL)
        amg.amg_coarse_solve(h, dev(bl), xl)
        torch.cuda.synchronize()
        assert relerr(host(xl), OA.coarse_solve(H, bl)) <= 1e-12


@pytest.mark.parametrize("n", [1000, 4096, 130])
def test_coarse_solve_padding(amg, n):
    """Dense Cholesky / inverse path with n_L not a multiple of the 64-wide tile."""
    torch = torch_cuda()
    A = W.poisson3d_7pt(10) if n == 1000 else (W.poisson3d_7pt(16) if n == 4096 else _fv((2, 5, 13), 1.0, 1))
    H = OA.build_hierarchy(A.to_scipy(), A.grid)
    assert H.L == 0
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    with hierarchy(A) as h:
        x = nan_vec(A.n)
        amg.amg_coarse_solve(h, dev(b), x)
        torch.cuda.synchronize()
        assert relerr(host(x), OA.coarse_solve(H, b)) <= 1e-12


# ---------------------------------------------------------------------------
# V-cycle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["poisson32", "fv_ragged"])
@pytest.mark.parametrize("kind", KINDS)
def test_vcycle_matches_oracle(amg, case, kind):
    torch = torch_cuda()
    if case == "poisson32":
        A = W.poisson3d_7pt(32)
        mc = 4096
    else:
        A = _fv((14, 18, 20), 2.0, 3)
        mc = 60
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=mc)
    r = np.random.default_rng(4).uniform(-1, 1, A.n)
    rd = dev(r)
    with hierarchy(A, max_coarse=mc) as h:
        for k in range(1, 7):
            z = nan_vec(A.n)
            amg.vcycle_apply(h, kind, k, rd, z)
            torch.cuda.synchronize()
            beta, _ = oracle_params(kind, k)
            zo = OA.vcycle(H, r, kind, k, beta)
            assert relerr(host(z), zo) <= TOL, (kind, k)
        assert np.array_equal(host(rd), r)


def test_vcycle_graph_replays_and_beta_change(amg):
    """The V-cycle is captured once per (kind, degree, buffers) and replayed: every replay, with
    eager work in between, equals the oracle; a new beta drops the captured graph."""
    torch = torch_cuda()
    A = W.poisson3d_7pt(24)
    H = OA.build_hierarchy(A.to_scipy(), A.grid, max_coarse=300)
    r = np.random.default_rng(8).uniform(-1, 1, A.n)
    rd = dev(r)
    beta, _ = oracle_params(2, 3)
    zo = OA.vcycle(H, r, 2, 3, beta)
    with hierarchy(A, max_coarse=300) as h:
        z = nan_vec(A.n)
        for rep in range(4):
            z.fill_(float("nan"))
            amg.vcycle_apply(h, 2, 3, rd, z)
            xs = nan_vec(A.n)
            amg.smoother_apply(h, 0, 1, 2, rd, xs, True)  # eager work between replays
            torch.cuda.synchronize()
            assert relerr(host(z), zo) <= TOL, rep
        nb = [1.1, 0.9, 1.3]
        amg.amg_set_beta(h, 3, -1, nb)
        amg.vcycle_apply(h, 2, 3, rd, z)
        torch.cuda.synchronize()
        assert relerr(host(z), OA.vcycle(H, r, 2, 3, nb)) <= TOL
        amg.amg_set_beta(h, 3, 1, [1.0, 1.0, 1.0])  # level 1 only
        amg.vcycle_apply(h, 2, 3, rd, z)
        torch.cuda.synchronize()
        per_level = [nb, [1.0, 1.0, 1.0]] + [nb] * (len(H.levels) - 2)
        assert relerr(host(z), OA.vcycle(H, r, 2, 3, None, betas_by_level=per_level)) <= TOL
        amg.amg_reset_beta(h)
        amg.vcycle_apply(h, 2, 3, rd, z)
        torch.cuda.synchronize()
        assert relerr(host(z), zo) <= TOL


def test_fp32_hierarchy(amg):
    """FP32 hierarchy inside FP64 CG (parity unpinned: no exact FP32 answer); bounded instead:
    converges to 1e-8 in the FP64 iteration count (+-1), true FP64 residual within 2e-8, and the
    FP32 V-cycle differs from the FP64 oracle V-cycle by no more than FP32 rounding allows."""
    torch = torch_cuda()
    g = W.gaussian_random_field((48, 48, 48), 8.0, W.SEED_GRF)
    A = W.fv_diffusion(np.exp(g))
    b = W.rhs_uniform(A.n, W.SEED_RHS + 3)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=4096)
    ro, _ = OA.amg_pcg(As, b, A.grid, 2, 4, H=H)
    with hierarchy(A, precision=amg.AMG_FP32) as h:
        z = nan_vec(A.n)
        amg.vcycle_apply(h, 2, 4, dev(b), z)
        torch.cuda.synchronize()
        e_v = relerr(host(z), OA.vcycle(H, b, 2, 4))
        assert e_v <= 1e-5
        for flexible in (False, True):
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve(h, 2, 4, dev(b), x, True, 1e-8, 200, flexible)
            torch.cuda.synchronize()
            assert rc == amg.AMG_OK and abs(it - ro.iters) <= 1
            xr = host(x)
            assert np.linalg.norm(b - As @ xr) <= 2e-8 * np.linalg.norm(b)
            assert relerr(xr, ro.x) <= 1e-6


@pytest.mark.parametrize("case", ["q1_20", "fv_ragged"])
def test_fp32_aligned_smoother(amg, case):
    """The FP32 hierarchy's smoother (smoother_apply_f32: float32 matrix, l1 diagonal, vectors and
    accumulation) on offset-aligned fine levels, whose float values sit in quads (27-point slices)
    or pairs (7-point) with the odd steps after them, and fewer offsets in boundary slices: every
    kind at degrees 1..6, from x = 0 and from x != 0, stays within FP32 rounding of the FP64
    oracle smoother (parity unpinned: no exact FP32 answer), and the float64 smoother_apply on the
    same handle runs the float64 copy of the level (oracle bar)."""
    torch = torch_cuda()
    A = W.q1_27pt(20) if case == "q1_20" else _fv((13, 11, 9), 1.0, 6)
    As = A.to_scipy()
    Minv = S.l1_diagonal(As)
    rng = np.random.default_rng(21)
    r = rng.uniform(-1, 1, A.n)
    x0 = rng.uniform(-1, 1, A.n)
    r32, x032 = r.astype(np.float32), x0.astype(np.float32)
    worst = 0.0
    with hierarchy(A, precision=amg.AMG_FP32) as h:
        _, lanes, aligned = amg.amg_level_layout(h, 0)
        assert aligned and lanes == 1
        for kind in KINDS:
            for k in range(1, 7):
                beta, a = oracle_params(kind, k)
                x = torch.full((A.n,), float("nan"), dtype=torch.float32, device="cuda")
                amg.smoother_apply_f32(h, 0, kind, k, dev(r32), x, True)
                xd = dev(x032)
                amg.smoother_apply_f32(h, 0, kind, k, dev(r32), xd, False)
                x64 = nan_vec(A.n)
                amg.smoother_apply(h, 0, kind, k, dev(r), x64, True)
                torch.cuda.synchronize()
                ref0 = S.smooth(As, Minv, r32.astype(np.float64), None, kind, k, beta, a)
                ref1 = S.smooth(As, Minv, r32.astype(np.float64), x032.astype(np.float64), kind, k, beta, a)
                e0 = relerr(host(x).astype(np.float64), ref0)
                e1 = relerr(host(xd).astype(np.float64), ref1)
                worst = max(worst, e0, e1)
                assert e0 <= 5e-6 and e1 <= 5e-6, (case, kind, k, e0, e1)
                assert relerr(host(x64), S.smooth(As, Minv, r, None, kind, k, beta, a)) <= TOL, (case, kind, k)
        with pytest.raises(amg.AmgError):
            amg.smoother_apply_f32(h, 0, 4, 2, dev(r32), dev(x032), False)
    with hierarchy(A) as h64:
        with pytest.raises(amg.AmgError) as e:
            amg.smoother_apply_f32(h64, 0, 2, 2, dev(r32), dev(x032), False)
        assert e.value.code == amg.AMG_EINVAL
    print(f"FP32 smoother on {case}: largest error against the FP64 oracle {worst:.2e}", flush=True)


def test_fp32_smoother_every_level(amg):
    """smoother_apply_f32 on every level of an FP32 box hierarchy of the 27-point problem (the
    offset-aligned fine level, the four-lane packed coarse levels and the coarsest level) against
    the FP64 oracle smoother on the oracle's level operator, within FP32 rounding."""
    torch = torch_cuda()
    A = W.q1_27pt(26, 22, 18)
    H = OA.build_hierarchy(A.to_scipy(), A.grid, max_coarse=60)
    rng = np.random.default_rng(23)
    with hierarchy(A, max_coarse=60, precision=amg.AMG_FP32) as h:
        assert amg.amg_num_levels(h) == len(H.levels) >= 4
        for l, lv in enumerate(H.levels):
            n = lv.A.shape[0]
            b32 = rng.uniform(-1, 1, n).astype(np.float32)
            for kind, k in ((0, 3), (1, 4), (2, 5), (3, 6)):
                beta, a = oracle_params(kind, k)
                x = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
                amg.smoother_apply_f32(h, l, kind, k, dev(b32), x, True)
                torch.cuda.synchronize()
                ref = S.smooth(lv.A, lv.Minv, b32.astype(np.float64), None, kind, k, beta, a)
                e = relerr(host(x).astype(np.float64), ref)
                assert e <= 5e-6, (l, n, kind, k, e)


def test_vcycle_full_size_c2(amg):
    """128^3 7-point Poisson, optimal 4th kind k = 4: the whole V-cycle output vs the oracle."""
    torch = torch_cuda()
    A, b, _ = W.config_problem(2)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid)
    with hierarchy(A) as h:
        for kind in (2, 3):
            z = nan_vec(A.n)
            amg.vcycle_apply(h, kind, 4, dev(b), z)
            torch.cuda.synchronize()
            beta, _ = oracle_params(kind, 4)
            assert relerr(host(z), OA.vcycle(H, b, kind, 4, beta)) <= TOL


# ---------------------------------------------------------------------------
# PCG
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", KINDS)
def test_pcg_iterations_match_oracle_32(amg, kind):
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=32)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid)
    with hierarchy(A) as h:
        for k in range(1, 7):
            x = nan_vec(A.n)
            rc, it, rel, hist = amg.pcg_solve(h, kind, k, dev(b), x, True, 1e-8, 1000, False, True)
            torch.cuda.synchronize()
            beta, _ = oracle_params(kind, k)
            ro, _ = OA.amg_pcg(As, b, A.grid, kind, k, H=H, beta=beta)
            assert rc == amg.AMG_OK and it == ro.iters, (kind, k, it, ro.iters)
            assert np.allclose(hist, ro.history, rtol=1e-6, atol=0)
            assert relerr(host(x), ro.x) <= 1e-10


DEGENERATE = {
    "single_row": ((1, 1, 1), 4096),   # one unknown: the coarsest level is the whole problem
    "tiny_2x3x1": ((2, 3, 1), 4096),   # six rows in one slice
    "line_x": ((5000, 1, 1), 4096),    # a 1D line along x, coarsened in x only
    "line_z": ((1, 1, 5000), 4096),    # the same line along z
    "plane_xz": ((70, 1, 70), 1000),   # a 2D problem in the x-z plane
    "odd_3x5x7": ((3, 5, 7), 8),       # odd extents on every level: 105 -> 24 -> 4 rows
}


@pytest.mark.parametrize("case", sorted(DEGENERATE))
def test_degenerate_shapes_match_oracle(amg, case):
    """Grids with extents of 1, a single unknown, and odd extents down to the coarsest level:
    smoother (from x = 0 and x != 0), V-cycle and PCG against the oracle (exact counts)."""
    torch = torch_cuda()
    grid, mc = DEGENERATE[case]
    A = W.poisson3d_7pt(*grid)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=mc)
    Minv = S.l1_diagonal(As)
    rng = np.random.default_rng(12)
    b = rng.uniform(-1, 1, A.n)
    x0 = rng.uniform(-1, 1, A.n)
    bd = dev(b)
    with hierarchy(A, max_coarse=mc) as h:
        assert amg.amg_num_levels(h) == len(H.levels), case
        for kind in KINDS:
            beta, a = oracle_params(kind, 3)
            x = nan_vec(A.n)
            amg.smoother_apply(h, 0, kind, 3, bd, x, True)
            xd = dev(x0)
            amg.smoother_apply(h, 0, kind, 3, bd, xd, False)
            z = nan_vec(A.n)
            amg.vcycle_apply(h, kind, 3, bd, z)
            torch.cuda.synchronize()
            assert relerr(host(x), S.smooth(As, Minv, b, None, kind, 3, beta, a)) <= TOL, (case, kind)
            assert relerr(host(xd), S.smooth(As, Minv, b, x0, kind, 3, beta, a)) <= TOL, (case, kind)
            assert relerr(host(z), OA.vcycle(H, b, kind, 3, beta)) <= TOL, (case, kind)
        for kind in (2, 3):
            beta, _ = oracle_params(kind, 4)
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve(h, kind, 4, bd, x, True, 1e-8, 1000)
            torch.cuda.synchronize()
            ro, _ = OA.amg_pcg(As, b, A.grid, kind, 4, H=H, beta=beta)
            assert rc == amg.AMG_OK and it == ro.iters, (case, kind, it, ro.iters)
            assert relerr(host(x), ro.x) <= 1e-10, (case, kind)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_pcg_high_degrees_match_oracle(amg, kind):
    """Degrees 8..12 (the higher-degree trends of the supplement): exact PCG counts at 24^3."""
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=24)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid, max_coarse=512)
    with hierarchy(A, max_coarse=512) as h:
        for k in range(8, 13):
            x = nan_vec(A.n)
            rc, it, rel, hist = amg.pcg_solve(h, kind, k, dev(b), x, True, 1e-8, 1000, False, True)
            torch.cuda.synchronize()
            beta, _ = oracle_params(kind, k)
            ro, _ = OA.amg_pcg(As, b, A.grid, kind, k, H=H, beta=beta)
            assert rc == amg.AMG_OK and it == ro.iters, (kind, k, it, ro.iters)
            assert np.allclose(hist, ro.history, rtol=1e-6, atol=0)


def _golden_c2():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_pcg_iterations_128.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            kind, k, it, rel = line.split()
            rows.append((int(kind), int(k), int(it), float(rel)))
    return rows


def test_pcg_iterations_full_size_c2(amg):
    """128^3: iteration counts of every (kind, degree) equal the oracle's stored counts."""
    torch = torch_cuda()
    A, b, _ = W.config_problem(2)
    bd = dev(b)
    with hierarchy(A) as h:
        for kind, k, it_o, rel_o in _golden_c2():
            x = nan_vec(A.n)
            rc, it, rel, _ = amg.pcg_solve(h, kind, k, bd, x, True, 1e-8, 1000)
            torch.cuda.synchronize()
            assert rc == amg.AMG_OK and it == it_o, (kind, k, it, it_o)
            assert rel == pytest.approx(rel_o, rel=1e-6)
            # true residual of the returned x (oracle SpMV)
            xr = host(x)
            assert np.linalg.norm(b - A.to_scipy() @ xr) <= 1.05e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("flexible", [False, True])
def test_pcg_iterate_at_the_iteration_limit(amg, flexible):
    """Solves stopped by their iteration limit (1, 2, 3 and 7 iterations) return the oracle's CG
    iterate after as many iterations, with the V-cycle and with the smoother alone as the
    preconditioner: inside the loop x trails by one iteration (its update rides on the next
    direction pass), so the exit must add the last iteration's alpha p."""
    torch = torch_cuda()
    g = W.gaussian_random_field((30, 36, 40), 4.0, 91)
    A = W.fv_diffusion(np.exp(g))
    b = W.rhs_uniform(A.n, 92)
    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid)
    beta, _ = oracle_params(2, 4)
    Minv = S.l1_diagonal(As)
    preconds = {"pcg_solve": lambda r: OA.vcycle(H, r, 2, 4, beta),
                "pcg_solve_smoother": lambda r: S.smooth(As, Minv, r, None, 2, 4, beta, None)}
    with hierarchy(A) as h:
        assert amg.amg_num_levels(h) == len(H.levels) > 1
        for name, precond in preconds.items():
            for maxit in (1, 2, 3, 7):
                x = nan_vec(A.n)
                rc, it, rel, _ = getattr(amg, name)(h, 2, 4, dev(b), x, True, 1e-14, maxit, flexible)
                torch.cuda.synchronize()
                ro = OA.pcg(As, b, precond, 1e-14, maxit, flexible)
                assert rc == amg.AMG_NOT_CONVERGED and it == maxit == ro.iters, (name, maxit)
                assert rel == pytest.approx(ro.relres, rel=1e-9), (name, maxit)
                assert relerr(host(x), ro.x) <= 1e-10, (name, maxit, flexible)


def test_pcg_deterministic(amg):
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=48)
    with hierarchy(A) as h:
        xs = []
        for _ in range(2):
            x = nan_vec(A.n)
            amg.pcg_solve(h, 2, 4, dev(b), x)
            torch.cuda.synchronize()
            xs.append(host(x))
    assert np.array_equal(xs[0], xs[1])


def test_pcg_nonzero_start_and_flexible(amg):
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=24)
    As = A.to_scipy()
    with hierarchy(A, max_coarse=512) as h:
        x = dev(np.random.default_rng(1).uniform(-1, 1, A.n))
        rc, it, rel, hist = amg.pcg_solve(h, 3, 3, dev(b), x, False, 1e-10, 200, True, True)
        torch.cuda.synchronize()
        assert rc == amg.AMG_OK and rel <= 1e-10 and hist[0] > 0.1
        assert np.linalg.norm(b - As @ host(x)) <= 2e-10 * np.linalg.norm(b)


# ---------------------------------------------------------------------------
# error paths (forced from the host)
# ---------------------------------------------------------------------------
def test_error_codes(amg):
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=16)
    with hierarchy(A) as h:
        x = nan_vec(A.n)
        for kind, k in ((4, 2), (-1, 2), (2, 0), (2, 13)):
            with pytest.raises(amg.AmgError) as ei:
                amg.smoother_apply(h, 0, kind, k, dev(b), x, True)
            assert ei.value.code == amg.AMG_EINVAL
        with pytest.raises(amg.AmgError):
            amg.smoother_apply(h, 5, 2, 2, dev(b), x, True)
        bn = b.copy()
        bn[17] = np.nan
        with pytest.raises(amg.AmgError) as ei:
            amg.pcg_solve(h, 2, 4, dev(bn), x)
        assert ei.value.code == amg.AMG_ENAN
        # 16^3 is a one-level hierarchy (V-cycle = exact solve): one iteration suffices
        rc, it, rel, _ = amg.pcg_solve(h, 2, 4, dev(b), x, True, 1e-8, 1)
        assert rc == amg.AMG_OK and it == 1 and rel < 1e-12
        rc, it, rel, _ = amg.pcg_solve(h, 2, 4, dev(np.zeros(A.n)), x)
        torch.cuda.synchronize()
        assert rc == amg.AMG_OK and it == 0 and np.all(host(x) == 0)
    A2, b2, _ = W.config_problem(2, size=24)
    with hierarchy(A2, max_coarse=512) as h:
        x = nan_vec(A2.n)
        rc, it, rel, _ = amg.pcg_solve(h, 2, 4, dev(b2), x, True, 1e-8, 1)
        assert rc == amg.AMG_NOT_CONVERGED and it == 1 and rel > 1e-8
    bad = W.poisson3d_7pt(6)
    r0, r1 = bad.row_ptr[10], bad.row_ptr[11]
    d = r0 + int(np.where(bad.col[r0:r1] == 10)[0][0])  # diagonal entry of row 10
    bad.val = bad.val.copy()
    bad.val[d] = -6.0
    with pytest.raises(amg.AmgError) as ei:
        with hierarchy(bad):
            pass
    assert ei.value.code == amg.AMG_ENOTSPD


def test_storage_layouts(amg):
    """Stencil levels use offset-aligned slices (no column indices read), dense or irregular rows
    the packed layout, and wide coarse rows several lanes per row; every layout matches the oracle."""
    torch = torch_cuda()
    A = W.poisson3d_7pt(32)
    with hierarchy(A) as h:
        for l in range(amg.amg_num_levels(h)):
            padded, lanes, aligned = amg.amg_level_layout(h, l)
            assert aligned and lanes == 1, (l, padded, lanes, aligned)
        padded, _, _ = amg.amg_level_layout(h, 0)
        # slices hold the offsets their rows use: seven inside, fewer on the boundary planes
        assert A.nnz <= padded <= 7 * A.n
    Q, _, _ = W.qdq_dense(256, "equispaced")
    with hierarchy(Q, max_coarse=4096) as h:
        padded, lanes, aligned = amg.amg_level_layout(h, 0)
        assert not aligned and lanes == 1 and padded == 256 * 256
    with hierarchy(W.poisson3d_7pt(24), max_coarse=100, smoothed=True) as h:
        lanes = [amg.amg_level_layout(h, l)[1] for l in range(amg.amg_num_levels(h))]
        assert lanes[0] == 1 and max(lanes[1:]) > 1, lanes
    # an irregular sparsity pattern (random SPD graph Laplacian): packed layout, smoother parity
    rng = np.random.default_rng(12)
    n = 3000
    G = sp_random_graph(n, 9, rng)
    with hierarchy(G, max_coarse=4096) as h:
        assert not amg.amg_level_layout(h, 0)[2]
        Gs = G.to_scipy()
        Minv = S.l1_diagonal(Gs)
        r = rng.uniform(-1, 1, n)
        for kind in KINDS:
            x = nan_vec(n)
            amg.smoother_apply(h, 0, kind, 4, dev(r), x, True)
            torch.cuda.synchronize()
            beta, a = oracle_params(kind, 4)
            assert relerr(host(x), S.smooth(Gs, Minv, r, None, kind, 4, beta, a)) <= 1e-12


def sp_random_graph(n, deg, rng):
    """Graph Laplacian of a random graph plus the identity (SPD, irregular pattern)."""
    import scipy.sparse as sps
    rows = np.repeat(np.arange(n), deg)
    cols = rng.integers(0, n, n * deg)
    keep = rows != cols
    Wm = sps.coo_matrix((rng.uniform(0.5, 1.5, keep.sum()), (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    Wm = (Wm + Wm.T).tocsr()
    Lap = sps.diags(np.asarray(Wm.sum(axis=1)).ravel() + 1.0) - Wm
    Lap = Lap.tocsr()
    Lap.sort_indices()
    return W.CSR(n=n, row_ptr=Lap.indptr.astype(np.int32), col=Lap.indices.astype(np.int32),
                 val=Lap.data.astype(np.float64), grid=(n, 1, 1))


@pytest.mark.parametrize("case", ["poisson_ragged", "q1_odd", "fv_batch", "poisson2d"])
def test_restriction_product(amg, case):
    """Box levels restrict with the product R = P^T A (b_c = P^T b - R x, no fine residual), stored
    in slices aligned on each aggregate's first row: 7-point levels keep at most 32 offsets per
    slice, 27-point ones at most 64.  On every level, in FP64 and FP32, b_c matches the oracle's
    P^T (b - A x); the smoothed prolongator reports its explicit transpose instead."""
    torch = torch_cuda()
    nbatch, mc, width = 1, 40, 32
    if case == "poisson_ragged":
        A = W.poisson3d_7pt(17, 10, 13)
    elif case == "q1_odd":
        A = W.q1_27pt(13, 9, 11)
        width = 64
    elif case == "fv_batch":
        A = W.stack_block_diagonal([_fv((9, 8, 6), s, 40 + p) for p, s in enumerate((0.5, 2.0))])
        nbatch, mc = 2, 8
    else:
        A = W.poisson2d_5pt(45, 38)
        width = 16
    H = OA.build_hierarchy(A.to_scipy(), A.grid, nbatch=nbatch, max_coarse=mc)
    for prec, tol in ((amg.AMG_FP64, 1e-14), (amg.AMG_FP32, 2e-6)):
        with hierarchy(A, nbatch=nbatch, max_coarse=mc, precision=prec) as h:
            assert amg.amg_num_levels(h) == len(H.levels) >= 3
            for l in range(len(H.levels) - 1):
                form, stored = amg.amg_level_transfer(h, l)
                n, nc = H.levels[l].A.shape[0], H.levels[l + 1].A.shape[0]
                assert form == amg.AMG_TRANSFER_PRODUCT, (l, form)
                assert stored % 64 == 0 and stored <= width * ((nc + 63) // 64 * 64), (l, stored)
                rng = np.random.default_rng(50 + l)
                b, x = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
                ref = H.levels[l].P.T @ (b - H.levels[l].A @ x)
                if prec == amg.AMG_FP64:
                    bc = nan_vec(nc)
                    amg.amg_restrict_residual(h, l, dev(b), dev(x), bc)
                    torch.cuda.synchronize()
                    assert relerr(host(bc), ref) <= tol, (l, relerr(host(bc), ref))
            if prec == amg.AMG_FP32:
                # the FP32 V-cycle restricts with the float copy of R: one cycle against the oracle
                z = nan_vec(A.n)
                r = W.rhs_uniform(A.n, 77)
                amg.vcycle_apply(h, 2, 3, dev(r), z)
                torch.cuda.synchronize()
                zo = OA.vcycle(H, r, 2, 3, oracle_params(2, 3)[0])
                assert relerr(host(z), zo) <= 1e-4
    with hierarchy(W.poisson3d_7pt(12), max_coarse=100, smoothed=True) as h:
        assert amg.amg_level_transfer(h, 0)[0] == amg.AMG_TRANSFER_EXPLICIT
    with pytest.raises(amg.AmgError):
        with hierarchy(W.poisson3d_7pt(8), max_coarse=100) as h:
            amg.amg_level_transfer(h, amg.amg_num_levels(h) - 1)
