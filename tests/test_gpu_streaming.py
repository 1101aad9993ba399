"""Full-vector parity of the streaming kernels (levels above 12288 blocks of 256 rows).

Levels of more than 3.1M rows take kernels with nontemporal loads and stores
and a block order that hands runs of 128 consecutive blocks to each XCD in
turn; the blocks past the last whole round of 8 runs (1024 blocks) keep the
launch order.  Every full-size workload runs its fine level on these kernels.
Here they are compared with the oracle on every entry (NaN-prefilled outputs,
the element-wise and norm-wise bound of `relerr`):
* 7-point 128 x 128 x 257 (4,210,688 rows, 16448 blocks: 16 rounds and a tail
  of 64 blocks), all four kinds at degrees 1..6 from x = 0, degree 3 from
  x != 0, and V-cycles;
* 7-point 256^3 (16,777,216 rows, 65536 blocks: whole rounds only), the
  optimal kinds at degrees 1..6, the other two at 1, 4 and 6, and one V-cycle;
* 27-point Q1 164^3 (4,410,944 rows, 17232 blocks: a tail of 848 blocks), and
  CG preconditioned by its smoother (the residual update feeding M^-1 r to it);
* the differentiable V-cycle and the training loss on 20 stacked 64^3
  diffusion problems (5,242,880 rows, 20480 blocks) at degree 6, against the
  oracle per problem and the complex-step derivative on sampled weights.
"""
import os
import sys
import time

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import dev, hierarchy, host, nan_vec, oracle_params, relerr, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402
from oracle import adjoint as AD  # noqa: E402
from oracle import amg as OA  # noqa: E402
from oracle import polynomials as P  # noqa: E402
from oracle import smoothers as S  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12
STREAM_MIN_BLOCKS = 12288
XCD_ROUND = 8 * 128  # blocks per round of XCD runs on streaming levels


def _log(msg):
    print(msg, flush=True)


def _blocks(n):
    return (n + 255) // 256


class _Problem:
    def __init__(self, A, seed):
        self.A = A
        self.As = A.to_scipy()
        self.Minv = S.l1_diagonal(self.As)
        self.b = W.rhs_uniform(A.n, seed)
        self.x0 = W.rhs_uniform(A.n, seed + 1)


@pytest.fixture(scope="module")
def p4m():
    torch_cuda()
    A = W.poisson3d_7pt(128, 128, 257)
    assert _blocks(A.n) > STREAM_MIN_BLOCKS and _blocks(A.n) % XCD_ROUND == 64
    return _Problem(A, 301)


@pytest.fixture(scope="module")
def p256():
    torch_cuda()
    t = time.time()
    A = W.poisson3d_7pt(256)
    pr = _Problem(A, 302)
    _log(f"256^3 assembled in {time.time() - t:.1f} s")
    return pr


def _check_smoother(amg, h, pr, kind, k, from_zero):
    torch = torch_cuda()
    beta, a = oracle_params(kind, k)
    if from_zero:
        x = nan_vec(pr.A.n)
        amg.smoother_apply(h, 0, kind, k, dev(pr.b), x, True)
        xo = S.smooth(pr.As, pr.Minv, pr.b, None, kind, k, beta, a)
    else:
        x = dev(pr.x0)
        amg.smoother_apply(h, 0, kind, k, dev(pr.b), x, False)
        xo = S.smooth(pr.As, pr.Minv, pr.b, pr.x0, kind, k, beta, a)
    torch.cuda.synchronize()
    e = relerr(host(x), xo)
    assert e <= TOL, (kind, k, from_zero, e)
    return e


def test_streaming_smoother_4m_all_kinds_degrees(p4m):
    import paper_2407_09848_amd as amg
    with hierarchy(p4m.A) as h:
        for kind in (0, 1, 2, 3):
            errs = [_check_smoother(amg, h, p4m, kind, k, True) for k in range(1, 7)]
            errs.append(_check_smoother(amg, h, p4m, kind, 3, False))
            _log(f"4.2M rows kind {kind}: max error over k = 1..6 and x0 != 0: {max(errs):.2e}")


def test_streaming_vcycle_4m(p4m):
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    H = OA.build_hierarchy(p4m.As, p4m.A.grid)
    with hierarchy(p4m.A) as h:
        assert amg.amg_num_levels(h) == len(H.levels)
        for kind, k in ((0, 2), (1, 2), (2, 2), (3, 2), (2, 6), (3, 5)):
            z = nan_vec(p4m.A.n)
            amg.vcycle_apply(h, kind, k, dev(p4m.b), z)
            torch.cuda.synchronize()
            beta, _ = oracle_params(kind, k)
            e = relerr(host(z), OA.vcycle(H, p4m.b, kind, k, beta))
            _log(f"4.2M rows V-cycle kind {kind} k {k}: {e:.2e}")
            assert e <= TOL, (kind, k, e)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_streaming_smoother_256(p256, kind):
    import paper_2407_09848_amd as amg
    degrees = range(1, 7) if kind in (2, 3) else (1, 4, 6)
    with hierarchy(p256.A) as h:
        errs = [_check_smoother(amg, h, p256, kind, k, True) for k in degrees]
    _log(f"256^3 kind {kind}: max error over k in {list(degrees)}: {max(errs):.2e}")


def test_streaming_vcycle_256(p256):
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    t = time.time()
    H = OA.build_hierarchy(p256.As, p256.A.grid)
    _log(f"256^3 oracle hierarchy in {time.time() - t:.1f} s")
    with hierarchy(p256.A) as h:
        z = nan_vec(p256.A.n)
        amg.vcycle_apply(h, 2, 4, dev(p256.b), z)
        torch.cuda.synchronize()
        e = relerr(host(z), OA.vcycle(H, p256.b, 2, 4))
    _log(f"256^3 V-cycle (optimal 4th kind, k = 4): {e:.2e}")
    assert e <= TOL


@pytest.fixture(scope="module")
def p27():
    torch_cuda()
    A = W.q1_27pt(164)
    assert _blocks(A.n) > STREAM_MIN_BLOCKS and ((_blocks(A.n) + 7) // 8 * 8) % XCD_ROUND == 848
    return _Problem(A, 303)


def test_streaming_27pt_tail_blocks(p27):
    torch_cuda()
    import paper_2407_09848_amd as amg
    pr = p27
    with hierarchy(pr.A) as h:
        padded, lanes, aligned = amg.amg_level_layout(h, 0)
        assert aligned and lanes == 1
        errs = [_check_smoother(amg, h, pr, kind, 4, True) for kind in (2, 3)]
        errs.append(_check_smoother(amg, h, pr, 2, 3, False))
        errs.append(_check_smoother(amg, h, pr, 0, 2, True))
    _log(f"27-point 164^3: max error {max(errs):.2e}")


def test_streaming_27pt_pcg_smoother_iterates(p27):
    """CG preconditioned by the fine-level smoother alone on the 27-point level: from the second
    iteration on, its residual update also writes u = M^-1 r, which the smoother's merged first
    two steps read in place of the gathered M^-1 and r.  The iterate after three iterations
    matches the oracle's CG iterate (kinds 1-3, degree 4; the optimal 4th kind also in the
    flexible CG, whose dot products take r_old as well)."""
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    pr = p27
    errs = []
    with hierarchy(pr.A) as h:
        for kind, flex in ((1, False), (2, False), (3, False), (2, True)):
            beta, a = oracle_params(kind, 4)
            x = nan_vec(pr.A.n)
            rc, it, rel, _ = amg.pcg_solve_smoother(h, kind, 4, dev(pr.b), x, True, 1e-14, 3, flex)
            torch.cuda.synchronize()
            ro = OA.pcg(pr.As, pr.b, lambda r: S.smooth(pr.As, pr.Minv, r, None, kind, 4, beta, a), 1e-14, 3, flex)
            assert rc == amg.AMG_NOT_CONVERGED and it == 3 == ro.iters, (kind, flex)
            assert rel == pytest.approx(ro.relres, rel=1e-9), (kind, flex)
            errs.append(relerr(host(x), ro.x))
            assert errs[-1] <= 1e-10, (kind, flex, errs[-1])
    _log(f"27-point 164^3 smoother-preconditioned CG: max error {max(errs):.2e}")


# ---------------------------------------------------------------------------
# differentiable V-cycle on a stack above the streaming threshold
# ---------------------------------------------------------------------------
SAMPLES = [(0, 0, 0), (7, 0, 5), (13, 1, 2), (19, 1, 5), (4, 0, 3), (11, 1, 0)]


@pytest.fixture(scope="module")
def stack20():
    torch_cuda()
    P_, n = 20, 64
    sig = W.config4_sigmas(P_)
    mats = [W.fv_diffusion(np.exp(sig[p] * W.gaussian_random_field((n,) * 3, 8.0, 400 + p))) for p in range(P_)]
    big = W.stack_block_diagonal(mats)
    assert _blocks(big.n) > STREAM_MIN_BLOCKS and _blocks(big.n) % XCD_ROUND == 0
    Hs = [OA.build_hierarchy(m.to_scipy(), m.grid) for m in mats]
    rng = np.random.default_rng(31)
    base = np.array(P.optimal_beta(6)[0])
    tab = np.tile(base, (P_, 3, 1))
    tab[:, :2, :] *= 1 + 0.05 * rng.standard_normal((P_, 2, 6))
    return mats, big, Hs, tab


def test_streaming_adjoint_stack(stack20):
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    mats, big, Hs, tab = stack20
    k, P_ = 6, len(mats)
    rng = np.random.default_rng(32)
    r = rng.uniform(-1, 1, big.n)
    c = rng.uniform(-1, 1, big.n)
    with hierarchy(big, nbatch=P_) as h:
        L = amg.amg_num_levels(h)
        assert L == 3 == len(Hs[0].levels)
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
    ez = eg = 0.0
    for p in range(P_):
        sl = slice(p * m0, (p + 1) * m0)
        betas = [tab[p, l] for l in range(L - 1)]
        ez = max(ez, relerr(zh[sl], AD.vcycle_beta(Hs[p], r[sl], k, betas)))
        eg = max(eg, relerr(grh[sl], AD.vcycle_beta(Hs[p], c[sl], k, betas)))
    _log(f"stack 20 x 64^3, k = 6: z error {ez:.2e}, dL/dr error {eg:.2e}")
    assert ez <= TOL and eg <= TOL
    assert np.all(gbh[:, L - 1] == 0)
    for (p, l, j) in SAMPLES:
        sl = slice(p * m0, (p + 1) * m0)
        bc = [np.array(tab[p, ll], dtype=complex) for ll in range(L - 1)]
        bc[l][j] += 1e-30j
        go = np.sum(c[sl] * AD.vcycle_beta(Hs[p], r[sl], k, bc)).imag / 1e-30
        assert gbh[p, l, j] == pytest.approx(go, rel=1e-9), (p, l, j, gbh[p, l, j], go)


def test_streaming_train_loss_stack(stack20):
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    mats, big, Hs, tab = stack20
    k, P_ = 6, len(mats)
    b = W.rhs_uniform(big.n, 33)
    m0 = mats[0].n
    with hierarchy(big, nbatch=P_) as h:
        L = amg.amg_num_levels(h)
        beta = dev(tab.ravel())
        g = torch.empty_like(beta)
        loss, ratios = amg.amg_train_loss_grad(h, k, beta, dev(b), g, P_)
        torch.cuda.synchronize()
        gh = host(g).reshape(P_, L, k)
    betas = [[tab[p, l] for l in range(L - 1)] for p in range(P_)]
    ro = [AD.two_cycle_ratio(Hs[p], b[p * m0:(p + 1) * m0], k, betas[p]) for p in range(P_)]
    for p in range(P_):
        assert ratios[p] == pytest.approx(ro[p], rel=1e-12), p
    assert loss == pytest.approx(sum(ro) / P_, rel=1e-12)
    for (p, l, j) in SAMPLES:
        bc = [np.array(v, dtype=complex) for v in betas[p]]
        bc[l][j] += 1e-30j
        go = AD.two_cycle_ratio(Hs[p], b[p * m0:(p + 1) * m0], k, bc).imag / 1e-30 / P_
        assert gh[p, l, j] == pytest.approx(go, rel=1e-9), (p, l, j, gh[p, l, j], go)
    _log(f"stack 20 x 64^3, k = 6: loss {loss:.6f}, {len(SAMPLES)} sampled gradient entries match")
