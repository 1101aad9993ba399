"""Setup rejects malformed input with AMG_EINVAL instead of reading past it: an empty matrix, grid
extents that do not multiply to n, and CSR arrays of the declared sizes whose contents break the
format (row pointers that do not start at 0, end at nnz or increase; column indices out of range,
unsorted or repeated in a row).  The library validates the pointers before it reads any column
index, so every case here stays within the arrays it is given."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import dev, host, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amg():
    torch_cuda()
    import paper_2407_09848_amd as amg
    return amg


def _setup(amg, rp, cl, vl, grid):
    torch = torch_cuda()
    h = amg.amg_setup(dev(rp.astype(np.int32)), dev(cl.astype(np.int32)), dev(vl.astype(np.float64)), *grid)
    torch.cuda.synchronize()
    return h


def _cases():
    A = W.poisson3d_7pt(4)
    rp, cl, vl = A.row_ptr.astype(np.int64), A.col.astype(np.int64), A.val.copy()
    n = A.n
    r5 = int(rp[5])

    def mod(rp_=None, cl_=None):
        return (rp if rp_ is None else rp_), (cl if cl_ is None else cl_)

    out = {}
    x = rp.copy()
    x[0] = 1
    out["ptr_start"] = mod(rp_=x)
    x = rp.copy()
    x[5], x[6] = x[6], x[5]
    out["ptr_decreasing"] = mod(rp_=x)
    x = rp.copy()
    x[n] -= 1
    out["ptr_end"] = mod(rp_=x)
    x = rp.copy()
    x[7] = len(cl) + 3
    out["ptr_beyond_nnz"] = mod(rp_=x)
    c = cl.copy()
    c[r5 + 1] = n
    out["col_past_n"] = mod(cl_=c)
    c = cl.copy()
    c[r5] = -1
    out["col_negative"] = mod(cl_=c)
    c = cl.copy()
    c[r5], c[r5 + 1] = c[r5 + 1], c[r5]
    out["col_unsorted"] = mod(cl_=c)
    c = cl.copy()
    c[r5 + 1] = c[r5]
    out["col_repeated"] = mod(cl_=c)
    return A, vl, out


@pytest.mark.parametrize("case", ["ptr_start", "ptr_decreasing", "ptr_end", "ptr_beyond_nnz", "col_past_n",
                                  "col_negative", "col_unsorted", "col_repeated"])
def test_malformed_csr_is_rejected(amg, case):
    A, vl, cases = _cases()
    rp, cl = cases[case]
    with pytest.raises(amg.AmgError) as e:
        _setup(amg, rp, cl, vl, A.grid)
    assert e.value.code == amg.AMG_EINVAL, case
    # the well-formed matrix still sets up on the same device afterwards
    h = _setup(amg, A.row_ptr, A.col, vl, A.grid)
    amg.amg_destroy(h)


def test_empty_and_mismatched_extents_are_rejected(amg):
    A = W.poisson3d_7pt(4)
    with pytest.raises(amg.AmgError) as e:
        _setup(amg, np.zeros(1), np.zeros(0), np.zeros(0), (1, 1, 1))
    assert e.value.code == amg.AMG_EINVAL
    for grid in ((4, 4, 5), (8, 4, 1), (0, 4, 16)):
        with pytest.raises(amg.AmgError) as e:
            _setup(amg, A.row_ptr, A.col, A.val, grid)
        assert e.value.code == amg.AMG_EINVAL, grid


def test_calls_follow_the_callers_stream(amg):
    """Every call enqueues on the caller's current stream (torch's, here a side stream of default
    priority): input written on that stream just before the call, behind a long matrix product,
    is what the call reads, with no synchronisation in between; the results equal those of the
    same calls on the default stream bitwise."""
    torch = torch_cuda()
    A, b, _ = W.config_problem(2, size=32)
    src = dev(b)
    with _hier(amg, A) as h:
        z_ref = torch.empty(A.n, dtype=torch.float64, device="cuda")
        amg.vcycle_apply(h, 2, 4, src, z_ref)
        x_ref = torch.empty_like(z_ref)
        rc, it_ref, _, _ = amg.pcg_solve(h, 2, 4, src, x_ref, True)
        torch.cuda.synchronize()
        big = torch.randn(2048, 2048, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            bd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            for _ in range(6):
                big = torch.tanh(big @ big / 2048.0)
            bd.copy_(src)
            z = torch.empty_like(bd)
            amg.vcycle_apply(h, 2, 4, bd, z)
            x = torch.empty_like(bd)
            rc2, it2, _, _ = amg.pcg_solve(h, 2, 4, bd, x, True)
        s.synchronize()
        assert rc2 == rc == amg.AMG_OK and it2 == it_ref
        assert torch.equal(z, z_ref) and torch.equal(x, x_ref)


class _hier:
    """Set up a handle on the default stream and destroy it at the end."""

    def __init__(self, amg, A):
        self.amg, self.A = amg, A

    def __enter__(self):
        self.h = _setup(self.amg, self.A.row_ptr, self.A.col, self.A.val, self.A.grid)
        return self.h

    def __exit__(self, *exc):
        torch_cuda().cuda.synchronize()
        self.amg.amg_destroy(self.h)
        return False


def test_cg_breakdown_reports_and_keeps_x(amg):
    """CG on a symmetric indefinite matrix with a positive diagonal (1D chain, a_ii = 1,
    a_i,i+1 = -2: eigenvalues 1 - 4 cos(j pi / (n + 1)), the smallest about -3): with b = M v,
    v the eigenvector of the smallest eigenvalue, the l1-Jacobi preconditioner of degree 1 gives
    z_0 = v, so (p_1, A p_1) = lambda_1 ||v||^2 < 0 at the first iteration.  The solve returns
    AMG_EBREAKDOWN and leaves x at the last iterate (x0 = 0), finite.  The setup takes l1-Jacobi
    sweeps on the coarsest level, so no factorisation sees the indefinite matrix."""
    torch = torch_cuda()
    n = 64
    rp = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        for j, v in ((i - 1, -2.0), (i, 1.0), (i + 1, -2.0)):
            if 0 <= j < n:
                cols.append(j)
                vals.append(v)
        rp[i + 1] = len(cols)
    cl = np.array(cols)
    vl = np.array(vals)
    M = np.array([1.0 + 2.0 * ((i > 0) + (i < n - 1)) for i in range(n)])
    v = np.sin(np.arange(1, n + 1) * np.pi / (n + 1))
    b = M * v
    h = amg.amg_setup(dev(rp.astype(np.int32)), dev(cl.astype(np.int32)), dev(vl), n, 1, 1, 1, 4096,
                      amg.AMG_FP64, coarse_sweeps=4)
    torch.cuda.synchronize()
    try:
        x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        with pytest.raises(amg.AmgError) as e:
            amg.pcg_solve_smoother(h, amg.AMG_L1JAC, 1, dev(b), x, True, 1e-8, 50)
        assert e.value.code == amg.AMG_EBREAKDOWN
        xh = host(x)
        assert np.all(np.isfinite(xh)) and np.all(xh == 0.0)
        # the flags are cleared by the next solve: a zero right-hand side returns at once
        rc, it, rel, _ = amg.pcg_solve_smoother(h, amg.AMG_L1JAC, 1, dev(np.zeros(n)), x, True, 1e-8, 50)
        assert rc == amg.AMG_OK and it == 0 and rel == 0.0
    finally:
        torch.cuda.synchronize()
        amg.amg_destroy(h)


def test_drop_fine_csr_frees_the_copy_and_keeps_results(amg):
    """drop_fine_csr = 1: setup reads the caller's CSR in place instead of copying it and keeps no
    CSR form of level 0 (12 bytes per stored entry less device memory); solves are bitwise the
    same, level-0 CSR export and the features are refused, the l1 diagonal and the coarser
    levels are still exported."""
    torch = torch_cuda()
    A = W.q1_27pt(96)
    b = dev(W.rhs_uniform(A.n, 51))
    rp, cl, vl = dev(A.row_ptr), dev(A.col), dev(A.val)
    out = {}
    # keep, drop, keep: the first setup of the process also pays one-time runtime allocations,
    # so the memory comparison uses the second
    for drop in (False, True, False):
        # the setup reads the caller's arrays in place with drop_fine_csr: they are left unchanged
        # and may be freed as soon as it returns
        rp2, cl2, vl2 = rp.clone(), cl.clone(), vl.clone()
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        h = amg.amg_setup(rp2, cl2, vl2, *A.grid, drop_fine_csr=drop)
        torch.cuda.synchronize()
        held = free0 - torch.cuda.mem_get_info()[0]
        assert torch.equal(rp2, rp) and torch.equal(cl2, cl) and torch.equal(vl2, vl)
        del rp2, cl2, vl2
        torch.cuda.empty_cache()
        try:
            x = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
            rc, it, rel, _ = amg.pcg_solve(h, 2, 4, b, x)
            assert rc == amg.AMG_OK
            n1, nnz1 = amg.amg_level_info(h, 1)
            c1 = amg.amg_level_export(h, 1)
            mi = torch.empty(A.n, dtype=torch.float64, device="cuda")
            assert amg._binding.lib().amg_level_export(h, 0, None, None, None, amg._binding._ptr(mi), None) == 0
            if drop:
                with pytest.raises(amg.AmgError) as e:
                    amg.amg_level_export(h, 0)
                assert e.value.code == amg.AMG_EINVAL
                with pytest.raises(amg.AmgError) as e:
                    amg.amg_level_features(h, 4, [0.0])
                assert e.value.code == amg.AMG_EINVAL
            else:
                amg.amg_level_features(h, 4, [0.0])
            torch.cuda.synchronize()
            out[drop] = (held, it, rel, host(x), host(mi), [host(t) for t in c1])
        finally:
            torch.cuda.synchronize()
            amg.amg_destroy(h)
    keep, drop = out[False], out[True]
    assert keep[1] == drop[1] and keep[2] == drop[2] and np.array_equal(keep[3], drop[3])
    assert np.array_equal(keep[4], drop[4])
    assert all(np.array_equal(a, c) for a, c in zip(keep[5], drop[5]))
    saved = keep[0] - drop[0]
    assert saved >= 0.95 * 12 * A.nnz, (keep[0], drop[0], 12 * A.nnz)
    print(f"Q1 96^3: handle {keep[0] / 1e6:.0f} MB with the level-0 CSR copy, {drop[0] / 1e6:.0f} MB without",
          flush=True)
