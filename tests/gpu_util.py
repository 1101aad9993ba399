"""Helpers shared by the GPU tests: move workload matrices to the device and
build hierarchies through the C ABI.  (Not collected: no test functions.)"""
import contextlib

import numpy as np

KINDS = [0, 1, 2, 3]


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda", dtype=dtype) if dtype is not None else t.to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


def nan_vec(n):
    torch = torch_cuda()
    return torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")


@contextlib.contextmanager
def hierarchy(A, nbatch=1, max_coarse=4096, precision=0, **opts):
    import paper_2407_09848_amd as amg
    torch = torch_cuda()
    nx, ny, nz = A.grid
    nz_per = nz // nbatch
    rp = dev(A.row_ptr.astype(np.int32))
    cl = dev(A.col.astype(np.int32))
    vl = dev(A.val.astype(np.float64))
    h = amg.amg_setup(rp, cl, vl, nx, ny, nz_per, nbatch, max_coarse, precision, **opts)
    torch.cuda.synchronize()
    try:
        yield h
    finally:
        torch.cuda.synchronize()
        amg.amg_destroy(h)


def relerr(a, b):
    """Relative error of a against b: the larger of the norm-wise ||a - b|| / ||b|| and the
    element-wise max_i |a_i - b_i| / max_i |b_i|, so that one wrong entry (a boundary row, a
    slice tail) is not averaged away over millions of correct ones.  NaN anywhere gives NaN,
    which fails every bound."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    d = a - b
    if d.size and not np.all(np.isfinite(d)):
        return float("nan")
    norm_wise = np.linalg.norm(d) / (nb if nb > 0 else 1.0)
    elem_wise = (np.abs(d).max() if d.size else 0.0) / (mb if mb > 0 else 1.0)
    return max(norm_wise, elem_wise)


def oracle_params(kind, k):
    from oracle import polynomials as P
    beta = P.optimal_beta(k)[0] if kind == 2 else None
    a = P.a_star(k) if kind == 3 else None
    return beta, a


def oracle_aggregates(H, aggregation, opts):
    """Aggregate index of every row of each non-coarsest level of the oracle hierarchy H, as the
    oracle builds them (box, VBM, or the composite of the matching steps)."""
    from oracle import amg as OA
    from oracle import matching as OM
    from oracle import vbm as OV
    out = []
    w = None
    for l, lv in enumerate(H.levels[:-1]):
        if aggregation == "box":
            agg, _ = OA.box_aggregates(lv.grid, lv.nbatch, opts.get("agg_edge", 2))
        elif aggregation == "vbm":
            agg, _ = OV.vbm_aggregates(lv.A, opts.get("vbm_theta", 0.08) * 0.5**l)
        else:
            Pm, w = OM.matching_prolongator(lv.A, w, opts.get("match_steps", 3))
            assert np.all(np.diff(Pm.indptr) == 1)
            agg = Pm.indices
        out.append(np.asarray(agg, dtype=np.int64))
    return out
