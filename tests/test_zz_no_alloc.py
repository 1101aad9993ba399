"""mlp_bwd_noalloc (the network backward with the library's static scratch) against mlp_bwd
(the same backward with a caller-supplied workspace): bitwise equal gradients on two calls in a
row, the second with a smaller batch; a batch above the scratch's capacity is rejected."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import dev, torch_cuda  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(amg, torch, params, batch, seed):
    rng = np.random.default_rng(seed)
    x = dev(rng.uniform(-1, 1, (batch, 8)).astype(np.float32))
    gy = dev(rng.uniform(-1, 1, (batch, 6)).astype(np.float32))
    y = torch.empty((batch, 6), dtype=torch.float32, device="cuda")
    cache = torch.empty((batch, 128), dtype=torch.float32, device="cuda")
    amg.mlp_fwd(params, x, y, cache)
    g_ref = torch.full_like(params, float("nan"))
    work = torch.empty(2 * batch * 64, dtype=torch.float32, device="cuda")
    amg.mlp_bwd(params, x, cache, gy, g_ref, work)
    g_new = torch.full_like(params, float("nan"))
    amg.mlp_bwd_noalloc(params, x, cache, gy, g_new)
    torch.cuda.synchronize()
    assert torch.isfinite(g_ref).all()
    assert torch.equal(g_new, g_ref), (batch, float((g_new - g_ref).abs().max()))


def test_noalloc_backward_matches_workspace_backward():
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    import workloads as W
    params = dev(np.asarray(W.mlp_init(W.SEED_MLP), dtype=np.float32))
    _case(amg, torch, params, 256, 71)   # the full capacity
    _case(amg, torch, params, 37, 72)    # a smaller batch on the same (reused) scratch
    x = torch.zeros((257, 8), dtype=torch.float32, device="cuda")
    c = torch.zeros((257, 128), dtype=torch.float32, device="cuda")
    gy = torch.zeros((257, 6), dtype=torch.float32, device="cuda")
    g = torch.empty_like(params)
    with pytest.raises(amg.AmgError) as e:
        amg.mlp_bwd_noalloc(params, x, c, gy, g)
    assert e.value.code == amg.AMG_ECAPACITY
