"""The bandwidth-ceiling kernels (amg_hbm_read, amg_hbm_copy): the read's block sums add up to the
sum of the array, the copy is exact, odd and tiny lengths included; misaligned or overlapping
arguments are rejected."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_util import dev, host, torch_cuda  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 3, 1000, 1_000_003, 16384 * 256 * 2 * 9 + 5])
def test_read_and_copy(n):
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    x = np.random.default_rng(n).uniform(-1, 1, n)
    xd = dev(x)
    part = torch.full((amg.AMG_HBM_PARTIALS,), float("nan"), dtype=torch.float64, device="cuda")
    amg.amg_hbm_read(xd, part)
    y = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    amg.amg_hbm_copy(xd, y)
    torch.cuda.synchronize()
    ph = host(part)
    assert np.all(np.isfinite(ph))
    assert abs(ph.sum() - x.sum()) <= 1e-12 * max(1.0, np.abs(x).sum())
    assert np.array_equal(host(y), x)


def test_rejects_misaligned_and_overlapping():
    torch = torch_cuda()
    import paper_2407_09848_amd as amg
    x = torch.ones(1025, dtype=torch.float64, device="cuda")
    part = torch.empty(amg.AMG_HBM_PARTIALS, dtype=torch.float64, device="cuda")
    for call in (lambda: amg.amg_hbm_read(x[1:], part), lambda: amg.amg_hbm_copy(x[1:], x[:1024].clone()),
                 lambda: amg.amg_hbm_copy(x[:512], x[256:768])):
        with pytest.raises(amg.AmgError) as e:
            call()
        assert e.value.code == amg.AMG_EINVAL
