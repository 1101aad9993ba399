"""Pin of the sampled-row check used at full size: after k smoother steps from x = 0, the
value at row i equals the oracle recurrence run on the radius-k sub-grid around i
(M^{-1} from the full rows).  Checked against the full oracle smoother on small grids."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import workloads as W  # noqa: E402
from oracle import smoothers as S  # noqa: E402
from test_gpu_large import _l1_rows, _local_value  # noqa: E402


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("k", [2, 4])
def test_local_subgrid_reproduces_full_smoother(kind, k):
    A = W.q1_27pt(14)
    As = A.to_scipy()
    b = W.rhs_uniform(A.n, 9)
    Minv = S.l1_diagonal(As)
    assert np.array_equal(_l1_rows(As, np.arange(A.n)), Minv)
    beta, a = (None, None)
    from oracle import polynomials as P
    if kind == 2:
        beta = P.optimal_beta(k)[0]
    if kind == 3:
        a = P.a_star(k)
    x = S.smooth(As, Minv, b, None, kind, k, beta, a)
    rng = np.random.default_rng(1)
    pts = [(0, 0, 0), (13, 13, 13), (7, 7, 7), (0, 5, 13)] + [tuple(int(v) for v in rng.integers(0, 14, 3))
                                                                 for _ in range(8)]
    for pt in pts:
        i = pt[0] + 14 * pt[1] + 196 * pt[2]
        xo = _local_value(As, Minv, b, A.grid, pt, kind, k, k)
        assert xo == pytest.approx(x[i], rel=1e-13, abs=1e-15)
        if k >= 2:
            # radius k - 2 is too small in the interior: the check is sharp
            if all(k <= c <= 13 - k for c in pt):
                xs = _local_value(As, Minv, b, A.grid, pt, kind, k, k - 2)
                assert abs(xs - x[i]) > 1e-14 * abs(x[i])
