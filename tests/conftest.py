import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run (oracle at large sizes)")


def load_paper_constants():
    rows = []
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(v) for v in line.split()])
    a = np.array(rows)
    return {"k": a[:, 0].astype(int), "a_star": a[:, 1], "gamma_cheb4": a[:, 2],
            "lambda_cheb1": a[:, 3], "gamma_optcheb4": a[:, 4]}


@pytest.fixture(scope="session")
def paper_constants():
    return load_paper_constants()
