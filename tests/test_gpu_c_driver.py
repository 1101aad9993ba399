"""The library called from plain C on the GPU (tests/c_driver.c: HIP runtime and the C ABI only,
no Python or torch in that process), checked against the oracle: one smoother application, one
V-cycle and a PCG solve on a ragged variable-coefficient diffusion problem (40 x 36 x 30, three
levels), at the parity bars of the other tests (1e-12 relative per application, the oracle's
iteration count)."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
sys.path.insert(0, ROOT)
from gpu_util import oracle_params, relerr, torch_cuda  # noqa: E402

import workloads as W  # noqa: E402
from oracle import amg as OA  # noqa: E402
from oracle import smoothers as S  # noqa: E402

pytestmark = pytest.mark.gpu


def _build(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pkg = os.path.join(ROOT, "paper_2407_09848_amd")
    if not os.path.exists(os.path.join(pkg, "libamgpoly.so")):
        raise RuntimeError("libamgpoly.so is not built")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "c_driver")
    cmd = [cc, "-O1", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), os.path.join(HERE, "c_driver.c"), "-L", pkg, "-lamgpoly",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", f"-Wl,-rpath,{pkg}", f"-Wl,-rpath,{rocm}/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_c_caller_matches_oracle(tmp_path):
    torch_cuda()
    exe = _build(tmp_path)
    g = W.gaussian_random_field((30, 36, 40), 4.0, 77)
    A = W.fv_diffusion(np.exp(1.5 * g))
    assert A.grid == (40, 36, 30)
    b = W.rhs_uniform(A.n, 78)
    with open(tmp_path / "A.bin", "wb") as f:
        np.array([A.n, A.nnz], dtype=np.int64).tofile(f)
        A.row_ptr.astype(np.int32).tofile(f)
        A.col.astype(np.int32).tofile(f)
        A.val.astype(np.float64).tofile(f)
    b.astype(np.float64).tofile(tmp_path / "b.bin")
    print(f"c_driver on {A.grid}, {A.n} rows", flush=True)
    r = subprocess.run([exe, str(tmp_path), *map(str, A.grid)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    words = r.stdout.split()
    levels, iters, relres = int(words[1]), int(words[3]), float(words[5])

    As = A.to_scipy()
    H = OA.build_hierarchy(As, A.grid)
    assert levels == len(H.levels) == 3
    read = lambda name: np.fromfile(tmp_path / name, dtype=np.float64)
    beta4, _ = oracle_params(2, 4)
    _, a3 = oracle_params(3, 3)
    xs = S.smooth(As, S.l1_diagonal(As), b, None, 2, 4, beta4, None)
    assert relerr(read("smooth.bin"), xs) <= 1e-12
    assert relerr(read("vcycle.bin"), OA.vcycle(H, b, 3, 3, None)) <= 1e-12
    ro, _ = OA.amg_pcg(As, b, A.grid, 2, 4, H=H, beta=beta4)
    assert iters == ro.iters and relres <= 1e-8
    assert relerr(read("pcg.bin"), ro.x) <= 1e-10
    print(f"C caller: {levels} levels, {iters} iterations (oracle {ro.iters})", flush=True)
