"""Host-side checks of the C-ABI library (no GPU compute).

* the built library loads and exports every function include/*.h declares;
* the library's compiled-in constant tables (its own generator) agree with
  the oracle's independently computed a*_k and optimal beta;
* argument validation that returns before any device work.
"""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(hdr).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:int|const char\s*\*|int64_t|size_t|double)\s*\**\s*([a-z_0-9]+)\s*\(", txt,
                            flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    import paper_2407_09848_amd as amg
    return amg.lib()


def test_library_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 17
    for nm in names:
        assert hasattr(L, nm), nm


def test_strerror_covers_codes(L):
    import paper_2407_09848_amd as amg
    for c in range(-7, 2):
        assert amg.amg_strerror(c) != "unknown error"
    assert amg.amg_strerror(99) == "unknown error"


@pytest.mark.parametrize("k", range(1, 13))
def test_astar_table_matches_oracle(k):
    import paper_2407_09848_amd as amg
    from oracle import polynomials as P
    assert amg.amg_default_astar(k) == pytest.approx(P.a_star(k), rel=4e-16)


@pytest.mark.parametrize("k", range(1, 7))
def test_beta_table_matches_oracle(k):
    import paper_2407_09848_amd as amg
    from oracle import polynomials as P
    lib_beta = np.array(amg.amg_default_beta(k))
    orc_beta = np.array(P.optimal_beta(k)[0])
    assert np.allclose(lib_beta, orc_beta, rtol=1e-14, atol=0)


def test_generator_is_independent_of_oracle():
    src = open(os.path.join(ROOT, "paper_2407_09848_amd", "gen_coeffs.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_argument_validation_before_device_work(L):
    import paper_2407_09848_amd as amg
    P = ctypes.c_void_p
    h = P()
    # null out pointer / null matrix / bad options are rejected without touching the GPU
    assert L.amg_setup(10, 10, None, None, None, None, None, None) == amg.AMG_EINVAL
    o = amg._binding.AmgOpts(2, 2, 2, 1, 0, 0)
    assert L.amg_setup(8, 8, None, None, None, ctypes.byref(o), None, ctypes.byref(h)) == amg.AMG_EINVAL
    assert L.amg_destroy(None) == amg.AMG_OK
    assert L.smoother_apply(None, 0, 0, 1, None, None, 1, None) == amg.AMG_EINVAL
    assert L.pcg_solve(None, 2, 4, None, None, 1, 1e-8, 10, 0, None, None, None, None) == amg.AMG_EINVAL
    buf = (ctypes.c_double * 13)()
    assert L.amg_default_beta(0, buf) == amg.AMG_EINVAL
    assert L.amg_default_beta(13, buf) == amg.AMG_EINVAL
    assert L.amg_default_beta(4, buf) == amg.AMG_OK
    # learned weights and the ceiling kernels: null handle / pointers, degree beyond the network
    assert L.amg_learned_beta(None, 4, None, 4096, None, None, None) == amg.AMG_EINVAL
    assert L.amg_learned_beta_grad(None, 4, None, None, None, None) == amg.AMG_EINVAL
    assert L.amg_hbm_read(None, 10, None, None) == amg.AMG_EINVAL
    assert L.amg_hbm_copy(None, None, 10, None) == amg.AMG_EINVAL
    # misaligned (not 16-byte) and overlapping ranges are rejected before any launch
    assert L.amg_hbm_read(P(8), 10, P(256), None) == amg.AMG_EINVAL
    assert L.amg_hbm_copy(P(256), P(272), 10, None) == amg.AMG_EINVAL
    # an option out of range is rejected before the (here fake) device pointers are touched
    o = amg._binding.AmgOpts(4, 4, 4, 1, 0, 0)
    o.drop_fine_csr = 2
    assert L.amg_setup(64, 64, P(4096), P(8192), P(16384), ctypes.byref(o), None, ctypes.byref(h)) == amg.AMG_EINVAL
    assert not h.value


def test_option_struct_layout_matches_the_header(tmp_path):
    """The binding's amg_opts mirrors the C struct: same size and field offsets (a C program built
    against include/amgpoly.h prints them)."""
    import shutil
    import subprocess

    import paper_2407_09848_amd as amg
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f[0] for f in amg._binding.AmgOpts._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"amgpoly.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(amg_opts));\n" +
                   "".join(f"  printf(\"%zu\\n\", offsetof(amg_opts, {f}));\n" for f in fields) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(amg._binding.AmgOpts)
    assert out[1:] == [getattr(amg._binding.AmgOpts, f).offset for f in fields]


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_2407_09848_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*.py"), recursive=True) + \
            glob.glob(os.path.join(pkg, "csrc", "*")) + [os.path.join(ROOT, "include", "amgpoly.h")]:
        txt = open(path).read()
        assert "from oracle" not in txt and "import oracle" not in txt, path
