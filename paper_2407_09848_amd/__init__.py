"""MI355X-native polynomial-smoothed AMG-PCG (hot path of arXiv 2407.09848).

Thin Python binding over the C ABI of ``libamgpoly.so`` (declared in
include/amgpoly.h).  Functions carry the C names and only marshal
arguments: torch tensors supply device memory and the current HIP stream;
every step of the computation runs in the library's HIP kernels.  There is
no fallback: if the library is not built, importing the binding raises.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import __all__  # noqa: F401
