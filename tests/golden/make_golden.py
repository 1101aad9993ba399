"""Write stored expected values computed by the CPU oracle only.

  c2_pcg_iterations_<N>.txt     AMG-PCG iteration counts and final relative residuals
                                on the 3D 7-point Poisson problem at N^3 (b ~ U(-1,1),
                                seed 1002), box-aggregation hierarchy down to 4096 rows
                                or fewer, dense Cholesky coarsest solve, stop at
                                ||r|| <= 1e-8 ||b||, every smoother kind at degrees 1..6.
  aniso_pcg_iterations_<N>.txt  the same on the anisotropic 2D Q1 problem of Section 4
                                (eps = 100, theta = pi/6) with N x N elements; 2x2 box
                                aggregates; degrees given by --degrees.
  qdq_pcg_iterations.txt        CG preconditioned by the polynomial smoother alone on
                                A = Q D Q^T (Fig. better-than-optimal), b = A 1,
                                stop at ||r|| <= 1e-5 ||b||, N in {64, 256}, the three
                                spectra, every kind, degrees 1..8.  For each case the
                                count is also taken with b scaled by (1 + 2^-52) and by
                                (1 - 2^-53); min and max over the three runs measure how
                                far rounding alone moves the count.

Run from the repository root:
  python tests/golden/make_golden.py c2 [--size N]
  python tests/golden/make_golden.py aniso [--size N] [--kinds 0,1,2,3] [--degrees 1,2,3,4]
  python tests/golden/make_golden.py qdq
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import amg  # noqa: E402
from oracle import polynomials as P  # noqa: E402
from oracle import smoothers as S  # noqa: E402

KIND_COLS = "# columns: kind (0 l1-Jacobi, 1 4th kind, 2 optimal 4th kind, 3 optimal 1st kind), degree,"


def write(name, lines):
    out = os.path.join(HERE, name)
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(out)


def c2(size):
    A, b, _ = W.config_problem(2, size=size)
    As = A.to_scipy()
    t0 = time.time()
    H = amg.build_hierarchy(As, A.grid)
    lines = [f"# oracle AMG-PCG on 3D 7-point Poisson {size}^3, b = U(-1,1) seed {W.SEED_RHS + 2},",
             f"# levels {[lv.A.shape[0] for lv in H.levels]}, rtol 1e-8, x0 = 0.",
             KIND_COLS,
             "#          iterations, final relative residual ||r_k||/||b|| (recursive residual)"]
    for kind in (S.L1JAC, S.CHEB4, S.OPTCHEB4, S.OPTCHEB1):
        for k in range(1, 7):
            res, _ = amg.amg_pcg(As, b, A.grid, kind, k, H=H)
            lines.append(f"{kind} {k} {res.iters} {res.relres:.17e}")
            print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    write(f"c2_pcg_iterations_{size}.txt", lines)


def aniso(size, kinds, degrees):
    A, b = W.anisotropy2d_q1(size)
    As = A.to_scipy()
    t0 = time.time()
    H = amg.build_hierarchy(As, A.grid)
    lines = [f"# oracle AMG-PCG on the anisotropic 2D Q1 problem (eps = 100, theta = pi/6), {size} x {size}",
             f"# elements, grid {A.grid}, levels {[lv.A.shape[0] for lv in H.levels]}, rtol 1e-8, x0 = 0.",
             KIND_COLS,
             "#          iterations, final relative residual ||r_k||/||b|| (recursive residual)"]
    for kind in kinds:
        for k in degrees:
            res, _ = amg.amg_pcg(As, b, A.grid, kind, k, H=H)
            lines.append(f"{kind} {k} {res.iters} {res.relres:.17e}")
            print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    write(f"aniso_pcg_iterations_{size}.txt", lines)


def qdq():
    lines = ["# oracle CG preconditioned by the degree-k polynomial smoother alone (z = p_k(M^-1 A) M^-1 r)",
             "# on A = Q D Q^T, b = A 1, rtol 1e-5, x0 = 0, maxit 5000.",
             "# columns: spectrum, N, kind, degree, iterations, final relative residual, min and max",
             "#          iterations over b, b (1 + 2^-52), b (1 - 2^-53)"]
    t0 = time.time()
    for spectrum in ("equispaced", "clustered", "gap"):
        for N in (64, 256):
            A, b, _ = W.qdq_dense(N, spectrum)
            Ad = A.to_scipy().toarray()
            Minv = S.l1_diagonal(A.to_scipy())
            for kind in (S.L1JAC, S.CHEB4, S.OPTCHEB4, S.OPTCHEB1):
                for k in range(1, 9):
                    beta = P.optimal_beta(k)[0] if kind == S.OPTCHEB4 else None
                    a = P.a_star(k) if kind == S.OPTCHEB1 else None

                    def pre(r):
                        return S.smooth(Ad, Minv, r, None, kind, k, beta, a)
                    runs = [amg.pcg(Ad, b * s, pre, 1e-5, 5000) for s in (1.0, 1.0 + 2.0**-52, 1.0 - 2.0**-53)]
                    its = [r.iters for r in runs]
                    lines.append(f"{spectrum} {N} {kind} {k} {its[0]} {runs[0].relres:.17e} {min(its)} {max(its)}")
            print(spectrum, N, f"({time.time() - t0:.0f} s)", flush=True)
    write("qdq_pcg_iterations.txt", lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=("c2", "aniso", "qdq"))
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--kinds", default="0,1,2,3")
    ap.add_argument("--degrees", default="1,2,3,4")
    args = ap.parse_args()
    if args.what == "c2":
        c2(args.size or 128)
    elif args.what == "aniso":
        aniso(args.size or 256, [int(v) for v in args.kinds.split(",")], [int(v) for v in args.degrees.split(",")])
    else:
        qdq()


if __name__ == "__main__":
    main()
