"""Write stored expected values computed by the CPU oracle only.

  c2_pcg_iterations.txt  AMG-PCG iteration counts and final relative residuals
                         on the 3D 7-point Poisson problem at 128^3 (b ~ U(-1,1),
                         seed 1002), box-aggregation hierarchy down to 16^3, dense
                         Cholesky coarsest solve, stop at ||r|| <= 1e-8 ||b||,
                         every smoother kind at degrees 1..6.

Run from the repository root:  python tests/golden/make_golden.py [--size N]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import amg  # noqa: E402
from oracle import smoothers as S  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=128)
    args = ap.parse_args()
    A, b, _ = W.config_problem(2, size=args.size)
    As = A.to_scipy()
    t0 = time.time()
    H = amg.build_hierarchy(As, A.grid)
    lines = [f"# oracle AMG-PCG on 3D 7-point Poisson {args.size}^3, b = U(-1,1) seed {W.SEED_RHS + 2},",
             f"# levels {[lv.A.shape[0] for lv in H.levels]}, rtol 1e-8, x0 = 0.",
             "# columns: kind (0 l1-Jacobi, 1 4th kind, 2 optimal 4th kind, 3 optimal 1st kind), degree,",
             "#          iterations, final relative residual ||r_k||/||b|| (recursive residual)"]
    for kind in (S.L1JAC, S.CHEB4, S.OPTCHEB4, S.OPTCHEB1):
        for k in range(1, 7):
            res, _ = amg.amg_pcg(As, b, A.grid, kind, k, H=H)
            lines.append(f"{kind} {k} {res.iters} {res.relres:.17e}")
            print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(HERE, f"c2_pcg_iterations_{args.size}.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(out)


if __name__ == "__main__":
    main()
