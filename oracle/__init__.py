"""Plain, slow, FP64 CPU oracle for the polynomial-smoothed AMG-PCG path.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
this package; only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library: the only
shared module is ``workloads`` (seeded problem generators, no method
arithmetic).

Modules
-------
polynomials  constants of the three polynomial families (a*_k, Lambda_k,
             gamma_k, the optimal 4th-kind beta) and scalar evaluators.
smoothers    l1-Jacobi diagonal and the four smoothers, written as the
             recurrences of Section 2 (eqs. polsmoother, polsmootheropt,
             polsmootheropt1kind, Algorithm 1).
amg          box aggregation, Galerkin coarse operators, coarsest Cholesky,
             the V-cycle of eq. (amg) and (flexible) PCG.
adjoint      complex-step derivative of the V-cycle residual loss with
             respect to the polynomial weights beta.
mlp          the 8-64-64-6 tanh network, its gradient and Adam, in FP64.

Parity status: every function is pinned by a test against values the paper
prints, closed forms, special cases or brute force, except the FP32 path and
the learned-beta heuristic ("parity unpinned": there is no exact answer to
pin them to; they are bounded by properties instead).
"""
