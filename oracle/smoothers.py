"""The l1-Jacobi basic smoother and its three polynomial accelerations (oracle).

TEST INFRASTRUCTURE ONLY.  Plain vector recurrences on a scipy.sparse CSR
matrix, in the order and notation of Section 2.  Vectors may be real or
complex (the complex-step gradient runs these same functions).

Kinds (the integer codes match the library's public enum):
  0 L1JAC     k sweeps of x <- x + M^{-1}(b - A x)            (eq. l1smooth)
  1 CHEB4     4th-kind Chebyshev recurrence                   (eq. polsmoother)
  2 OPTCHEB4  the same with x^{(j)} = x^{(j-1)} + beta_j z^{(j)} (eq. polsmootheropt)
  3 OPTCHEB1  1st-kind Chebyshev on [a, 1]                    (eq. polsmootheropt1kind, Algorithm 1)

The spectral scale rho(M^{-1}A) is replaced by 1: for the l1-Jacobi M the
spectrum of M^{-1}A lies in (0, 1] (comments of Algorithm 1).
"""
from __future__ import annotations

import numpy as np

L1JAC, CHEB4, OPTCHEB4, OPTCHEB1 = 0, 1, 2, 3
KIND_NAMES = {L1JAC: "l1jacobi", CHEB4: "cheb4", OPTCHEB4: "optcheb4", OPTCHEB1: "optcheb1"}


def l1_diagonal(A) -> np.ndarray:
    """M_i = a_ii + sum_{j != i} |a_ij| (eq. l1smooth); returns 1/M_i (applied by multiplication)."""
    A = A.tocsr()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    diag_mask = A.indices == rows
    M = np.zeros(n)
    np.add.at(M, rows[diag_mask], A.data[diag_mask])
    np.add.at(M, rows[~diag_mask], np.abs(A.data[~diag_mask]))
    return 1.0 / M


def smooth_l1jacobi(A, Minv, b, x0, k):
    """k sweeps x <- x + M^{-1}(b - A x); x0=None means x0 = 0."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    for _ in range(k):
        x = x + Minv * (b - A @ x)
    return x


def smooth_cheb4(A, Minv, b, x0, k, beta=None):
    """4th-kind recurrence (eq. polsmoother); with ``beta`` the optimal variant (eq. polsmootheropt).

    z^{(0)} = 0, r^{(0)} = b - A x^{(0)};  for j = 1..k:
      z^{(j)} = (2j-3)/(2j+1) z^{(j-1)} + (8j-4)/(2j+1) M^{-1} r^{(j-1)}
      x^{(j)} = x^{(j-1)} + beta_j z^{(j)}          (beta_j = 1 for the plain 4th kind)
      r^{(j)} = r^{(j-1)} - A z^{(j)}               (not needed after the last step)
    The residual is always updated with the unweighted z.
    """
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - A @ x
    z = np.zeros_like(b)
    for j in range(1, k + 1):
        z = (2 * j - 3) / (2 * j + 1) * z + (8 * j - 4) / (2 * j + 1) * (Minv * r)
        w = 1.0 if beta is None else beta[j - 1]
        x = x + w * z
        if j < k:
            r = r - A @ z
    return x


def smooth_cheb1(A, Minv, b, x0, k, a):
    """1st-kind Chebyshev acceleration on [a, 1] (Algorithm 1; eq. polsmootheropt1kind).

    theta = (1+a)/2, delta = (1-a)/2, sigma_1 = theta/delta, rho_0 = 1/sigma_1
    r^{(0)} = M^{-1}(b - A x^{(0)}), d^{(0)} = r^{(0)}/theta, x^{(1)} = x^{(0)} + d^{(0)}
    for j = 1..k-1:
      s^{(j)} = M^{-1} A d^{(j-1)};  rho_j = 1/(2 sigma_1 - rho_{j-1})
      r^{(j)} = r^{(j-1)} - s^{(j)}
      d^{(j)} = rho_j rho_{j-1} d^{(j-1)} + (2 rho_j/delta) r^{(j)}
      x^{(j+1)} = x^{(j)} + d^{(j)}
    """
    theta = (1.0 + a) / 2.0
    delta = (1.0 - a) / 2.0
    if x0 is None:
        x = np.zeros_like(b)
        r = Minv * b
    else:
        x = x0.copy()
        r = Minv * (b - A @ x)
    sigma1 = theta / delta
    rho_prev = 1.0 / sigma1
    d = r / theta
    x = x + d
    for _ in range(1, k):
        s = Minv * (A @ d)
        rho = 1.0 / (2.0 * sigma1 - rho_prev)
        r = r - s
        d = rho * rho_prev * d + (2.0 * rho / delta) * r
        x = x + d
        rho_prev = rho
    return x


def smooth(A, Minv, b, x0, kind, k, beta=None, a=None):
    """Dispatch on ``kind``.  ``beta`` (OPTCHEB4) and ``a`` (OPTCHEB1) are the tabulated constants."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if kind == L1JAC:
        return smooth_l1jacobi(A, Minv, b, x0, k)
    if kind == CHEB4:
        return smooth_cheb4(A, Minv, b, x0, k, None)
    if kind == OPTCHEB4:
        if beta is None or len(beta) != k:
            raise ValueError("OPTCHEB4 needs k weights")
        return smooth_cheb4(A, Minv, b, x0, k, beta)
    if kind == OPTCHEB1:
        if a is None:
            raise ValueError("OPTCHEB1 needs the interval end a")
        return smooth_cheb1(A, Minv, b, x0, k, a)
    raise ValueError(f"unknown kind {kind}")


def error_polynomial(kind, k, beta=None, a=None):
    """The scalar polynomial p with e_out = p(M^{-1}A) e_in for each kind (closed forms, not recurrences)."""
    from . import polynomials as P

    if kind == L1JAC:
        return lambda x: P.p_l1jacobi(k, x)
    if kind == CHEB4:
        return lambda x: P.p_cheb4(k, x)
    if kind == OPTCHEB4:
        return lambda x: P.p_optcheb4(beta, x)
    if kind == OPTCHEB1:
        return lambda x: P.tau_shifted(k, a, x)
    raise ValueError(kind)
