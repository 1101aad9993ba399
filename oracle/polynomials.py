"""Polynomial families and their offline constants (oracle, test infrastructure only).

Everything here is matrix independent: it is the offline part of the method
(Section 2: "the optimization procedure can be carried out offline ... the
parameters ... are precomputed and tabulated").

Notation follows the paper:
  * Pi_k: polynomials of degree <= k with p(0) = 1 and |p| <= 1 on [0, 1] (eq. polspace).
  * f_p(x) = x p(x)^2 / (1 - p(x)^2); gamma(p) = sup_{0<x<=1} f_p(x) (Prop. 1, eq. prob1).
  * W_j: 4th-kind Chebyshev polynomial, W_j(cos t) = sin((j+1/2) t) / sin(t/2).
    The paper prints cos((k+1/2)t)/cos(t/2), which is the 3rd kind; the
    4th kind is the one that reproduces the recurrence (polsmoother) and the
    bound 3/(4k(k+1)) of eq. (lottebound-4cheby).
  * tau_k^{[a,1]}: scaled and shifted 1st-kind Chebyshev polynomial
    (Section 2.2, the display defining tau_k^{[a,b]} with b = 1).
  * a*_k: square of the root in (0,1) of eq. (optimalparameter).
"""
from __future__ import annotations

from functools import lru_cache
from math import comb

import mpmath as mp
import numpy as np
from scipy.optimize import brentq, linprog

# ---------------------------------------------------------------------------
# 1st kind (Sections 2.2 and 2.3)
# ---------------------------------------------------------------------------


def cheb_T(k: int, t):
    """1st-kind Chebyshev polynomial T_k(t) by its trigonometric/hyperbolic closed form
    (property (i) of Section 2.3.1), valid for any real t."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(k * np.arccos(t[inside]))
    big = t > 1.0
    out[big] = np.cosh(k * np.arccosh(t[big]))
    small = t < -1.0
    out[small] = (-1.0) ** k * np.cosh(k * np.arccosh(-t[small]))
    return out


def tau_shifted(k: int, a: float, x):
    """tau_k^{[a,1]}(x) = T_k((1+a-2x)/(1-a)) / T_k((1+a)/(1-a)) (Section 2.2, b = 1)."""
    x = np.asarray(x, dtype=np.float64)
    y0 = (1.0 + a) / (1.0 - a)
    return cheb_T(k, (1.0 + a - 2.0 * x) / (1.0 - a)) / cheb_T(k, np.array([y0]))[0]


def optimal_parameter_poly(k: int, x):
    """phi(x) = 8k(1-x^2)^{2k} + x[(1-x)^{4k} - (1+x)^{4k}] (eq. optimalparameter)."""
    return 8 * k * (1 - x * x) ** (2 * k) + x * ((1 - x) ** (4 * k) - (1 + x) ** (4 * k))


@lru_cache(maxsize=None)
def a_star(k: int) -> float:
    """a*_k: the square of the unique root in (0,1) of eq. (optimalparameter).

    Located with Brent's method (the paper uses MATLAB fzero, a Brent variant)
    and polished with a 40-digit Newton step in mpmath.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    r = brentq(lambda x: optimal_parameter_poly(k, x), 1e-12, 1.0 - 1e-15, xtol=1e-300, rtol=8.9e-16,
               maxiter=500)
    with mp.workdps(40):
        phi = lambda x: 8 * k * (1 - x * x) ** (2 * k) + x * ((1 - x) ** (4 * k) - (1 + x) ** (4 * k))
        r = mp.mpf(r)
        for _ in range(6):  # Newton polish from Brent's bracketed root
            r = r - phi(r) / mp.diff(phi, r)
        return float(r * r)


def lambda_c1(k: int, a: float) -> float:
    """1/(2|c_1^{(a,k)}|) in the binomial-sum form derived from eq. (c1) (Section 2.3.2)."""
    num = sum(comb(2 * k, 2 * j) * a ** j for j in range(k + 1))
    den = 2 * k * sum(comb(2 * k, 2 * j + 1) * a ** j for j in range(k))
    return num / den


def lambda_at_one(k: int, a: float) -> float:
    """x tau^2/(1-tau^2) at x = 1 in closed form (Section 2.3.2, the value at x = 1)."""
    s = np.sqrt(a)
    u = ((1 + s) / (1 - s)) ** k + ((1 - s) / (1 + s)) ** k
    return 4.0 / (u * u - 4.0)


def Lambda(k: int) -> float:
    """Lambda_k of eq. (lambdak): the minimax value over the 1st-kind family, attained at a*_k."""
    return lambda_c1(k, a_star(k))


def lemma2_g(k: int, x):
    """g(x) of Lemma 2 (the binomial ratio), increasing on (0, 1)."""
    x = np.asarray(x, dtype=np.float64)
    num = sum(comb(2 * k, 2 * j) * x ** j for j in range(k + 1))
    den = 2 * k * sum(comb(2 * k, 2 * j + 1) * x ** j for j in range(k))
    return num / den


# ---------------------------------------------------------------------------
# 4th kind (Section 2.1)
# ---------------------------------------------------------------------------


def cheb_W(j: int, y):
    """4th-kind Chebyshev W_j(y) by the three-term recurrence W_0 = 1, W_1 = 2y+1,
    W_{j+1} = 2y W_j - W_{j-1} (works for real or mpmath/complex scalars and arrays)."""
    w_prev, w = 1.0 + 0.0 * y, 2.0 * y + 1.0
    if j == 0:
        return w_prev
    for _ in range(1, j):
        w_prev, w = w, 2.0 * y * w - w_prev
    return w


def cheb_W_trig(j: int, theta):
    """W_j(cos t) = sin((j + 1/2) t) / sin(t / 2): the defining closed form (independent of the recurrence)."""
    theta = np.asarray(theta, dtype=np.float64)
    return np.sin((j + 0.5) * theta) / np.sin(0.5 * theta)


def p_cheb4(k: int, x):
    """Error polynomial of the 4th-kind smoother (polsmoother): W_k(1-2x)/(2k+1)."""
    return cheb_W(k, 1.0 - 2.0 * np.asarray(x, dtype=np.float64)) / (2 * k + 1)


def p_optcheb4(beta, x):
    """p_k(x) = sum_{j=0}^k (beta_j - beta_{j+1})/(2j+1) W_j(1-2x), beta_0 = 1, beta_{k+1} = 0
    (Section 2.1, the expansion preceding eq. polsmootheropt).  ``beta`` = (beta_1..beta_k)."""
    b = [1.0] + [float(v) for v in beta] + [0.0]
    y = 1.0 - 2.0 * np.asarray(x, dtype=np.float64)
    return sum((b[j] - b[j + 1]) / (2 * j + 1) * cheb_W(j, y) for j in range(len(beta) + 1))


def p_l1jacobi(k: int, x):
    """Error polynomial of k plain l1-Jacobi sweeps: (1-x)^k."""
    return (1.0 - np.asarray(x, dtype=np.float64)) ** k


def p_cheb1(k: int, x):
    """Error polynomial of the optimal 1st-kind smoother: tau_k^{[a*_k,1]}(x)."""
    return tau_shifted(k, a_star(k), x)


# ---------------------------------------------------------------------------
# The bound constant gamma(p) = sup_{0<x<=1} x p^2/(1-p^2)  (Prop. 1, eq. prob1)
# ---------------------------------------------------------------------------


def gamma_of(poly_mp, dps: int = 40, ngrid: int = 4000) -> float:
    """sup over (0,1] of x p(x)^2/(1-p(x)^2) for a polynomial given as an mpmath callable.

    The limit at 0+ equals 1/(2|p'(0)|) (f = p^2/(q(1+p)) with q = (1-p)/x).
    Interior maxima are bracketed on a grid (geometric near 0, uniform
    elsewhere) and refined by golden-section search, all in ``dps`` digits.
    """
    with mp.workdps(dps):
        def f(x):
            p = poly_mp(x)
            return x * p * p / (1 - p * p)
        f0 = 1 / (2 * abs(mp.diff(poly_mp, 0)))
        xs = sorted(set([mp.mpf(v) for v in np.geomspace(1e-9, 1e-2, ngrid // 4)]
                        + [mp.mpf(v) for v in np.linspace(1e-2, 1.0, 3 * ngrid // 4)]))
        fs = [f(x) for x in xs]
        best = max(f0, fs[-1])
        for i in range(1, len(xs) - 1):
            if fs[i] >= fs[i - 1] and fs[i] >= fs[i + 1]:
                lo, hi = xs[i - 1], xs[i + 1]
                g = (mp.sqrt(5) - 1) / 2
                c, d = hi - g * (hi - lo), lo + g * (hi - lo)
                fc, fd = f(c), f(d)
                for _ in range(120):
                    if fc > fd:
                        hi, d, fd = d, c, fc
                        c = hi - g * (hi - lo)
                        fc = f(c)
                    else:
                        lo, c, fc = c, d, fd
                        d = lo + g * (hi - lo)
                        fd = f(d)
                best = max(best, fc, fd)
        return float(best)


def gamma_cheb4_closed(k: int) -> float:
    """Closed form of gamma for the 4th kind: 3/(4k(k+1)) (eq. lottebound-4cheby)."""
    return 3.0 / (4.0 * k * (k + 1))


# ---------------------------------------------------------------------------
# Optimal 4th-kind weights beta_{j,k} (Section 2.1, eqs. prob1 and polsmootheropt)
# ---------------------------------------------------------------------------


def _lp_minimax(k: int, iters: int = 60):
    """Discretised eq. (prob1) as a sequence of LP feasibility problems (bisection on gamma).

    For a fixed gamma, f_p <= gamma on (0,1] is equivalent to
    |p(x)| <= sqrt(gamma/(x+gamma)) there, plus p'(0) <= -1/(2 gamma) for the
    limit at 0+.  p is written as sum_m a_m T_m(1-2x) with sum_m a_m = 1
    (p(0) = 1).  Returns (gamma, a) on the grid.
    """
    xs = np.unique(np.concatenate([np.geomspace(1e-5, 1e-2, 400), np.linspace(1e-2, 1.0, 3000)]))
    y = 1.0 - 2.0 * xs
    T = np.stack([cheb_T(m, y) for m in range(k + 1)], axis=1)
    slope = np.array([-2.0 * m * m for m in range(k + 1)])  # d/dx T_m(1-2x) at x = 0
    A_eq = np.ones((1, k + 1))
    b_eq = np.array([1.0])

    def feasible(g):
        s = np.sqrt(g / (xs + g))
        A_ub = np.vstack([T, -T, slope[None, :]])
        b_ub = np.concatenate([s, s, [-1.0 / (2.0 * g)]])
        res = linprog(np.zeros(k + 1), A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                      bounds=[(None, None)] * (k + 1), method="highs")
        return res.status == 0, (res.x if res.status == 0 else None)

    lo, hi = 0.0, gamma_cheb4_closed(k) * 1.01
    ok, a_hi = feasible(hi)
    assert ok
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ok, a = feasible(mid)
        if ok:
            hi, a_hi = mid, a
        else:
            lo = mid
    return hi, a_hi


def _cheb_basis_to_mp(a):
    a = [mp.mpf(float(v)) for v in a]

    def p(x):
        y = 1 - 2 * x
        # Clenshaw-free: T_m via cos/cosh closed form in mpmath
        tot = mp.mpf(0)
        for m, am in enumerate(a):
            tot += am * mp.chebyt(m, y)
        return tot
    return p


@lru_cache(maxsize=None)
def optimal_beta(k: int, dps: int = 40):
    """beta_{1..k,k} of the optimal 4th-kind smoother, and its gamma.

    1. Solve the discretised minimax (eq. prob1) by LP bisection.
    2. Polish with Newton on the equi-oscillation conditions (the approach the
       paper attributes to Lottes): f_p = gamma at 0+, at x = 1 and at k-1
       interior points where also f_p' = 0.  Unknowns: the k free coefficients,
       gamma and the k-1 interior points.
    3. Expand p in the basis W_j(1-2x)/(2j+1) and sum the coefficients from
       the top to obtain beta_j (so that beta_0 = 1, beta_{k+1} = 0).
    Returns (beta tuple of floats, gamma float).
    """
    g_lp, a_lp = _lp_minimax(k)
    p_lp = _cheb_basis_to_mp(a_lp)
    with mp.workdps(dps):
        # monomial coefficients c_1..c_k of p = 1 + sum c_m x^m from the LP polynomial
        xs_fit = [mp.mpf(i + 1) / (k + 1) for i in range(k)]
        M = mp.matrix([[x ** m for m in range(1, k + 1)] for x in xs_fit])
        rhs = mp.matrix([p_lp(x) - 1 for x in xs_fit])
        c0 = mp.lu_solve(M, rhs)

        def pm(c, x):
            return 1 + sum(c[m - 1] * x ** m for m in range(1, k + 1))

        def fm(c, x):
            p = pm(c, x)
            return x * p * p / (1 - p * p)

        def dfm(c, x):
            p = pm(c, x)
            dp = sum(m * c[m - 1] * x ** (m - 1) for m in range(1, k + 1))
            num = x * p * p
            den = 1 - p * p
            dnum = p * p + 2 * x * p * dp
            dden = -2 * p * dp
            return (dnum * den - num * dden) / (den * den)

        # interior maxima of f for the LP polynomial (located in double precision)
        grid = np.linspace(1e-4, 1.0, 20001)
        pg = sum(float(am) * cheb_T(m, 1.0 - 2.0 * grid) for m, am in enumerate(a_lp))
        fv = grid * pg * pg / (1.0 - pg * pg)
        xi = [mp.mpf(grid[i]) for i in range(1, len(grid) - 1) if fv[i] >= fv[i - 1] and fv[i] >= fv[i + 1]]
        if len(xi) != k - 1:
            raise RuntimeError(f"k={k}: expected {k-1} interior maxima, found {len(xi)}")

        def F(*u):
            c = u[:k]
            g = u[k]
            xi_ = u[k + 1:]
            eqs = [1 / (-2 * c[0]) - g, fm(c, mp.mpf(1)) - g]
            for x in xi_:
                eqs.append(fm(c, x) - g)
                eqs.append(dfm(c, x))
            return eqs

        u0 = list(c0) + [mp.mpf(g_lp)] + xi
        sol = mp.findroot(F, u0, tol=mp.mpf(10) ** (-(dps - 8)), maxsteps=200)
        sol = [sol[i] for i in range(len(u0))]
        c = sol[:k]
        gamma = sol[k]

        # expansion in W_j(1-2x)/(2j+1): match values at k+1 nodes
        nodes = [mp.cos(mp.pi * (2 * i + 1) / (2 * (k + 1))) * mp.mpf(0.5) + mp.mpf(0.5) for i in range(k + 1)]
        B = mp.matrix([[cheb_W(j, 1 - 2 * x) / (2 * j + 1) for j in range(k + 1)] for x in nodes])
        vals = mp.matrix([pm(c, x) for x in nodes])
        d = mp.lu_solve(B, vals)
        beta = [sum(d[i] for i in range(j, k + 1)) for j in range(k + 1)]
        if abs(beta[0] - 1) > mp.mpf(10) ** (-(dps - 10)):
            raise RuntimeError("beta_0 != 1")
        return tuple(float(b) for b in beta[1:]), float(gamma)


def beta_table(kmax: int = 6):
    """{k: (beta_1..beta_k)} for k = 1..kmax."""
    return {k: optimal_beta(k)[0] for k in range(1, kmax + 1)}
