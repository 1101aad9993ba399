"""Offline generator of the library's tabulated polynomial constants.

Writes ``csrc/coeffs.inc`` (hex-float literals) with, for degrees k = 1..KMAX:
  * a*_k, the left end of the optimal 1st-kind interval: the square of the
    root in (0,1) of 8k(1-s^2)^{2k} + s[(1-s)^{4k} - (1+s)^{4k}] = 0
    (eq. optimalparameter), found here by plain bisection in 60-digit arithmetic;
  * beta_{1..k,k}, the weights of the optimal 4th-kind smoother
    (eq. polsmootheropt): the minimiser of sup_{0<x<=1} x p^2/(1-p^2) over
    p(0) = 1 (eq. prob1), found by a Remez-style exchange: alternate between
    (i) solving for the polynomial whose objective takes one common value at
    the current reference set {0+, k-1 interior points, 1}, and (ii) moving the
    interior points to the local maxima of the new objective; then expanded in
    the basis W_j(1-2x)/(2j+1) (W the 4th-kind Chebyshev polynomials) by
    back-substitution on the leading coefficients, beta_j being the tail sums.

The paper computes these constants offline and tabulates them (Section 2,
after eq. prob1); so does this library.  Run ``python -m
paper_2407_09848_amd.gen_coeffs`` to regenerate the include file.
"""
from __future__ import annotations

import os

import mpmath as mp

KMAX = 12
DPS = 60


def _astar(k: int) -> mp.mpf:
    phi = lambda s: 8 * k * (1 - s * s) ** (2 * k) + s * ((1 - s) ** (4 * k) - (1 + s) ** (4 * k))
    lo, hi = mp.mpf(0), mp.mpf(1)  # phi(0) = 8k > 0, phi(1) = -2^{4k} < 0
    for _ in range(220):
        mid = (lo + hi) / 2
        if phi(mid) > 0:
            lo = mid
        else:
            hi = mid
    s = (lo + hi) / 2
    return s * s


def _w_monomial(j: int):
    """Monomial coefficients (in x, ascending) of W_j(1-2x) via W_{j+1} = 2y W_j - W_{j-1}."""
    y = [mp.mpf(1), mp.mpf(-2)]  # 1 - 2x

    def mul(a, b):
        out = [mp.mpf(0)] * (len(a) + len(b) - 1)
        for i, ai in enumerate(a):
            for l, bl in enumerate(b):
                out[i + l] += ai * bl
        return out

    def add(a, b, sb=1):
        n = max(len(a), len(b))
        a = a + [mp.mpf(0)] * (n - len(a))
        b = b + [mp.mpf(0)] * (n - len(b))
        return [u + sb * v for u, v in zip(a, b)]

    w0 = [mp.mpf(1)]
    w1 = add([2 * c for c in y], [mp.mpf(1)])
    if j == 0:
        return w0
    for _ in range(1, j):
        w0, w1 = w1, add(mul([2 * c for c in y], w1), w0, -1)
    return w1


def _poly(c, x):
    """p(x) = 1 + sum_{m>=1} c[m-1] x^m (Horner)."""
    acc = mp.mpf(0)
    for cm in reversed(c):
        acc = acc * x + cm
    return 1 + acc * x


def _obj(c, x):
    p = _poly(c, x)
    return x * p * p / (1 - p * p)


def _local_maxima(c, k):
    xs = [mp.mpf(i) / 8000 for i in range(1, 8000)]
    fs = [_obj(c, x) for x in xs]
    pts = []
    for i in range(1, len(xs) - 1):
        if fs[i] >= fs[i - 1] and fs[i] > fs[i + 1]:
            # golden-section refinement on [x_{i-1}, x_{i+1}]
            lo, hi = xs[i - 1], xs[i + 1]
            g = (mp.sqrt(5) - 1) / 2
            for _ in range(200):
                a, b = hi - g * (hi - lo), lo + g * (hi - lo)
                if _obj(c, a) > _obj(c, b):
                    hi = b
                else:
                    lo = a
            pts.append((lo + hi) / 2)
    return pts


def _optimal_beta(k: int):
    if k == 1:
        # one free coefficient: 1/(2|c1|) = f(1) gives c1 = -3/2, beta_1 = 9/8
        c = [mp.mpf(-3) / 2]
        ref = []
    else:
        # start from the 4th-kind polynomial W_k(1-2x)/(2k+1)
        w = _w_monomial(k)
        c = [wi / (2 * k + 1) for wi in w[1:]]
        ref = _local_maxima(c, k)
        assert len(ref) == k - 1, (k, len(ref))
        for _ in range(60):
            def F(*u):
                cc = list(u[:k])
                E = u[k]
                eqs = [1 / (-2 * cc[0]) - E, _obj(cc, mp.mpf(1)) - E]
                eqs += [_obj(cc, x) - E for x in ref]
                return eqs
            E0 = max([1 / (-2 * c[0]), _obj(c, mp.mpf(1))] + [_obj(c, x) for x in ref])
            u = mp.findroot(F, c + [E0], tol=mp.mpf(10) ** (-DPS + 10), maxsteps=100)
            c = [u[i] for i in range(k)]
            new_ref = _local_maxima(c, k)
            assert len(new_ref) == k - 1
            moved = max(abs(a - b) for a, b in zip(new_ref, ref))
            ref = new_ref
            vals = [1 / (-2 * c[0]), _obj(c, mp.mpf(1))] + [_obj(c, x) for x in ref]
            if moved < mp.mpf(10) ** (-25) and (max(vals) - min(vals)) < mp.mpf(10) ** (-40):
                break
        else:
            raise RuntimeError(f"exchange did not converge for k={k}")
    gamma = max([1 / (-2 * c[0]), _obj(c, mp.mpf(1))] + [_obj(c, x) for x in ref])
    # expansion in W_j(1-2x)/(2j+1): back-substitute from the leading coefficient
    coef = [mp.mpf(1)] + list(c)
    d = [mp.mpf(0)] * (k + 1)
    for j in range(k, -1, -1):
        wj = [v / (2 * j + 1) for v in _w_monomial(j)]
        d[j] = coef[j] / wj[j]
        for m in range(j + 1):
            coef[m] -= d[j] * wj[m]
    beta = [sum(d[j:]) for j in range(k + 1)]
    assert abs(beta[0] - 1) < mp.mpf(10) ** (-40)
    return [beta[j] for j in range(1, k + 1)], gamma


def generate(path: str | None = None) -> str:
    mp.mp.dps = DPS
    lines = ["// Generated by paper_2407_09848_amd/gen_coeffs.py -- do not edit.",
             "// Tabulated constants of the polynomial smoothers, degrees 1..%d." % KMAX,
             "#pragma once",
             "#define AMGP_KMAX %d" % KMAX,
             "// a*_k: left end of the optimal 1st-kind interval [a*_k, 1] (eq. optimalparameter).",
             "static const double kAStar[AMGP_KMAX + 1] = {0.0,"]
    for k in range(1, KMAX + 1):
        lines.append("  %s, // k=%d  %s" % (float(_astar(k)).hex(), k, mp.nstr(_astar(k), 17)))
    lines.append("};")
    lines.append("// beta_{j,k}, j = 1..k, of the optimal 4th-kind smoother (eq. polsmootheropt); row k.")
    lines.append("static const double kOptBeta[AMGP_KMAX + 1][AMGP_KMAX] = {{0.0},")
    gam = []
    for k in range(1, KMAX + 1):
        beta, g = _optimal_beta(k)
        gam.append(g)
        lines.append("  {" + ", ".join(float(b).hex() for b in beta) + "}, // k=%d" % k)
    lines.append("};")
    lines.append("// gamma_k of the optimal 4th-kind polynomial (for reference and tests).")
    lines.append("static const double kOptGamma[AMGP_KMAX + 1] = {0.0,")
    for k, g in enumerate(gam, 1):
        lines.append("  %s, // k=%d  %s" % (float(g).hex(), k, mp.nstr(g, 17)))
    lines.append("};")
    text = "\n".join(lines) + "\n"
    if path is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "coeffs.inc")
    with open(path, "w") as fh:
        fh.write(text)
    return path


if __name__ == "__main__":
    print(generate())
