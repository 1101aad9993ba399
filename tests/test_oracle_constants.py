"""Pins of the oracle's offline constants against what the paper prints and proves.

Sources: Fig. constantbounds / Fig. boundcomparison data (tests/golden/paper_constants.txt),
eq. (lottebound-4cheby), eq. (c1), the value at x = 1 (Section 2.3.2), Lemma 1,
Lemma 2 (with the interlacing roots of its proof, Appendix A), Theorem 1.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import polynomials as P

K15 = range(1, 16)


@pytest.mark.parametrize("k", K15)
def test_a_star_matches_printed(k, paper_constants):
    assert P.a_star(k) == pytest.approx(paper_constants["a_star"][k - 1], rel=1e-13)


@pytest.mark.parametrize("k", K15)
def test_lambda_matches_printed_and_equioscillates(k, paper_constants):
    a = P.a_star(k)
    lam = P.Lambda(k)
    assert lam == pytest.approx(paper_constants["lambda_cheb1"][k - 1], rel=1e-13)
    # at a*, the two branches of eq. (max2) are equal: 1/(2|c1|) = value at x = 1
    assert P.lambda_c1(k, a) == pytest.approx(P.lambda_at_one(k, a), rel=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_lambda_is_the_sup_of_f_for_tau(k):
    """Brute-force sup of x tau^2/(1-tau^2) with tau from mpmath's own Chebyshev T (no recurrence)."""
    a = mp.mpf(P.a_star(k))
    y0 = (1 + a) / (1 - a)
    tau = lambda x: mp.chebyt(k, (1 + a - 2 * x) / (1 - a)) / mp.chebyt(k, y0)
    assert P.gamma_of(tau, ngrid=2000) == pytest.approx(P.Lambda(k), rel=1e-10)


@pytest.mark.parametrize("k", range(1, 9))
def test_gamma_cheb4_closed_form(k, paper_constants):
    assert P.gamma_cheb4_closed(k) == pytest.approx(paper_constants["gamma_cheb4"][k - 1], rel=1e-14)
    # the sup of f for W_k(1-2x)/(2k+1), evaluated from the trigonometric definition of W
    def p(x):
        th = mp.acos(1 - 2 * x)
        if th == 0:
            return mp.mpf(1)
        return mp.sin((k + mp.mpf(1) / 2) * th) / mp.sin(th / 2) / (2 * k + 1)
    assert P.gamma_of(p, ngrid=2000) == pytest.approx(3.0 / (4 * k * (k + 1)), rel=1e-10)


def test_W_recurrence_matches_trig_definition():
    th = np.linspace(0.01, np.pi - 0.01, 101)
    for j in range(0, 16):
        assert np.allclose(P.cheb_W(j, np.cos(th)), P.cheb_W_trig(j, th), rtol=1e-12, atol=1e-12)
    # W_k(1) = 2k+1 so that p(0) = 1
    for j in range(0, 16):
        assert P.cheb_W(j, 1.0) == 2 * j + 1


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_optimal_beta_reproduces_printed_gamma(k, paper_constants):
    beta, gamma = P.optimal_beta(k)
    assert gamma == pytest.approx(paper_constants["gamma_optcheb4"][k - 1], rel=1e-13)
    # gamma of the polynomial rebuilt from beta by the W expansion (independent sup search)
    bb = [mp.mpf(1)] + [mp.mpf(v) for v in beta] + [mp.mpf(0)]
    def p(x):
        y = 1 - 2 * x
        return sum((bb[j] - bb[j + 1]) / (2 * j + 1) * P.cheb_W(j, y) for j in range(k + 1))
    assert P.gamma_of(p, ngrid=2000) == pytest.approx(gamma, rel=1e-10)
    # membership in Pi_k: p(0) = 1 and |p| <= 1 on [0, 1]
    xs = np.linspace(0, 1, 20001)
    pv = P.p_optcheb4(beta, xs)
    assert pv[0] == pytest.approx(1.0, abs=1e-14)
    assert np.abs(pv).max() <= 1.0 + 1e-14


@pytest.mark.parametrize("k", [7, 8, 10, 15])
def test_optimal_beta_high_degree(k, paper_constants):
    _, gamma = P.optimal_beta(k)
    assert gamma == pytest.approx(paper_constants["gamma_optcheb4"][k - 1], rel=2e-13)


def test_optimal_beta_special_cases():
    beta1, g1 = P.optimal_beta(1)
    assert g1 == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert beta1[0] == pytest.approx(9.0 / 8.0, rel=1e-15)
    _, g2 = P.optimal_beta(2)
    assert g2 == pytest.approx(1.0 - 2.0 / math.sqrt(5.0), rel=1e-14)


@pytest.mark.parametrize("k", range(2, 7))
def test_optimal_is_no_worse_than_either_family(k):
    _, g = P.optimal_beta(k)
    assert g < P.Lambda(k)
    assert g < P.gamma_cheb4_closed(k)


def test_first_kind_beats_fourth_kind_only_up_to_degree_4():
    wins = [k for k in range(1, 16) if P.Lambda(k) < P.gamma_cheb4_closed(k)]
    assert wins == [1, 2, 3, 4]


@pytest.mark.parametrize("k", range(3, 101))
def test_theorem1_bounds(k):
    a = P.a_star(k)
    lk = math.log(k)
    assert lk ** 2 / (9 * k * k) <= a <= lk ** 2 / (k * k)
    lam = P.lambda_c1(k, a)
    assert lk / (6 * k * k) <= lam <= 1.03 * lk / (2 * k * k)


@pytest.mark.parametrize("k", [1, 2, 4, 6, 9])
@pytest.mark.parametrize("afrac", [0.5, 1.0, 2.0])
def test_lemma1_f_positive_decreasing_on_0_a(k, afrac):
    a = min(0.9, afrac * P.a_star(k))
    x = np.linspace(a * 1e-3, a, 2000)
    t = P.tau_shifted(k, a, x)
    f = x * t * t / (1 - t * t)
    assert np.all(f > 0)
    assert np.all(np.diff(f) < 1e-15 * f[:-1])


@pytest.mark.parametrize("k", [2, 3, 5, 8, 12])
def test_lemma2_g_increasing_and_interlacing_roots(k):
    x = np.linspace(1e-6, 1 - 1e-6, 5000)
    assert np.all(np.diff(P.lemma2_g(k, x)) > 0)
    # roots of p(x) = sum C(2k,2j) x^j and q(x) = sum C(2k,2j+1) x^j (proof of Lemma 2)
    pc = [math.comb(2 * k, 2 * j) for j in range(k + 1)]
    qc = [math.comb(2 * k, 2 * j + 1) for j in range(k)]
    rp = np.sort(np.roots(pc[::-1]).real)[::-1]
    rq = np.sort(np.roots(qc[::-1]).real)[::-1]
    alpha = -np.tan((2 * np.arange(k) + 1) * np.pi / (4 * k)) ** 2
    delta = -np.tan(np.arange(1, k) * np.pi / (2 * k)) ** 2
    assert np.allclose(rp, np.sort(alpha)[::-1], rtol=1e-8)
    assert np.allclose(rq, np.sort(delta)[::-1], rtol=1e-8)
    inter = np.empty(2 * k - 1)
    inter[0::2] = np.sort(alpha)[::-1]
    inter[1::2] = np.sort(delta)[::-1]
    assert np.all(np.diff(inter) < 0) and inter[0] < 0


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_lambda_minimises_over_a(k):
    """a*_k minimises max(1/(2|c1|), value at 1) over a: nearby a are worse (Fig. minimax)."""
    a = P.a_star(k)
    obj = lambda aa: max(P.lambda_c1(k, aa), P.lambda_at_one(k, aa))
    for s in (0.85, 0.95, 1.05, 1.15):
        assert obj(s * a) > obj(a)
