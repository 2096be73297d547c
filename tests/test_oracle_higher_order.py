"""Pins of the higher-order fixed-mu schemes in the CPU oracle (no GPU).

The scheme: f_i(X) = P_{m,m}(alpha (X - I/2) + I/2) with m odd and alpha >= 1 the root of
Eq. 3 (the generalisation of Algorithm 1 stated with Eqs. 2 and 3); alpha = 1 is the unscaled
grand-canonical P_{m,m} iteration.  Pinned against: the binomial (incomplete-beta) closed form
of P_{i,j} and its derivative, the closed-form alpha of Algorithm 1 (m = 1), an independent
root of Eq. 3 by Brent's method on the binomial form, a brute-force check that alpha is the
largest scaling that keeps the folded interval below the gap edge, the exact projector, and
the spectral oracle.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import dense, exact, polynomials as poly, schedule as sch, spectral
from paper_1101_0265_amd import hamiltonians as H

HO = ("snf_fixmu3", "snf_fixmu5", "pmm3", "pmm5")


def _binomial_form(i, j):
    """P_{i,j}(x) = x^{i+1} sum_{k=0}^{j} C(i+k, k) (1-x)^k, expanded exactly."""
    coef = [Fraction(0)] * (i + j + 2)
    for k in range(j + 1):
        ck = math.comb(i + k, k)
        for t in range(k + 1):             # (1-x)^k = sum_t C(k,t) (-x)^t
            coef[i + 1 + t] += Fraction(ck * math.comb(k, t) * (-1) ** t)
    return coef


def _eval_binomial(i, j, x):
    return sum(math.comb(i + k, k) * (1.0 - x) ** k for k in range(j + 1)) * x ** (i + 1)


@pytest.mark.parametrize("i,j", [(0, 1), (1, 0), (1, 1), (1, 3), (3, 1), (3, 3), (5, 5),
                                 (2, 4)])
def test_exact_coefficients_match_binomial_form(i, j):
    assert poly.p_ij_exact(i, j) == _binomial_form(i, j)


@pytest.mark.parametrize("m", [1, 3, 5])
def test_exact_pmm_derivative_and_symmetry(m):
    c = poly.p_ij_exact(m, m)
    d = [k * c[k] for k in range(1, len(c))]            # P'
    cm = Fraction(math.factorial(2 * m + 1), math.factorial(m) ** 2)
    want = [Fraction(0)] * (2 * m + 1)                  # cm x^m (1-x)^m
    for t in range(m + 1):
        want[m + t] += cm * math.comb(m, t) * (-1) ** t
    assert d == want
    # P(1 - x) = 1 - P(x): compare at rational points exactly
    for x in (Fraction(1, 7), Fraction(2, 5), Fraction(-3, 4), Fraction(9, 8)):
        p = sum(ck * x ** k for k, ck in enumerate(c))
        q = sum(ck * (1 - x) ** k for k, ck in enumerate(c))
        assert p + q == 1


@pytest.mark.parametrize("m", [1, 3])
def test_exact_equals_float_definition(m):
    a = np.array([float(v) for v in poly.p_ij_exact(m, m)])
    b = poly.p_ij_coefficients(m, m)
    assert np.allclose(a, b, rtol=0, atol=1e-9 * np.max(np.abs(a)))


@pytest.mark.parametrize("beta", [1e-9, 1e-4, 0.01, 0.1, 0.3, 0.45, 0.49, 0.4999])
def test_alpha_m1_equals_algorithm1(beta):
    assert abs(sch.pmm_alpha(1, beta) - sch.alg1_alpha(beta)) <= 4e-15 * sch.alg1_alpha(beta)


@pytest.mark.parametrize("m", [3, 5])
@pytest.mark.parametrize("beta", [1e-6, 1e-3, 0.05, 0.2, 0.4, 0.49, 0.49975])
def test_alpha_solves_eq3_independently(m, beta):
    a = sch.pmm_alpha(m, beta)

    def g(al):     # Eq. 3 with P from the binomial form, not the oracle's coefficients
        return (_eval_binomial(m, m, 0.5 * (1 - al))
                - _eval_binomial(m, m, al * (beta - 0.5) + 0.5))

    ref = brentq(g, 1.0, 1.0 / (1.0 - 2.0 * beta), xtol=1e-15, rtol=1e-15, maxiter=500)
    assert abs(a - ref) <= 1e-12 * ref
    assert a >= 1.0


@pytest.mark.parametrize("m", [1, 3, 5])
@pytest.mark.parametrize("beta", [0.01, 0.2, 0.45])
def test_alpha_is_the_largest_scaling_that_keeps_the_gap(m, beta):
    """Brute force over the occupied-side interval [0, beta] (its mirror follows by symmetry):
    with alpha from Eq. 3 the largest image is that of the gap edge; any larger alpha folds
    the far end above it, so the gap would shrink."""
    xs = np.linspace(0.0, beta, 20001)

    def images(al):
        return poly.pmm(m, al * (xs - 0.5) + 0.5)

    a = sch.pmm_alpha(m, beta)
    y = images(a)
    edge = poly.pmm(m, a * (beta - 0.5) + 0.5)
    assert np.all(y >= -1e-15)
    assert np.max(y) <= edge * (1 + 1e-10) + 1e-300
    y2 = images(a * (1 + 1e-4))
    edge2 = poly.pmm(m, a * (1 + 1e-4) * (beta - 0.5) + 0.5)
    assert np.max(y2) > edge2 * (1 + 1e-8)
    # and the new beta is below the unscaled one: scaling helps
    assert sch.pmm_beta_next(m, beta, a) < sch.pmm_beta_next(m, beta, 1.0)


@pytest.mark.parametrize("scheme", HO)
def test_dense_reaches_exact_projector(scheme):
    h = H.random_spectrum_hamiltonian(48, 21, -1.0, 0.08, 0.12, 1.1, seed=11)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ,
              mu=0.1, xi=0.04, tol=1e-11, max_iter=100)
    r = dense.purify(h.F, scheme, **kw)
    assert r["status"] == "ok"
    D_ref = exact.projector(F=h.F, n_occ=h.n_occ)
    assert np.linalg.norm(r["D"] - D_ref) < 1e-9
    m = sch.HIGHER_ORDER[scheme][0]
    assert r["products"] == (m + 1) * r["iterations"] + 1
    assert set(r["branches"]) == {sch.PMM[m]}


@pytest.mark.parametrize("scheme", HO)
def test_spectral_equals_dense(scheme):
    h = H.random_spectrum_hamiltonian(60, 25, -0.9, 0.0, 0.05, 1.0, seed=5)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ,
              mu=0.025, xi=0.05, tol=1e-11, max_iter=100)
    d = dense.purify(h.F, scheme, **kw)
    s = spectral.purify_spectrum(h.eigvals, scheme, **kw)
    assert d["status"] == s["status"] == "ok"
    assert d["products"] == s["products"] and d["branches"] == s["branches"]
    for a, b in zip(d["log"], s["log"]):
        assert abs(a["t1"] - b["t1"]) < 1e-9 and abs(a["e"] - b["e"]) < 1e-9 * max(1.0, b["e"])
        if "alpha" in a:
            assert a["alpha"] == b["alpha"]


@pytest.mark.parametrize("m", [3, 5])
@pytest.mark.parametrize("xi", [0.05, 1e-3])
def test_scaling_needs_fewer_products(m, xi):
    scaled = spectral.products_to_accuracy(f"snf_fixmu{m}", 0.5, xi, acc=1e-9)
    plain = spectral.products_to_accuracy(f"pmm{m}", 0.5, xi, acc=1e-9)
    assert scaled < plain


def test_higher_order_count_table():
    """Products to an eigenvalue error of 1e-9 (spectrum [0, 1], gap centred at 1/2): with
    the m + 1 products per iteration of the odd-symmetric evaluation, P_{1,1} (Algorithm 1)
    stays the cheapest scaled scheme at every gap -- higher order buys fewer iterations but
    not fewer products."""
    table = {}
    for xi in (0.05, 1e-3, 1e-5):
        row = [spectral.products_to_accuracy(s, 0.5, xi, acc=1e-9)
               for s in ("snf_fixmu", "snf_fixmu3", "snf_fixmu5")]
        table[xi] = row
        assert row[0] <= row[1] <= row[2]
    assert table == {0.05: [14, 20, 24], 1e-3: [22, 32, 42], 1e-5: [32, 48, 60]}
