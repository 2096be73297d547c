"""Pins of the asymmetric fixed-mu schemes in the CPU oracle (no GPU).

The scheme (paragraph before Algorithm 1: scale-and-fold also works for P_{i,j} with i, j odd,
scaled about the polynomial's unstable fixed point x*, which is not 0.5 when i != j):
X_0 = (mu I - F)/gamma + x* I and f_i(X) = P_{i,j}(alpha (X - x* I) + x* I).  The reading of
gamma, of the two tracked bounds and of alpha is stated in ``oracle.schedule``.  Pinned
against: the defining property P(x*) = x* in exact arithmetic and a library root finder, the
mirror identity 1 - P_{i,j}(1 - x) = P_{j,i}(x), the closed-form alpha of Algorithm 1 and the
P_{m,m} roots of Eq. 3 when i = j, a brute-force minimisation of each side's new bound over
alpha, brute-force images of sampled spectra (the tracked bounds must contain them), the
exact projector, and the spectral oracle.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense, polynomials as poly, schedule as sch, spectral

PAIRS = [(1, 3), (3, 1), (1, 5), (5, 1), (3, 5), (5, 3)]


@pytest.mark.parametrize("i,j", PAIRS + [(1, 1), (3, 3), (5, 5)])
def test_fixed_point_exact_and_against_library_root(i, j):
    xs = sch.pij_xstar(i, j)
    assert 0.0 < xs < 1.0
    # |P(x*) - x*| within a few units of the last place, exactly evaluated
    g = poly.pij_fraction(i, j, Fraction(xs)) - Fraction(xs)
    assert abs(float(g)) <= 4 * math.ulp(xs)
    # sign change around x*: P below the diagonal on the left, above on the right
    for d in (1e-9, 1e-6, 1e-3):
        assert poly.pij_fraction(i, j, Fraction(xs - d)) < Fraction(xs - d)
        assert poly.pij_fraction(i, j, Fraction(xs + d)) > Fraction(xs + d)
    # the only interior root of P(x) - x, from numpy's companion-matrix root finder
    c = np.array([float(v) for v in poly.p_ij_exact(i, j)])
    c[1] -= 1.0
    roots = np.polynomial.polynomial.polyroots(c)
    inside = [r.real for r in roots if abs(r.imag) < 1e-9 and 1e-6 < r.real < 1 - 1e-6]
    assert len(inside) == 1
    assert abs(inside[0] - xs) < 1e-9
    if i == j:
        assert xs == 0.5


@pytest.mark.parametrize("i,j", PAIRS)
def test_mirror_identity_and_fixed_points(i, j):
    # 1 - P_{i,j}(1 - x) = P_{j,i}(x), exactly at rational points
    for x in (Fraction(1, 9), Fraction(3, 7), Fraction(-2, 5), Fraction(11, 10)):
        assert 1 - poly.pij_fraction(i, j, 1 - x) == poly.pij_fraction(j, i, x)
    assert abs(sch.pij_xstar(i, j) + sch.pij_xstar(j, i) - 1.0) <= 2 * math.ulp(1.0)


def test_gamma_and_edges_reduce_to_algorithm1():
    for lmin, lmax, mu, xi in [(-1.0, 1.0, 0.0, 0.05), (-2.0, 1.0, 0.3, 0.1),
                               (-0.7, 1.9, -0.2, 0.01)]:
        g = sch.pij_gamma(lmin, lmax, mu, 0.5)
        assert g == sch.alg1_gamma(lmin, lmax, mu)
        a, abar = sch.pij_edges0(xi, g, 0.5)
        assert a == abar
        assert abs(a - sch.alg1_beta0(xi, g)) <= 2 * math.ulp(0.5)


@pytest.mark.parametrize("i,j", PAIRS)
def test_f0_fills_unit_interval(i, j):
    xs = sch.pij_xstar(i, j)
    for lmin, lmax, mu in [(-1.0, 1.0, -0.5), (-1.0, 1.0, 0.6), (0.0, 3.0, 1.0)]:
        g = sch.pij_gamma(lmin, lmax, mu, xs)
        lo = (mu - lmax) / g + xs
        hi = (mu - lmin) / g + xs
        assert lo >= -1e-15 and hi <= 1.0 + 1e-15
        assert min(abs(lo), abs(hi - 1.0)) <= 1e-15       # one end touches


@pytest.mark.parametrize("beta", [0.05, 0.2, 0.35, 0.45, 0.499])
def test_alpha_reduces_to_closed_forms_when_symmetric(beta):
    # m = 1: Algorithm 1's alpha = 3 / sqrt(12 beta^2 - 18 beta + 9)
    a = sch.pij_alpha(1, 1, 0.5, beta, beta)
    assert a == pytest.approx(sch.alg1_alpha(beta), rel=1e-14)
    for m in (3, 5):
        assert sch.pij_alpha(m, m, 0.5, beta, beta) == pytest.approx(sch.pmm_alpha(m, beta),
                                                                     rel=1e-14)


def _side_bound(i, j, xs, a, al):
    return max(float(poly.pij(i, j, xs * (1.0 - al))), float(poly.pij(i, j, xs - al * (xs - a))))


@pytest.mark.parametrize("i,j", PAIRS)
@pytest.mark.parametrize("frac", [0.1, 0.5, 0.9, 0.99])
def test_side_alpha_solves_eq3_and_minimises_the_side_bound(i, j, frac):
    xs = sch.pij_xstar(i, j)
    a = xs * frac                      # gap edge somewhere below x*
    al = sch.pij_alpha_side(i, j, xs, a)
    assert 1.0 <= al <= xs / (xs - a)
    lhs = float(poly.pij(i, j, xs * (1.0 - al)))
    rhs = float(poly.pij(i, j, xs - al * (xs - a)))
    assert abs(lhs - rhs) <= 1e-12 * max(lhs, rhs, 1e-300) + 1e-300
    # brute force: no alpha on a fine grid of [1, x*/(x* - a)] gives a smaller bound
    grid = np.linspace(1.0, xs / (xs - a), 4001)
    best = min(_side_bound(i, j, xs, a, g) for g in grid)
    assert _side_bound(i, j, xs, a, al) <= best * (1.0 + 1e-9) + 1e-300


@pytest.mark.parametrize("i,j", PAIRS)
def test_alpha_is_the_smaller_root_and_improves_both_sides(i, j):
    xs = sch.pij_xstar(i, j)
    rng = np.random.default_rng(7)
    for _ in range(20):
        a = xs * rng.uniform(0.05, 0.999)
        abar = (1.0 - xs) * rng.uniform(0.05, 0.999)
        al = sch.pij_alpha(i, j, xs, a, abar)
        lo = sch.pij_alpha_side(i, j, xs, a)
        hi = sch.pij_alpha_side(j, i, 1.0 - xs, abar)
        assert al == min(lo, hi)
        a2, b2 = sch.pij_next(i, j, xs, a, abar, al)
        a1, b1 = sch.pij_next(i, j, xs, a, abar, 1.0)     # unscaled step
        assert a2 <= a1 * (1.0 + 1e-12) and b2 <= b1 * (1.0 + 1e-12)
        assert 0.0 <= a2 < xs and 0.0 <= b2 < 1.0 - xs


@pytest.mark.parametrize("scheme", ["snf_pij", "pij"])
@pytest.mark.parametrize("i,j", PAIRS)
def test_tracked_bounds_contain_every_image(scheme, i, j):
    """Brute force on a dense sample of X_0's possible spectrum: after every step all images
    of the unoccupied part stay in [0, a] and of the occupied part in [1 - a-bar, 1]."""
    lmin, lmax, mu, xi = -1.0, 1.0, -0.4, 0.04
    st = sch.SchemeState(scheme, lmin, lmax, mu=mu, xi=xi, poly_ij=(i, j))
    lam_v = np.linspace(mu + xi / 2, lmax, 3001)        # unoccupied, edges included
    lam_o = np.linspace(lmin, mu - xi / 2, 3001)        # occupied
    pv = spectral.f0_eigs(lam_v, scheme, lmin, lmax, mu, st)
    po = spectral.f0_eigs(lam_o, scheme, lmin, lmax, mu, st)
    assert pv.max() <= st.beta * (1 + 1e-13) and po.min() >= st.betabar * (1 - 1e-13)
    for _ in range(12):
        if st.bound() < 1e-14:
            break
        br, al = st.choose()
        pv = spectral.apply_branch(pv, br, al, st)
        po = spectral.apply_branch(po, br, al, st)
        st.advance(br, al)
        tol = 1e-12
        assert pv.min() >= -tol and pv.max() <= st.beta + tol
        assert po.max() <= 1.0 + tol and po.min() >= 1.0 - st.abar - tol


def _rotated(n, lam, seed):
    rng = np.random.default_rng(seed)
    Q, r = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(r))
    F = (Q * lam) @ Q.T
    return 0.5 * (F + F.T), Q


@pytest.mark.parametrize("i,j", PAIRS)
@pytest.mark.parametrize("mu", [-0.5, 0.0, 0.45])
def test_dense_oracle_reaches_exact_projector(i, j, mu):
    n, xi = 96, 0.05
    rng = np.random.default_rng(1101 + i * 10 + j)
    n_occ = int(n * (mu + 1.0) / 2.0)
    lam = np.concatenate([rng.uniform(-1.0, mu - xi / 2, n_occ - 2), [-1.0, mu - xi / 2],
                          rng.uniform(mu + xi / 2, 1.0, n - n_occ - 2), [mu + xi / 2, 1.0]])
    lam.sort()
    F, Q = _rotated(n, lam, 5)
    kw = dict(lambda_min=-1.0, lambda_max=1.0, mu=mu, xi=xi, n_occ=n_occ, tol=1e-10,
              poly_ij=(i, j))
    d = dense.purify(F, "snf_pij", **kw)
    s = spectral.purify_spectrum(lam, "snf_pij", **kw)
    assert d["status"] == "ok" and s["status"] == "ok"
    D_ref = Q[:, :n_occ] @ Q[:, :n_occ].T
    assert np.linalg.norm(d["D"] - D_ref) <= 1e-9
    assert abs(np.trace(d["D"]) - n_occ) < 1e-9
    assert d["iterations"] == s["iterations"] and d["products"] == s["products"]
    assert d["products"] == d["iterations"] * ((i + j) // 2 + 1) + 1
    for rd, rs in zip(d["log"], s["log"]):
        assert rd["e"] == pytest.approx(rs["e"], rel=1e-6, abs=1e-11)
        if "alpha" in rs:
            assert rd["alpha"] == rs["alpha"]


@pytest.mark.parametrize("m", [1, 3, 5])
def test_symmetric_pair_matches_pmm_schemes(m):
    kw = dict(lambda_min=-1.0, lambda_max=1.0, mu=0.0, xi=0.05, homo=-0.025, lumo=0.025)
    gen = spectral.decision_sequence("snf_pij", poly_ij=(m, m), steps=8, **kw)
    ref = spectral.decision_sequence("snf_fixmu" if m == 1 else f"snf_fixmu{m}", steps=8, **kw)
    for (bg, ag, beg, bbg), (br, ar, ber, bbr) in zip(gen, ref):
        assert ag == pytest.approx(ar, rel=1e-13)
        assert beg == pytest.approx(ber, rel=1e-9, abs=1e-300)


def test_matching_side_of_an_off_centre_mu_is_cheaper():
    """With mu at a quarter of the spectrum (the setting of the paper's McWeeny illustration)
    the polynomial whose fixed point sits on the same side needs fewer products than its
    mirror: the occupied part is short, the unoccupied part long, so x* near 1 spends the
    unit interval where the spectrum is."""
    kw = dict(lambda_min=-1.0, lambda_max=1.0, mu=-0.5, xi=0.01)
    p31 = spectral.products_to_accuracy_pij((3, 1), **kw)
    p13 = spectral.products_to_accuracy_pij((1, 3), **kw)
    assert p31 < p13
