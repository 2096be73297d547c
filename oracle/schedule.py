"""Scalar parameter schedules, in IEEE FP64 Python floats (test infrastructure only).

Every expression keeps the paper's operation order, evaluated left to right with no fused
multiply-add, so the decisions it takes are reproducible bit for bit by any FP64 code that
evaluates the same expressions in the same order.

* Algorithm 1 (McWeeny-based fixed-mu scale-and-fold): gamma, X_0 scaling and beta at set-up;
  per iteration alpha = 3 / sqrt(12 beta^2 - 18 beta + 9), beta_s = alpha (beta - 0.5) + 0.5,
  beta <- 3 beta_s^2 - 2 beta_s^3.  alpha solves Eq. 3 for m = 1.  alpha = 1 gives the regular
  grand-canonical McWeeny scheme.
* Algorithm 2 (P_{0,1} & P_{1,0} varying-mu scale-and-fold): beta = f0(lumo),
  beta-bar = f0(homo); if beta + beta-bar > 1 square with alpha = beta / (2 - beta), else fold
  with alpha = (1 - beta-bar) / (1 + beta-bar).  alpha = 0 gives the unscaled second-order
  trace-correcting scheme with the eigenvalue-based choice.
* Trace rule (the original trace-correcting choice, paragraph after Eqs. 4-5): square iff
  |tr(X^2) - N| < |2 tr X - tr(X^2) - N|; a tie folds.
* Higher-order fixed-mu scale-and-fold (the generalisation of Algorithm 1 to P_{m,m}, m odd,
  stated with Eqs. 2 and 3): f_i(X) = P_{m,m}(alpha (X - 0.5 I) + 0.5 I), alpha >= 1 the root
  of Eq. 3, beta <- P_{m,m}(alpha (beta - 0.5) + 0.5).  Eq. 3 has no closed form for m > 1; it
  is solved here by bisection.  alpha = 1 gives the unscaled grand-canonical P_{m,m} scheme.

* Asymmetric fixed-mu scale-and-fold (same paragraph: P_{i,j} with i, j odd, scaled about
  the polynomial's unstable fixed point x*, which differs from 0.5 when i != j).  The paper
  gives no parameters for it; the reading used here: X_0 = (mu I - F)/gamma + x* I with
  gamma = max((mu - lambda_min)/(1 - x*), (lambda_max - mu)/x*), so the spectrum fills
  [0, 1]; the state is a (upper end of the unoccupied part, below x*) and a-bar (distance of
  the occupied part's lower end from 1); f_i(X) = P_{i,j}(alpha (X - x* I) + x* I).  Each
  side has its own Eq.-3 root -- the alpha at which the folded image of the interval end
  equals the image of the gap edge, i.e. the alpha minimising that side's new bound -- and
  alpha is the smaller of the two, the largest scaling that speeds up both sides.  For
  i = j both roots are Eq. 3's.  alpha = 1 gives the unscaled grand-canonical P_{i,j}.

Parity: pinned (Eq. 3 residual, closed-form images of the interval ends, alpha = 0 / 1
reductions, exact-rational decisions).
"""
from __future__ import annotations

import math
from fractions import Fraction

from . import polynomials as poly

SQUARE = "S"   # P_{1,0} branch: X <- ((1+a) X - a I)^2
FOLD = "F"     # P_{0,1} branch: X <- 2 (1+a) X - (1+a)^2 X^2
MCW = "M"      # P_{1,1} branch: X <- 3 Xs^2 - 2 Xs^3, Xs = a (X - I/2) + I/2
PMM = {3: "3", 5: "5"}   # P_{m,m} branch: X <- P_{m,m}(Xs)

# scheme name -> (m, scaled) of the higher-order fixed-mu schemes
HIGHER_ORDER = {"snf_fixmu3": (3, True), "snf_fixmu5": (5, True),
                "pmm3": (3, False), "pmm5": (5, False)}
PIJ = "P"                # P_{i,j} branch: X <- P_{i,j}(alpha (X - x* I) + x* I)
# scheme name -> scaled, of the P_{i,j} fixed-mu schemes (i, j odd, passed separately)
GENERAL = {"snf_pij": True, "pij": False}
FIXED_MU = ("mcweeny", "snf_fixmu") + tuple(HIGHER_ORDER) + tuple(GENERAL)


# ---- Algorithm 1 -----------------------------------------------------------------------

def alg1_gamma(lambda_min: float, lambda_max: float, mu: float) -> float:
    """gamma = 2 max(lambda_max - mu, mu - lambda_min)."""
    return 2.0 * max(lambda_max - mu, mu - lambda_min)


def alg1_f0_scalar(lam: float, mu: float, gamma: float) -> float:
    """Image of an eigenvalue under X_0 = (mu I - F)/gamma + 0.5 I."""
    return (mu - lam) / gamma + 0.5


def alg1_beta0(xi: float, gamma: float) -> float:
    """beta = 0.5 (1 - xi / gamma): X-space image of the level nearest mu (symmetric gap)."""
    return 0.5 * (1.0 - xi / gamma)


def alg1_alpha(beta: float) -> float:
    """alpha = 3 / sqrt(12 beta^2 - 18 beta + 9), the root alpha >= 1 of Eq. 3 for m = 1."""
    return 3.0 / math.sqrt(12.0 * beta * beta - 18.0 * beta + 9.0)


def alg1_beta_next(beta: float, alpha: float) -> float:
    """beta_s = alpha (beta - 0.5) + 0.5; beta <- 3 beta_s^2 - 2 beta_s^3."""
    bs = alpha * (beta - 0.5) + 0.5
    return 3.0 * bs * bs - 2.0 * bs * bs * bs


# ---- Eq. 3 for P_{m,m} -------------------------------------------------------------------

def pmm_alpha(m: int, beta: float) -> float:
    """The root alpha >= 1 of Eq. 3, P(alpha (beta - 0.5) + 0.5) = P(0.5 (1 - alpha)), for
    P = P_{m,m} (m odd) and 0 < beta < 0.5.

    G(alpha) = P(0.5 (1 - alpha)) - P(alpha (beta - 0.5) + 0.5) is -P(beta) < 0 at alpha = 1
    and P(0.5 (1 - alpha)) > 0 where the scaled gap edge reaches 0, alpha = 1 / (1 - 2 beta);
    P decreases on x < 0 and increases on [0, 1], so G increases in between and the root is
    unique.  Plain bisection until the bracket stops shrinking.
    """
    if not 0.0 < beta < 0.5:
        raise ValueError("beta must lie in (0, 0.5)")

    def G(a):
        return poly.pmm(m, 0.5 * (1.0 - a)) - poly.pmm(m, a * (beta - 0.5) + 0.5)

    lo, hi = 1.0, 1.0 / (1.0 - 2.0 * beta)
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            return lo
        if G(mid) < 0.0:
            lo = mid
        else:
            hi = mid


def pmm_beta_next(m: int, beta: float, alpha: float) -> float:
    """beta <- P_{m,m}(alpha (beta - 0.5) + 0.5)."""
    return float(poly.pmm(m, alpha * (beta - 0.5) + 0.5))


# ---- P_{i,j}, i and j odd: scale-and-fold about the unstable fixed point -------------------

def check_poly(poly) -> tuple:
    i, j = (int(poly[0]), int(poly[1])) if poly is not None else (0, 0)
    if i < 1 or j < 1 or i % 2 == 0 or j % 2 == 0:
        raise ValueError("P_{i,j} fixed-mu schemes need odd i, j >= 1")
    return i, j


def pij_xstar(i: int, j: int) -> float:
    """The unstable fixed point of P_{i,j}: the root of P(x) = x inside (0, 1).

    P(x) - x is negative just above 0 (P has a zero of order i + 1 there) and positive just
    below 1, and P is S-shaped (P' = C x^i (1 - x)^j rises then falls), so the interior root
    is unique.  Bisection on dyadic rationals with the exact coefficients, to 2^-64."""
    lo, hi = Fraction(0), Fraction(1)
    for _ in range(64):
        mid = (lo + hi) / 2
        g = poly.pij_fraction(i, j, mid) - mid
        if g == 0:
            return float(mid)
        if g < 0:
            lo = mid
        else:
            hi = mid
    return float((lo + hi) / 2)


def pij_gamma(lambda_min: float, lambda_max: float, mu: float, xs: float) -> float:
    """Smallest gamma for which X_0 = (mu I - F)/gamma + x* I has its spectrum in [0, 1]."""
    return max((mu - lambda_min) / (1.0 - xs), (lambda_max - mu) / xs)


def pij_edges0(xi: float, gamma: float, xs: float) -> tuple:
    """(a, a-bar) of X_0 for a gap of width xi centred at mu: the gap edges sit at
    x* -/+ xi / (2 gamma)."""
    h = xi / (2.0 * gamma)
    return xs - h, (1.0 - xs) - h


def pij_alpha_side(i: int, j: int, xs: float, a: float) -> float:
    """One side's Eq. 3: the root alpha >= 1 of P(x* (1 - alpha)) = P(x* - alpha (x* - a))
    for 0 < a < x*, P = P_{i,j} (the folded image of the interval end 0 meets the image of the
    gap edge a).  G(alpha) = P(x* (1 - alpha)) - P(x* - alpha (x* - a)) is -P(a) < 0 at
    alpha = 1 and positive where the scaled edge reaches 0, alpha = x* / (x* - a); P falls on
    x < 0 and rises on [0, x*], so the root is unique.  Plain bisection until the bracket stops
    shrinking.  Outside (0, x*): 1."""
    if not 0.0 < a < xs:
        return 1.0

    def G(al):
        return poly.pij(i, j, xs * (1.0 - al)) - poly.pij(i, j, xs - al * (xs - a))

    lo, hi = 1.0, xs / (xs - a)
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            return lo
        if G(mid) < 0.0:
            lo = mid
        else:
            hi = mid


def pij_alpha(i: int, j: int, xs: float, a: float, abar: float) -> float:
    """alpha = the smaller of the two sides' roots.  The occupied side is the unoccupied side
    of the mirrored polynomial: 1 - P_{i,j}(1 - y) = P_{j,i}(y), fixed point 1 - x*."""
    return min(pij_alpha_side(i, j, xs, a), pij_alpha_side(j, i, 1.0 - xs, abar))


def pij_next(i: int, j: int, xs: float, a: float, abar: float, alpha: float) -> tuple:
    """(a, a-bar) after f_i: each side's new bound is the larger of the images of its
    interval end (folded when alpha > 1) and of its gap edge."""
    xm = 1.0 - xs
    a2 = max(poly.pij(i, j, xs * (1.0 - alpha)), poly.pij(i, j, xs - alpha * (xs - a)))
    b2 = max(poly.pij(j, i, xm * (1.0 - alpha)), poly.pij(j, i, xm - alpha * (xm - abar)))
    return float(a2), float(b2)


# ---- Algorithm 2 -----------------------------------------------------------------------

def alg2_f0_scalar(lam: float, lambda_min: float, lambda_max: float) -> float:
    """Image of an eigenvalue under X_0 = (lambda_max I - F)/(lambda_max - lambda_min)."""
    return (lambda_max - lam) / (lambda_max - lambda_min)


def alg2_choose_square(beta: float, betabar: float) -> bool:
    """The branch test of Algorithm 2: square (P_{1,0}) iff beta + beta-bar > 1."""
    return beta + betabar > 1.0


def alg2_square_alpha(beta: float) -> float:
    return beta / (2.0 - beta)


def alg2_square_scalar(x: float, alpha: float) -> float:
    """((1 + alpha) x - alpha)^2."""
    y = (1.0 + alpha) * x - alpha
    return y * y


def alg2_fold_alpha(betabar: float) -> float:
    return (1.0 - betabar) / (1.0 + betabar)


def alg2_fold_scalar(x: float, alpha: float) -> float:
    """2 (1 + alpha) x - (1 + alpha)^2 x^2."""
    return 2.0 * (1.0 + alpha) * x - (1.0 + alpha) * (1.0 + alpha) * x * x


# ---- trace rule ------------------------------------------------------------------------

def trace_choose_square(tr_x: float, tr_x2: float, n_occ: int) -> bool:
    """Square iff the trace after squaring is strictly closer to N than after folding."""
    return abs(tr_x2 - n_occ) < abs(2.0 * tr_x - tr_x2 - n_occ)


def trace_margin(tr_x: float, tr_x2: float, n_occ: int) -> float:
    """Signed distance of the trace decision from a tie (positive favours folding)."""
    return abs(tr_x2 - n_occ) - abs(2.0 * tr_x - tr_x2 - n_occ)


def products_per_iteration(scheme: str, poly_ij=None) -> int:
    """Matrix products one f_i costs.  Algorithm 1: X_s^2 and X_s^3.  P_{m,m} (m odd): the
    polynomial is point-symmetric about (1/2, 1/2), P(1/2 + v) = 1/2 + v r(v^2) with r of
    degree m, so v^2, then r by Horner (m - 1 products), then v r: m + 1 products.
    P_{i,j} (degree d = i + j + 1, odd): P(x* + v) = x* + v Q(v) with Q of even degree d - 1;
    Q by Horner's rule in v^2 with coefficients linear in v (v^2, then (d - 3)/2 Horner
    products), then v Q: (i + j)/2 + 1 products."""
    if scheme in HIGHER_ORDER:
        return HIGHER_ORDER[scheme][0] + 1
    if scheme in GENERAL:
        i, j = check_poly(poly_ij)
        return (i + j) // 2 + 1
    return 2 if scheme in ("mcweeny", "snf_fixmu") else 1


# ---- one step of the scalar state (used by the spectral and dense drivers) --------------

class SchemeState:
    """beta / beta-bar tracking for a scheme, one ``step`` per iteration.

    scheme: "sp2" (trace rule, no scaling), "tc2" (Algorithm 2, alpha = 0),
    "snf_varmu" (Algorithm 2), "mcweeny" (Algorithm 1, alpha = 1), "snf_fixmu"
    (Algorithm 1), "snf_fixmu3" / "snf_fixmu5" (scaled P_{3,3} / P_{5,5}), "pmm3" / "pmm5"
    (the same with alpha = 1), "snf_pij" / "pij" (P_{i,j} about its fixed point x*, scaled /
    alpha = 1; ``poly_ij`` = (i, j), both odd; beta-bar = 1 - a-bar).  For "sp2" the tracked beta / beta-bar follow the branches
    actually taken (they are reported only; the choice uses traces).
    """

    def __init__(self, scheme: str, lambda_min: float, lambda_max: float, *,
                 homo: float = None, lumo: float = None, mu: float = None,
                 xi: float = None, poly_ij=None):
        self.scheme = scheme
        self.xs = 0.5
        if scheme in GENERAL:
            self.i, self.j = check_poly(poly_ij)
            self.xs = pij_xstar(self.i, self.j)
            self.gamma = pij_gamma(lambda_min, lambda_max, mu, self.xs)
            self.beta, self.abar = pij_edges0(xi, self.gamma, self.xs)
            self.betabar = 1.0 - self.abar
        elif scheme in ("sp2", "tc2", "snf_varmu"):
            self.beta = alg2_f0_scalar(lumo, lambda_min, lambda_max) if lumo is not None else 0.0
            self.betabar = (alg2_f0_scalar(homo, lambda_min, lambda_max)
                            if homo is not None else 1.0)
            self.gamma = None
        elif scheme in FIXED_MU:
            self.gamma = alg1_gamma(lambda_min, lambda_max, mu)
            self.beta = alg1_beta0(xi, self.gamma)
            self.betabar = 1.0 - self.beta
        else:
            raise ValueError(f"unknown scheme {scheme!r}")

    def choose(self, tr_x: float = None, tr_x2: float = None, n_occ: int = None):
        """Return (branch, alpha) for the next iteration without changing the state."""
        s = self.scheme
        if s == "sp2":
            return (SQUARE if trace_choose_square(tr_x, tr_x2, n_occ) else FOLD), 0.0
        if s in ("tc2", "snf_varmu"):
            if alg2_choose_square(self.beta, self.betabar):
                return SQUARE, (alg2_square_alpha(self.beta) if s == "snf_varmu" else 0.0)
            return FOLD, (alg2_fold_alpha(self.betabar) if s == "snf_varmu" else 0.0)
        if s in GENERAL:
            return PIJ, (pij_alpha(self.i, self.j, self.xs, self.beta, self.abar)
                         if GENERAL[s] else 1.0)
        if s in HIGHER_ORDER:
            m, scaled = HIGHER_ORDER[s]
            return PMM[m], (pmm_alpha(m, self.beta) if scaled and self.beta > 0.0 else 1.0)
        return MCW, (alg1_alpha(self.beta) if s == "snf_fixmu" else 1.0)

    def advance(self, branch: str, alpha: float) -> None:
        if branch == SQUARE:
            self.beta = alg2_square_scalar(self.beta, alpha)
            self.betabar = alg2_square_scalar(self.betabar, alpha)
        elif branch == FOLD:
            self.beta = alg2_fold_scalar(self.beta, alpha)
            self.betabar = alg2_fold_scalar(self.betabar, alpha)
        elif branch == MCW:
            self.beta = alg1_beta_next(self.beta, alpha)
            self.betabar = 1.0 - self.beta
        elif branch == PIJ:
            self.beta, self.abar = pij_next(self.i, self.j, self.xs, self.beta, self.abar,
                                            alpha)
            self.betabar = 1.0 - self.abar
        else:
            m = 3 if branch == PMM[3] else 5
            self.beta = pmm_beta_next(m, self.beta, alpha)
            self.betabar = 1.0 - self.beta

    def bound(self) -> float:
        """A-priori eigenvalue error bound max(beta, 1 - beta-bar) with exact bounds."""
        if self.scheme in GENERAL:
            return max(self.beta, self.abar)
        return max(self.beta, 1.0 - self.betabar)
