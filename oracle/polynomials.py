"""Purification polynomials P_{i,j} (test infrastructure only; see ``oracle/__init__``).

Definition (paragraph introducing the notation, after Eq. 1): P_{i,j} is the polynomial of
degree 1+i+j with fixed points 0 and 1, i vanishing derivatives at 0 and j vanishing
derivatives at 1.  ``p_ij_coefficients`` builds it from exactly these conditions by solving
the Hermite interpolation system; the closed forms used by the algorithms (P_{1,0} = x^2,
P_{0,1} = 2x - x^2, P_{1,1} = 3x^2 - 2x^3, Algorithm 1's update) are written separately and
the tests pin one against the other.

The higher-order fixed-mu schemes need P_{m,m} for odd m exactly, and the asymmetric ones
P_{i,j} with i != j both odd: ``p_ij_exact`` solves the same Hermite system in rational
arithmetic, so its coefficients carry no rounding.

Parity: pinned (closed forms == definition; fixed points and derivative conditions; the exact
coefficients against the binomial form of P_{i,j} and the derivative x^m (1-x)^m).
"""
from __future__ import annotations

import functools
from fractions import Fraction

import numpy as np


def p_ij_coefficients(i: int, j: int) -> np.ndarray:
    """Monomial coefficients c[0..d] (ascending) of P_{i,j}, d = 1+i+j.

    Conditions: P(0)=0, P^(k)(0)=0 for k=1..i, P(1)=1, P^(k)(1)=0 for k=1..j.
    That is 1+i + 1+j = d+1 linear conditions for d+1 unknowns.
    """
    d = 1 + i + j
    rows, rhs = [], []

    def deriv_row(x: float, k: int) -> np.ndarray:
        r = np.zeros(d + 1)
        for m in range(k, d + 1):
            fac = 1.0
            for t in range(k):
                fac *= (m - t)
            r[m] = fac * (x ** (m - k))
        return r

    for k in range(0, i + 1):
        rows.append(deriv_row(0.0, k))
        rhs.append(0.0)
    rows.append(deriv_row(1.0, 0))
    rhs.append(1.0)
    for k in range(1, j + 1):
        rows.append(deriv_row(1.0, k))
        rhs.append(0.0)
    return np.linalg.solve(np.array(rows), np.array(rhs))


def p_ij(i: int, j: int, x):
    """Evaluate P_{i,j}(x) from its defining conditions."""
    c = p_ij_coefficients(i, j)
    return np.polynomial.polynomial.polyval(x, c)


# Closed forms the algorithms use (text after the scale-and-fold idea; Algorithm 1).
def p10(x):
    """P_{1,0}(x) = x^2: folds the unoccupied side once it is stretched below 0."""
    return x * x


def p01(x):
    """P_{0,1}(x) = 2x - x^2: folds the occupied side once it is stretched above 1."""
    return 2.0 * x - x * x


def p11(x):
    """P_{1,1}(x) = 3x^2 - 2x^3 (McWeeny); odd in both ends, folds both sides."""
    return 3.0 * x * x - 2.0 * x * x * x


def p_ij_exact(i: int, j: int) -> list:
    """Monomial coefficients (ascending, ``Fraction``) of P_{i,j} from the same defining
    conditions as ``p_ij_coefficients``, solved by exact Gaussian elimination."""
    return list(_p_ij_exact(i, j))


@functools.lru_cache(maxsize=None)
def _p_ij_exact(i: int, j: int) -> tuple:
    d = 1 + i + j

    def deriv_row(x: int, k: int) -> list:
        r = [Fraction(0)] * (d + 1)
        for m in range(k, d + 1):
            fac = 1
            for t in range(k):
                fac *= (m - t)
            r[m] = Fraction(fac * (x ** (m - k)))
        return r

    rows = [deriv_row(0, k) + [Fraction(0)] for k in range(0, i + 1)]
    rows.append(deriv_row(1, 0) + [Fraction(1)])
    rows += [deriv_row(1, k) + [Fraction(0)] for k in range(1, j + 1)]
    size = d + 1
    for c in range(size):                       # exact elimination with row pivoting
        piv = next(r for r in range(c, size) if rows[r][c] != 0)
        rows[c], rows[piv] = rows[piv], rows[c]
        for r in range(size):
            if r != c and rows[r][c] != 0:
                f = rows[r][c] / rows[c][c]
                rows[r] = [a - f * b for a, b in zip(rows[r], rows[c])]
    return tuple(rows[k][size] / rows[k][k] for k in range(size))


def pmm(m: int, x):
    """P_{m,m}(x) in FP64, Horner on the exact coefficients rounded once to FP64."""
    c = [float(v) for v in p_ij_exact(m, m)]
    x = np.asarray(x, dtype=np.float64) if not np.isscalar(x) else float(x)
    y = c[-1]
    for k in range(len(c) - 2, -1, -1):
        y = y * x + c[k]
    return y


def pij(i: int, j: int, x):
    """P_{i,j}(x) in FP64, Horner on the exact coefficients rounded once to FP64 (any i, j;
    ``pmm`` is the case i = j)."""
    c = [float(v) for v in p_ij_exact(i, j)]
    x = np.asarray(x, dtype=np.float64) if not np.isscalar(x) else float(x)
    y = c[-1]
    for k in range(len(c) - 2, -1, -1):
        y = y * x + c[k]
    return y


def pij_fraction(i: int, j: int, x: Fraction) -> Fraction:
    """P_{i,j}(x) exactly, for a rational x."""
    y = Fraction(0)
    for c in reversed(p_ij_exact(i, j)):
        y = y * x + c
    return y
