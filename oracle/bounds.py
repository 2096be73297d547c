"""Spectral and gap-edge bounds for the purification inputs (test infrastructure only).

Both algorithms take bounds as inputs: the extremal eigenvalues of F or bounds of them, and
for the scaled varying-mu scheme a lower bound of the highest occupied and an upper bound of
the lowest unoccupied eigenvalue (the bounds paragraph after Fig. 3, which points to methods
for interior eigenvalues).  Written here from textbook definitions:

* ``lanczos`` -- the Lanczos recurrence with full reorthogonalisation by classical
  Gram-Schmidt applied twice: w = A v_j, w <- w - V h, h = V^T w (twice), alpha_j the sum of
  the two h_j, beta_j = ||w||, v_{j+1} = w / beta_j.  The tridiagonal T = tridiag(beta, alpha,
  beta) has the Ritz values; the residual of a Ritz pair (theta, V s) is beta_k |s_k|, and an
  eigenvalue of A lies within it of theta.  T is truncated at the first beta_j below
  1e-12 max |alpha| (an invariant subspace was found).  ``scipy.linalg.eigh_tridiagonal``
  diagonalises T.
* ``spectral_bounds`` -- [theta_min - r_min, theta_max + r_max] from Lanczos on F, widened by
  1e-13 max |theta| for the rounding of converged pairs (outer bounds once the extreme Ritz
  pairs belong to the extreme eigenvalues).
* ``gap_bounds`` -- from a projector D onto the occupied subspace: the largest eigenvalue of
  D (F - lambda_min I) D is HOMO - lambda_min and that of (I - D)(lambda_max I - F)(I - D) is
  lambda_max - LUMO; Ritz values never exceed the largest eigenvalue, so
  homo = lambda_min + theta_1 <= HOMO and lumo = lambda_max - theta_2 >= LUMO hold at any
  number of steps (exactly when D is the exact projector; a subspace error phi of D moves
  them by O(phi^2 (lambda_max - lambda_min))); both widened by 1e-13 (lambda_max -
  lambda_min) for rounding.
* ``gershgorin`` -- the union of the Gershgorin discs, a rigorous enclosure.

Parity: pinned (all Ritz values equal the eigenvalues at k = n; interlacing and residual
enclosures; gap bounds equal the exact edges at k = n and bound them at small k; Gershgorin
enclosure).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal

BREAKDOWN = 1e-12


def lanczos(apply, v0: np.ndarray, steps: int):
    """Returns (alpha, beta) of the first k <= steps Lanczos steps (beta[k-1] = residual
    coupling of the last step)."""
    n = v0.size
    V = np.zeros((steps + 1, n))
    V[0] = v0 / np.linalg.norm(v0)
    alpha, beta = [], []
    for j in range(steps):
        w = apply(V[j])
        h = V[:j + 1] @ w
        w = w - V[:j + 1].T @ h
        h2 = V[:j + 1] @ w
        w = w - V[:j + 1].T @ h2
        alpha.append(h[j] + h2[j])
        b = float(np.linalg.norm(w))
        beta.append(b)
        if b <= BREAKDOWN * max(abs(a) for a in alpha):
            break
        V[j + 1] = w / b
    return np.array(alpha), np.array(beta)


def truncate_tridiagonal(alpha: np.ndarray, beta: np.ndarray):
    """Keep T up to the first breakdown (beta_j <= 1e-12 max |alpha_0..j|): (alpha, beta, k)."""
    k = len(alpha)
    for j in range(len(beta)):
        if beta[j] <= BREAKDOWN * np.max(np.abs(alpha[:j + 1])):
            k = j + 1
            return alpha[:k], beta[:k], k, True
    return alpha[:k], beta[:k], k, False


def ritz_extremes(alpha: np.ndarray, beta: np.ndarray):
    """(theta_min, r_min, theta_max, r_max) of the tridiagonal with diagonal alpha and
    off-diagonal beta[:-1]; r = beta[-1] |s_last| (0 after a breakdown)."""
    a, b, k, broke = truncate_tridiagonal(alpha, beta)
    if k == 1:
        w, s = np.array([a[0]]), np.array([[1.0]])
    else:
        w, s = eigh_tridiagonal(a, b[:k - 1])
    tail = 0.0 if broke else b[k - 1]
    return w[0], tail * abs(s[-1, 0]), w[-1], tail * abs(s[-1, -1])


def spectral_bounds(F: np.ndarray, v0: np.ndarray, steps: int):
    """Widened by the residuals and by 1e-13 max |theta| (rounding of converged pairs)."""
    al, be = lanczos(lambda v: F @ v, v0, steps)
    tmin, rmin, tmax, rmax = ritz_extremes(al, be)
    pad = 1e-13 * max(abs(tmin), abs(tmax))
    return tmin - rmin - pad, tmax + rmax + pad


def gap_bounds(F: np.ndarray, D: np.ndarray, lambda_min: float, lambda_max: float,
               v0: np.ndarray, steps: int):
    """(homo, lumo) with homo <= HOMO and lumo >= LUMO (for an exact projector D)."""
    P = np.eye(F.shape[0]) - D

    def a1(v):
        y = D @ v
        return D @ (F @ y - lambda_min * y)

    def a2(v):
        y = P @ v
        return P @ (lambda_max * y - F @ y)

    t1 = ritz_extremes(*lanczos(a1, v0, steps))[2]
    t2 = ritz_extremes(*lanczos(a2, v0, steps))[2]
    pad = 1e-13 * (lambda_max - lambda_min)
    return lambda_min + t1 - pad, lambda_max - t2 + pad


def gershgorin(F: np.ndarray):
    d = np.diag(F)
    r = np.sum(np.abs(F), axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))
