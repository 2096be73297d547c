"""Subspace correction of an approximate density matrix that re-references F (test
infrastructure only).

Not in the paper, which reasons in exact arithmetic.  A purification run with low-precision
products ends, after FP64 refinement, at a projector D~ that is idempotent and has the right
trace but spans a slightly rotated subspace: refinement by purification is a function of the
iterate, not of F, so it cannot see the rotation.  One Newton step on the invariant subspace
removes it to first order, and this module computes that step by its definitions:

* ``block_split(F, Dt)``: with respect to the projector Dt, F = F_bd + V where
  F_bd = Dt F Dt + (I - Dt) F (I - Dt) commutes with Dt (so Dt is the projector onto the lowest
  rank(Dt) eigenvectors of F_bd while the rotation is small) and V = Dt F (I - Dt) +
  (I - Dt) F Dt is the coupling between the two subspaces.
* ``dk_response(F_bd, V, n_occ)``: the first-order change of D = theta(mu I - F) at F_bd in the
  direction V, by the Daleckii-Krein formula: in the eigenbasis of F_bd the change of entry
  (a, b) is V_ab (theta_a - theta_b) / (lambda_a - lambda_b), theta = 1 for the n_occ lowest
  eigenvalues and 0 otherwise (zero inside each subspace).
* ``pair_response(X0, X1_0, steps)``: the same first-order change obtained the way a
  purification reaches D: the recurrence X <- c2 X^2 + c1 X + c0 I applied to X0 = f_0(F_bd)
  carries its derivative along, X1 <- c2 (X X1 + X1 X) + c1 X1, from X1_0 = f_0'(V).  As the
  polynomials converge to the step function, X1 converges to ``dk_response``.
* ``newton_correct(F, Dt, ...)``: the correction as the library runs it: f_0 of Algorithm 2
  maps F to G = (lambda_max I - F) / (lambda_max - lambda_min); G is split with respect to Dt
  (its coupling is -V / (lambda_max - lambda_min)); the pair recurrence runs Algorithm 2's
  branch and alpha sequence from the gap-edge bounds until max(beta, 1 - beta-bar) <= eps;
  D = Dt + X1; then plain trace-correcting steps (x^2 or 2x - x^2 by the trace rule) restore
  idempotency to tol.

Parity: pinned against central finite differences of exact projectors (the definition of the
derivative), the recurrence against Daleckii-Krein, the zero correction at the exact projector,
and the quadratic error reduction of the Newton step (tests/test_oracle_correction.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import schedule as sch


def block_split(F: np.ndarray, Dt: np.ndarray) -> tuple:
    """(F_bd, V) with F = F_bd + V, F_bd block-diagonal and V off-diagonal w.r.t. Dt."""
    n = F.shape[0]
    Q = np.eye(n) - Dt
    F_bd = Dt @ F @ Dt + Q @ F @ Q
    V = Dt @ F @ Q + Q @ F @ Dt
    return F_bd, V


def dk_response(F_bd: np.ndarray, V: np.ndarray, n_occ: int) -> np.ndarray:
    """First-order change of the projector onto the n_occ lowest eigenvectors of F_bd in the
    direction V (Daleckii-Krein divided differences of the step function)."""
    lam, U = np.linalg.eigh(F_bd)
    theta = np.zeros(lam.size)
    theta[np.argsort(lam, kind="stable")[:n_occ]] = 1.0
    dl = lam[:, None] - lam[None, :]
    dt = theta[:, None] - theta[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        gamma = np.where(dt != 0.0, dt / np.where(dl != 0.0, dl, 1.0), 0.0)
    return U @ (gamma * (U.T @ V @ U)) @ U.T


def pair_response(X0: np.ndarray, X1_0: np.ndarray, steps) -> tuple:
    """Apply X <- c2 X^2 + c1 X + c0 I for each (c2, c1, c0) in ``steps`` to X0 and carry its
    derivative X1 <- c2 (X X1 + X1 X) + c1 X1 from X1_0.  Returns (X, X1)."""
    X, X1 = X0.copy(), X1_0.copy()
    I = np.eye(X.shape[0])
    for c2, c1, c0 in steps:
        X1 = c2 * (X @ X1 + X1 @ X) + c1 * X1
        X = c2 * (X @ X) + c1 * X + c0 * I
    return X, X1


def expanded_coefficients(branch: str, alpha: float) -> tuple:
    """Algorithm 2's two maps in powers of X: ((1+a) X - a I)^2 = (1+a)^2 X^2 - 2a(1+a) X +
    a^2 I and 2(1+a) X - (1+a)^2 X^2."""
    if branch == sch.SQUARE:
        return (1.0 + alpha) ** 2, -2.0 * alpha * (1.0 + alpha), alpha * alpha
    return -((1.0 + alpha) ** 2), 2.0 * (1.0 + alpha), 0.0


def alg2_steps(lambda_min: float, lambda_max: float, homo: float, lumo: float,
               eps: float, max_iter: int = 200) -> list:
    """(c2, c1, c0) of Algorithm 2's iterations until max(beta, 1 - beta-bar) <= eps."""
    st = sch.SchemeState("snf_varmu", lambda_min, lambda_max, homo=homo, lumo=lumo)
    out = []
    for _ in range(max_iter):
        if st.bound() <= eps:
            return out
        branch, alpha = st.choose()
        out.append(expanded_coefficients(branch, alpha))
        st.advance(branch, alpha)
    raise RuntimeError("the bounds do not converge")


def refine_trace(X: np.ndarray, n_occ: int, tol: float, max_iter: int = 60) -> tuple:
    """Trace-correcting steps (square iff |tr X^2 - N| < |2 tr X - tr X^2 - N|) until
    ||X^2 - X||_F <= tol; returns (X, products) with the certifying product counted."""
    products = 0
    for _ in range(max_iter + 1):
        X2 = X @ X
        products += 1
        if np.linalg.norm(X2 - X) <= tol:
            return X, products
        if sch.trace_choose_square(float(np.trace(X)), float(np.trace(X2)), n_occ):
            X = X2
        else:
            X = 2.0 * X - X2
    raise RuntimeError("refinement did not converge")


def newton_correct(F: np.ndarray, Dt: np.ndarray, *, lambda_min: float, lambda_max: float,
                   homo: float, lumo: float, n_occ: int, eps: float = 1e-10,
                   tol: float = 1e-10) -> dict:
    """One Newton step on the subspace of Dt for F, then refinement; see the module text."""
    n = F.shape[0]
    G = (lambda_max * np.eye(n) - F) / (lambda_max - lambda_min)
    G_bd, V_G = block_split(G, Dt)
    steps = alg2_steps(lambda_min, lambda_max, homo, lumo, eps)
    _, X1 = pair_response(G_bd, V_G, steps)
    D1 = Dt + X1
    D, refine = refine_trace(D1, n_occ, tol)
    return dict(D=D, D_linear=D1, response=X1, iterations=len(steps), refine_products=refine)
