"""Exact targets (test infrastructure only).

* ``projector`` -- the definition D = theta(mu I - F): the orthogonal projector onto the
  eigenvectors of F whose eigenvalues lie below the gap, D = Q_occ Q_occ^T.  Either from the
  construction's own (eigenvalues, Q) or from a symmetric eigendecomposition.
* ``invariants`` -- ||D^2 - D||_F, tr D - N_occ and ||F D - D F||_F (a projector onto an
  invariant subspace of F has all three zero).
* ``alg2_decisions_exact`` -- the branch sequence of Algorithm 2 in exact rational arithmetic
  (it uses only + - * /), started from the FP64 values of the four bounds.  Ties are seen
  exactly, with no rounding.

Parity: pinned (definition; special cases reduce to numpy.linalg.eigh).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def projector(F: np.ndarray = None, n_occ: int = None, eigvals: np.ndarray = None,
              Q: np.ndarray = None) -> np.ndarray:
    """D = Q_occ Q_occ^T for the n_occ lowest eigenvalues."""
    if Q is None:
        eigvals, Q = np.linalg.eigh(np.asarray(F, dtype=np.float64))
    order = np.argsort(eigvals, kind="stable")
    qo = Q[:, order[:n_occ]]
    return qo @ qo.T


def projector_entries(Q: np.ndarray, eigvals: np.ndarray, n_occ: int, rows: np.ndarray,
                      cols: np.ndarray) -> np.ndarray:
    """Selected entries D[rows[k], cols[k]] = sum over occupied eigenvectors q_r q_c."""
    order = np.argsort(eigvals, kind="stable")[:n_occ]
    qo = Q[:, order]
    return np.einsum("kj,kj->k", qo[rows], qo[cols])


def invariants(D: np.ndarray, F: np.ndarray, n_occ: int) -> dict:
    return dict(idem=float(np.linalg.norm(D @ D - D)),
                trace_err=float(np.trace(D) - n_occ),
                commutator=float(np.linalg.norm(F @ D - D @ F)))


def alg2_decisions_exact(lambda_min: float, lambda_max: float, homo: float, lumo: float,
                         steps: int, scaled: bool = True) -> list:
    """Branch letters (S/F) of Algorithm 2 (scaled) or its alpha = 0 form, exactly.

    Rational sizes double with each squaring, so keep ``steps`` modest (<= 16).
    """
    lmin, lmax = Fraction(lambda_min), Fraction(lambda_max)
    beta = (lmax - Fraction(lumo)) / (lmax - lmin)
    betabar = (lmax - Fraction(homo)) / (lmax - lmin)
    out = []
    one, two = Fraction(1), Fraction(2)
    for _ in range(steps):
        if beta + betabar > one:
            a = beta / (two - beta) if scaled else Fraction(0)
            beta = ((one + a) * beta - a) ** 2
            betabar = ((one + a) * betabar - a) ** 2
            out.append("S")
        else:
            a = (one - betabar) / (one + betabar) if scaled else Fraction(0)
            beta = two * (one + a) * beta - (one + a) ** 2 * beta ** 2
            betabar = two * (one + a) * betabar - (one + a) ** 2 * betabar ** 2
            out.append("F")
    return out
