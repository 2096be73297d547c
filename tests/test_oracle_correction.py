"""Pins of the subspace correction oracle (oracle/correction.py), CPU only.

The correction is not in the paper; what pins it is the mathematics it rests on:
* the Daleckii-Krein response equals the derivative of the exact projector, checked against
  central finite differences of eigendecomposition projectors and against the closed form at
  n = 2;
* the response is traceless and has no component inside either subspace;
* the purification pair recurrence converges to the Daleckii-Krein response;
* at the exact projector the coupling vanishes and the correction changes nothing;
* one Newton step turns an error e of a rotated projector into at most O(e^2): the ratio
  error_after / error_before^2 does not grow while error_before drops by 10.
A plausible slip (a sign of V, a transposed block, a missing factor of the f_0 scaling)
breaks the finite-difference or the quadratic pin.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import correction as corr
from oracle import exact
from paper_1101_0265_amd import hamiltonians as H


def _rotated(D: np.ndarray, eps: float, seed: int) -> np.ndarray:
    """exp(eps K) D exp(-eps K) for a random antisymmetric K with ||K||_F = 1."""
    rng = np.random.default_rng(seed)
    K = rng.standard_normal(D.shape)
    K = K - K.T
    K /= np.linalg.norm(K)
    R = expm(eps * K)
    return R @ D @ R.T


def _case(n=40, n_occ=17, seed=3):
    h = H.random_spectrum_hamiltonian(n, n_occ, -1.0, -0.05, 0.05, 1.0, seed)
    D = exact.projector(n_occ=n_occ, eigvals=h.eigvals, Q=h.Q)
    return h, D


def test_two_by_two_closed_form():
    a, b, c = -0.3, 1e-3, 0.4
    F = np.array([[a, b], [b, c]])
    Dt = np.diag([1.0, 0.0])
    F_bd, V = corr.block_split(F, Dt)
    assert np.array_equal(F_bd, np.diag([a, c])) and np.array_equal(V, [[0.0, b], [b, 0.0]])
    L = corr.dk_response(F_bd, V, 1)
    assert np.allclose(L, [[0.0, b / (a - c)], [b / (a - c), 0.0]], rtol=1e-14, atol=0)


def test_response_equals_finite_differences():
    h, D = _case()
    Dt = _rotated(D, 1e-2, seed=1)
    F_bd, V = corr.block_split(h.F, Dt)
    L = corr.dk_response(F_bd, V, h.n_occ)
    t = 1e-4
    fd = (exact.projector(F=F_bd + t * V, n_occ=h.n_occ)
          - exact.projector(F=F_bd - t * V, n_occ=h.n_occ)) / (2 * t)
    assert np.linalg.norm(fd - L) <= 1e-6 * np.linalg.norm(L)
    assert np.linalg.norm(L) > 1e-3


def test_response_is_traceless_and_off_diagonal():
    h, D = _case(seed=4)
    Dt = _rotated(D, 3e-3, seed=2)
    F_bd, V = corr.block_split(h.F, Dt)
    assert np.linalg.norm(F_bd @ Dt - Dt @ F_bd) <= 1e-13
    L = corr.dk_response(F_bd, V, h.n_occ)
    Q = np.eye(h.n) - Dt
    assert abs(np.trace(L)) <= 1e-12
    assert np.linalg.norm(Dt @ L @ Dt) <= 1e-10 * np.linalg.norm(L)
    assert np.linalg.norm(Q @ L @ Q) <= 1e-10 * np.linalg.norm(L)


def test_pair_recurrence_converges_to_daleckii_krein():
    h, D = _case(n=60, n_occ=25, seed=5)
    Dt = _rotated(D, 1e-2, seed=3)
    G = (h.lambda_max * np.eye(h.n) - h.F) / (h.lambda_max - h.lambda_min)
    G_bd, V_G = corr.block_split(G, Dt)
    steps = corr.alg2_steps(h.lambda_min, h.lambda_max, h.homo, h.lumo, 1e-13)
    X, X1 = corr.pair_response(G_bd, V_G, steps)
    F_bd, V = corr.block_split(h.F, Dt)
    L = corr.dk_response(F_bd, V, h.n_occ)
    assert np.linalg.norm(X1 - L) <= 1e-8 * np.linalg.norm(L)
    assert np.linalg.norm(X - Dt) <= 1e-9            # the recurrence itself reaches Dt
    # and the coupling of G is that of F scaled by f_0's factor
    assert np.allclose(V_G, -V / (h.lambda_max - h.lambda_min), atol=1e-14)


def test_exact_projector_is_a_fixed_point():
    h, D = _case(seed=6)
    F_bd, V = corr.block_split(h.F, D)
    assert np.linalg.norm(V) <= 1e-13
    r = corr.newton_correct(h.F, D, lambda_min=h.lambda_min, lambda_max=h.lambda_max,
                            homo=h.homo, lumo=h.lumo, n_occ=h.n_occ)
    assert np.linalg.norm(r["D"] - D) <= 1e-11


def test_newton_step_is_quadratic():
    h, D = _case(n=80, n_occ=37, seed=7)
    ratios, errs = [], []
    for eps in (1e-2, 1e-3):
        Dt = _rotated(D, eps, seed=11)
        before = np.linalg.norm(Dt - D)
        r = corr.newton_correct(h.F, Dt, lambda_min=h.lambda_min, lambda_max=h.lambda_max,
                                homo=h.homo, lumo=h.lumo, n_occ=h.n_occ)
        after = np.linalg.norm(r["D"] - D)
        errs.append((before, after))
        ratios.append(after / before ** 2)
        # the corrected D is a projector with the right trace
        assert np.linalg.norm(r["D"] @ r["D"] - r["D"]) <= 1e-10
        assert abs(np.trace(r["D"]) - h.n_occ) <= 1e-9
    (b1, a1), (b2, a2) = errs
    assert a1 <= b1 ** 2 and a2 <= b2 ** 2, errs
    # at least quadratic: after / before^2 does not grow as the error shrinks (it falls: the
    # second-order part of a rotation lies inside the two subspaces, where the refinement's
    # projection removes it)
    assert ratios[1] <= 4.0 * ratios[0], (errs, ratios)
