"""Pins of two oracle helpers that GPU parity tests rely on (no GPU).

* ``dense.block_truncation_mask`` -- the fixed-threshold block truncation used by every
  block-sparse parity test (a reading; the sparsity paragraph of the paper names truncation of
  small elements but gives no rule): after a step, block (I, J), I < J, is dropped together
  with its mirror (J, I) when its Frobenius norm is below tau; a block exactly at tau stays;
  diagonal blocks always stay.  Pinned on hand-built blocks at the threshold and one ulp below
  it, on asymmetric inputs (the decision follows the upper block), and against a brute-force
  loop over the blocks.
* ``exact.projector_entries`` -- selected entries of D = Q_occ Q_occ^T, the reference of the
  large parity tests.  Pinned against the full projector (and numpy's eigendecomposition) at
  small orders, with the eigenvalues passed unsorted.
"""
import math

import numpy as np
import pytest

from oracle import dense, exact

B = 4
TAU = 2.0 ** -20        # a power of two: a block holding the single entry TAU has norm TAU


def _blocks_kept(Y: np.ndarray, b: int) -> np.ndarray:
    nb = Y.shape[0] // b
    return np.array([[np.any(Y[I * b:(I + 1) * b, J * b:(J + 1) * b] != 0.0)
                      for J in range(nb)] for I in range(nb)])


def _single_entry(nb: int, I: int, J: int, v: float, mirror: bool = True) -> np.ndarray:
    X = np.zeros((nb * B, nb * B))
    X[I * B + 1, J * B + 2] = v
    if mirror:
        X[J * B + 2, I * B + 1] = v
    return X


def test_block_exactly_at_threshold_is_kept():
    X = _single_entry(3, 0, 2, TAU)
    assert math.sqrt(TAU * TAU) == TAU
    Y = dense.block_truncation_mask(B, TAU)(X)
    assert np.array_equal(Y, X)


def test_block_one_ulp_below_is_dropped_with_its_mirror():
    v = np.nextafter(TAU, 0.0)
    X = _single_entry(3, 0, 2, v) + _single_entry(3, 1, 2, 3.0 * TAU)
    Y = dense.block_truncation_mask(B, TAU)(X)
    kept = _blocks_kept(Y, B)
    assert not kept[0, 2] and not kept[2, 0]
    assert kept[1, 2] and kept[2, 1]
    assert np.array_equal(Y, _single_entry(3, 1, 2, 3.0 * TAU))


def test_diagonal_block_below_threshold_is_kept():
    X = np.zeros((3 * B, 3 * B))
    X[B + 1, B + 3] = X[B + 3, B + 1] = TAU / 8
    X[2 * B, 2 * B] = TAU / 1024
    Y = dense.block_truncation_mask(B, TAU)(X)
    assert np.array_equal(Y, X)


def test_decision_follows_the_upper_block():
    # upper block below tau, its mirror above: both dropped; the other way round: both kept
    X = _single_entry(2, 0, 1, TAU / 2, mirror=False)
    X[B + 2, 1] = 4.0 * TAU
    assert not np.any(dense.block_truncation_mask(B, TAU)(X))
    X = _single_entry(2, 0, 1, 4.0 * TAU, mirror=False)
    X[B + 2, 1] = TAU / 2
    assert np.array_equal(dense.block_truncation_mask(B, TAU)(X), X)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mask_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    nb, b = 9, 3
    n = nb * b
    scale = 10.0 ** rng.uniform(-9, -3, size=(nb, nb))
    X = rng.standard_normal((n, n)) * np.kron(scale, np.ones((b, b)))
    X = 0.5 * (X + X.T)
    tau = 1e-6
    want = np.zeros_like(X)
    for I in range(nb):
        for J in range(nb):
            lo, hi = min(I, J), max(I, J)
            up = X[lo * b:(lo + 1) * b, hi * b:(hi + 1) * b]
            norm = math.sqrt(sum(float(v) * float(v) for v in up.ravel()))
            if I == J or norm >= tau:
                want[I * b:(I + 1) * b, J * b:(J + 1) * b] = X[I * b:(I + 1) * b,
                                                               J * b:(J + 1) * b]
    got = dense.block_truncation_mask(b, tau)(X)
    assert np.array_equal(got, want)
    kept = _blocks_kept(got, b)
    assert 0 < kept.sum() < nb * nb                       # the case is not trivial


@pytest.mark.parametrize("n,n_occ", [(1, 1), (7, 3), (40, 17), (64, 32)])
def test_projector_entries_match_full_projector(n, n_occ):
    rng = np.random.default_rng(n)
    lam = rng.uniform(-1.0, 1.0, n)                       # unsorted on purpose
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    D = exact.projector(n_occ=n_occ, eigvals=lam, Q=q)
    rows = rng.integers(0, n, 200)
    cols = rng.integers(0, n, 200)
    got = exact.projector_entries(q, lam, n_occ, rows, cols)
    assert np.max(np.abs(got - D[rows, cols])) <= 1e-14
    # the same projector from numpy's eigendecomposition of F = Q diag(lam) Q^T
    F = (q * lam) @ q.T
    D2 = exact.projector(F=0.5 * (F + F.T), n_occ=n_occ)
    assert np.max(np.abs(D2 - D)) <= 1e-10
    # all entries: the diagonal sums to N_occ
    ii = np.arange(n)
    assert abs(float(np.sum(exact.projector_entries(q, lam, n_occ, ii, ii))) - n_occ) <= 1e-12
