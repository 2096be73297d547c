"""Pins of the bound estimators of the CPU oracle (no GPU): Lanczos Ritz values against a
symmetric eigensolver, the interlacing and residual enclosures, gap-edge bounds against the
exact edges, Gershgorin enclosure, and purification driven by estimated bounds."""
import numpy as np
import pytest

from oracle import bounds, dense, exact
from paper_1101_0265_amd import hamiltonians as H


def _rand_sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return 0.5 * (A + A.T), rng.standard_normal(n)


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_full_lanczos_reproduces_the_spectrum(n):
    F, v0 = _rand_sym(n, n)
    al, be = bounds.lanczos(lambda v: F @ v, v0, n)
    a, b, k, _ = bounds.truncate_tridiagonal(al, be)
    T = np.diag(a) + np.diag(b[:k - 1], 1) + np.diag(b[:k - 1], -1)
    w = np.linalg.eigvalsh(F)
    assert k == n
    assert np.allclose(np.linalg.eigvalsh(T), w, atol=1e-10 * np.max(np.abs(w)))


@pytest.mark.parametrize("steps", [5, 15, 30])
def test_ritz_interlacing_and_residual_enclosure(steps):
    F, v0 = _rand_sym(120, 3)
    w = np.linalg.eigvalsh(F)
    tmin, rmin, tmax, rmax = bounds.ritz_extremes(*bounds.lanczos(lambda v: F @ v, v0, steps))
    assert w[0] <= tmin + 1e-12 and tmax <= w[-1] + 1e-12          # Ritz values inside
    # an eigenvalue within the residual of each extreme Ritz value
    assert np.min(np.abs(w - tmax)) <= rmax * (1 + 1e-9) + 1e-12
    assert np.min(np.abs(w - tmin)) <= rmin * (1 + 1e-9) + 1e-12


def test_spectral_bounds_enclose_after_convergence():
    h = H.random_spectrum_hamiltonian(300, 140, -1.3, -0.1, 0.05, 0.9, seed=4)
    for steps in (40, 80, 120, 300):
        lo, hi = bounds.spectral_bounds(h.F, np.random.default_rng(1).standard_normal(300),
                                        steps)
        assert lo <= h.lambda_min and hi >= h.lambda_max
    assert h.lambda_min - lo < 1e-10 and hi - h.lambda_max < 1e-10


@pytest.mark.parametrize("steps", [4, 12, 200])
def test_gap_bounds_bound_the_edges(steps):
    h = H.random_spectrum_hamiltonian(200, 90, -1.0, -0.04, 0.03, 1.2, seed=9)
    D = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    v0 = np.random.default_rng(2).standard_normal(200)
    homo, lumo = bounds.gap_bounds(h.F, D, h.lambda_min, h.lambda_max, v0, steps)
    assert homo <= h.homo and lumo >= h.lumo
    if steps == 200:
        assert abs(homo - h.homo) < 1e-10 and abs(lumo - h.lumo) < 1e-10


def test_gershgorin_encloses():
    for seed in range(5):
        F, _ = _rand_sym(50, seed)
        lo, hi = bounds.gershgorin(F)
        w = np.linalg.eigvalsh(F)
        assert lo <= w[0] and hi >= w[-1]


def test_purification_with_estimated_bounds():
    """Trace scheme with Lanczos extremal bounds, then scale-and-fold with gap bounds from its
    D: the same projector as with exact bounds, at most two more products (bounds paragraph:
    loose bounds cost some efficiency, never correctness)."""
    h = H.random_spectrum_hamiltonian(160, 70, -1.0, 0.02, 0.08, 1.0, seed=12)
    v0 = np.random.default_rng(3).standard_normal(160)
    lo, hi = bounds.spectral_bounds(h.F, v0, 30)
    r1 = dense.purify(h.F, "sp2", lambda_min=lo, lambda_max=hi, n_occ=h.n_occ, tol=1e-11)
    homo, lumo = bounds.gap_bounds(h.F, r1["D"], lo, hi, v0, 30)
    r2 = dense.purify(h.F, "snf_varmu", lambda_min=lo, lambda_max=hi, homo=homo, lumo=lumo,
                      n_occ=h.n_occ, tol=1e-11)
    ref = dense.purify(h.F, "snf_varmu", lambda_min=h.lambda_min, lambda_max=h.lambda_max,
                       homo=h.homo, lumo=h.lumo, n_occ=h.n_occ, tol=1e-11)
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert r2["status"] == "ok" and np.linalg.norm(r2["D"] - D_ref) < 1e-9
    assert r2["products"] <= ref["products"] + 2
