"""GPU bound estimators (Lanczos on the device, C ABI) against the CPU oracle.

Bars: with the same start vector the bounds equal the oracle's within 1e-9 of the spectral
width (both run the same recurrence in FP64; only summation orders differ); the Gershgorin
enclosure within 1e-12; the enclosure properties (outer extremal bounds after convergence,
gap bounds never inside the gap) hold exactly; a solve driven by estimated bounds reaches the
exact projector with at most two more products than with exact bounds.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bounds, dense, exact  # noqa: E402
from paper_1101_0265_amd import hamiltonians as H  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_0265_amd import snf as s
    s.lib()
    return s


def _dev(a):
    return torch.tensor(a, device="cuda:0", dtype=torch.float64)


@pytest.mark.parametrize("n,steps", [(17, 40), (130, 30), (300, 60), (1000, 50)])
def test_spectral_bounds_match_oracle(snf, n, steps):
    h = H.random_spectrum_hamiltonian(n, n // 2, -1.2, -0.05, 0.05, 0.9, seed=n)
    v0 = np.random.default_rng(n).standard_normal(n)
    lo, hi, glo, ghi = snf.spectral_bounds(_dev(h.F), steps, start=_dev(v0))
    olo, ohi = bounds.spectral_bounds(h.F, v0, steps)
    ogl, ogh = bounds.gershgorin(h.F)
    width = h.lambda_max - h.lambda_min
    assert abs(lo - olo) <= 1e-9 * width and abs(hi - ohi) <= 1e-9 * width, (lo, olo, hi, ohi)
    assert abs(glo - ogl) <= 1e-12 * width and abs(ghi - ogh) <= 1e-12 * width
    assert glo <= h.lambda_min and ghi >= h.lambda_max
    if n == 17:       # breakdown at k = n: the Ritz values are the eigenvalues
        assert h.lambda_min - lo <= 1e-12 and hi - h.lambda_max <= 1e-12
        assert lo <= h.lambda_min and hi >= h.lambda_max


def test_spectral_bounds_enclose_lattice(snf):
    h = H.lattice_hamiltonian((8, 8, 4), seed=2)
    lo, hi, glo, ghi = snf.spectral_bounds(_dev(h.F), 80)
    w = np.linalg.eigvalsh(h.F)
    assert lo <= w[0] and hi >= w[-1]
    assert w[0] - lo < 1e-6 and hi - w[-1] < 1e-6
    assert glo <= lo and ghi >= hi


@pytest.mark.parametrize("steps", [6, 25, 200])
def test_gap_bounds_match_oracle_and_bound_the_edges(snf, steps):
    h = H.random_spectrum_hamiltonian(200, 90, -1.0, -0.04, 0.03, 1.2, seed=9)
    D = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    v0 = np.random.default_rng(2).standard_normal(200)
    homo, lumo = snf.gap_bounds(_dev(h.F), _dev(D), h.lambda_min, h.lambda_max, steps,
                                start=_dev(v0))
    ohomo, olumo = bounds.gap_bounds(h.F, D, h.lambda_min, h.lambda_max, v0, steps)
    width = h.lambda_max - h.lambda_min
    assert abs(homo - ohomo) <= 1e-9 * width and abs(lumo - olumo) <= 1e-9 * width
    assert homo <= h.homo and lumo >= h.lumo
    if steps == 200:
        assert h.homo - homo < 1e-10 and lumo - h.lumo < 1e-10


def test_bounds_drive_a_solve(snf):
    """Trace scheme with device extremal bounds, gap bounds from its D, then scale-and-fold."""
    h = H.random_spectrum_hamiltonian(512, 230, -1.0, 0.02, 0.08, 1.0, seed=12)
    F = _dev(h.F)
    lo, hi, _, _ = snf.spectral_bounds(F, 60)
    assert lo <= h.lambda_min and hi >= h.lambda_max
    D1, r1 = snf.purify_dense(F, "sp2", lambda_min=lo, lambda_max=hi, n_occ=h.n_occ,
                              tol=1e-10, max_iter=100)
    assert r1["status"] == "ok"
    homo, lumo = snf.gap_bounds(F, D1, lo, hi, 60)
    assert homo <= h.homo and lumo >= h.lumo
    D2, r2 = snf.purify_dense(F, "snf_varmu", lambda_min=lo, lambda_max=hi, homo=homo,
                              lumo=lumo, n_occ=h.n_occ, tol=1e-10, max_iter=100)
    _, ref = snf.purify_dense(F, "snf_varmu", lambda_min=h.lambda_min,
                              lambda_max=h.lambda_max, homo=h.homo, lumo=h.lumo,
                              n_occ=h.n_occ, tol=1e-10, max_iter=100)
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert r2["status"] == "ok"
    assert np.linalg.norm(D2.cpu().numpy() - D_ref) <= 1e-8 * math.sqrt(h.n)
    assert r2["products"] <= ref["products"] + 2
    print(f"\nestimated bounds [{lo:.6f}, {hi:.6f}] gap [{homo:.6f}, {lumo:.6f}] "
          f"(exact [{h.lambda_min}, {h.lambda_max}] [{h.homo}, {h.lumo}]): "
          f"{r2['products']} products vs {ref['products']} with exact bounds")


def test_bounds_lattice_4096(snf):
    """The bound pipeline of the n = 4096 lattice workload at full size, with the benchmark's
    40 Lanczos steps: spectral and gap bounds equal the oracle's for the same start vectors,
    enclose the exact extreme levels and gap edges, and the scale-and-fold solve they drive
    reaches the solve with exact bounds."""
    h = H.lattice_hamiltonian((16, 16, 8), seed=2)
    n, steps = h.n, 40
    F = _dev(h.F)
    v0 = np.random.default_rng(40).standard_normal(n)
    v1 = np.random.default_rng(41).standard_normal(n)
    width = h.lambda_max - h.lambda_min
    lo, hi, _, _ = snf.spectral_bounds(F, steps, start=_dev(v0))
    olo, ohi = bounds.spectral_bounds(h.F, v0, steps)
    assert abs(lo - olo) <= 1e-9 * width and abs(hi - ohi) <= 1e-9 * width, (lo, olo, hi, ohi)
    assert lo <= h.lambda_min and hi >= h.lambda_max
    D1, r1 = snf.purify_dense(F, "sp2", lambda_min=lo, lambda_max=hi, n_occ=h.n_occ, tol=1e-8,
                              max_iter=100)
    assert r1["status"] == "ok"
    homo, lumo = snf.gap_bounds(F, D1, lo, hi, steps, start=_dev(v1))
    ohomo, olumo = bounds.gap_bounds(h.F, D1.cpu().numpy(), lo, hi, v1, steps)
    assert abs(homo - ohomo) <= 1e-9 * width and abs(lumo - olumo) <= 1e-9 * width
    assert homo <= h.homo and lumo >= h.lumo
    D2, r2 = snf.purify_dense(F, "snf_varmu", lambda_min=lo, lambda_max=hi, homo=homo,
                              lumo=lumo, n_occ=h.n_occ, tol=1e-8, max_iter=100)
    Dx, rx = snf.purify_dense(F, "snf_varmu", lambda_min=h.lambda_min,
                              lambda_max=h.lambda_max, homo=h.homo, lumo=h.lumo,
                              n_occ=h.n_occ, tol=1e-8, max_iter=100)
    assert r2["status"] == "ok" and rx["status"] == "ok"
    assert float(torch.linalg.norm(D2 - Dx)) <= 1e-7 * math.sqrt(n)
    assert r2["products"] <= rx["products"] + 2
    print(f"\nn=4096 lattice: bounds [{lo:.6f}, {hi:.6f}] gap [{homo:.6f}, {lumo:.6f}] "
          f"(exact [{h.lambda_min:.6f}, {h.lambda_max:.6f}] [{h.homo:.6f}, {h.lumo:.6f}]); "
          f"{r2['products']} products vs {rx['products']} with exact bounds")


def test_bounds_invalid_arguments(snf):
    F = _dev(np.eye(4))
    with pytest.raises(RuntimeError):
        snf.spectral_bounds(F, 0)
    with pytest.raises(RuntimeError):
        snf.spectral_bounds(F, 10000)
    with pytest.raises(RuntimeError):
        snf.gap_bounds(F, F, 1.0, -1.0, 10)
