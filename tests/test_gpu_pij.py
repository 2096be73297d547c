"""GPU parity of the asymmetric fixed-mu schemes (P_{i,j}, i and j odd, scaled about the
polynomial's fixed point x*, and their alpha = 1 forms) against the CPU oracle, through the
C ABI.

The device evaluates P(x* + v) = x* + v Q(v) by Horner's rule in W = v^2 with coefficients
linear in v ((i + j)/2 + 1 products; the first product also writes the top Horner level as a
second epilogue output) and solves each side's Eq. 3 by bisection on the incomplete-beta form
of P_{i,j}; the oracle finds x* by exact bisection, evaluates the polynomial by Horner's rule
in X_s on exact coefficients and bisects on the monomial form.  Bars: branch letters,
iteration and product counts and status identical; alpha within 1e-12 relative; the two
tracked bounds within 1e-10 relative (the same conditioning as the P_{m,m} schemes); traces
and idempotency as for the other dense schemes; ||D_gpu - D_oracle||_F <= 1e-8 sqrt(n).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense, exact  # noqa: E402
from paper_1101_0265_amd import hamiltonians as H  # noqa: E402

pytestmark = pytest.mark.gpu

PAIRS = [(1, 3), (3, 1), (1, 5), (5, 1), (3, 5), (5, 3)]


@pytest.fixture(scope="module")
def snf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_0265_amd import snf as s
    s.lib()
    return s


def _off_centre(n=256, seed=1101, mu=-0.5, gap=0.05):
    """Spectrum in [-1, 1] with the gap centred at mu (a quarter of the way up for mu = -0.5,
    as in the paper's McWeeny illustration); n_occ in proportion."""
    n_occ = int(round(n * (mu + 1.0) / 2.0))
    return H.random_spectrum_hamiltonian(n, n_occ, -1.0, mu - gap / 2, mu + gap / 2, 1.0,
                                         seed=seed, name=f"dense-n{n}-mu{mu}")


def _kw(h, pij, tol=1e-10, max_iter=120):
    return dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ,
                mu=h.mu, xi=h.xi, tol=tol, max_iter=max_iter, poly_ij=pij)


def _compare(snf, h, scheme, pij, tol=1e-10):
    kw = _kw(h, pij, tol)
    print(f"\n{scheme} P_{pij} n={h.n} n_occ={h.n_occ}", flush=True)
    D, r = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), scheme, **kw)
    o = dense.purify(h.F, scheme, **kw)
    n = h.n
    assert r["status"] == o["status"] == "ok", (r["status"], o["status"])
    assert r["branches"] == o["branches"] == "P" * o["iterations"]
    assert r["iterations"] == o["iterations"] and r["products"] == o["products"]
    for a, b in zip(r["log"], o["log"]):
        assert abs(a["beta"] - b["beta"]) <= 1e-10 * b["beta"] + 1e-300
        abar_g, abar_o = 1.0 - a["betabar"], 1.0 - b["betabar"]
        assert abs(abar_g - abar_o) <= 1e-10 * abar_o + 4e-16
        if "alpha" in b:
            assert abs(a["alpha"] - b["alpha"]) <= 1e-12 * b["alpha"]
        assert abs(a["t1"] - b["t1"]) <= 1e-9 * max(1.0, abs(b["t1"]))
        assert abs(a["t2"] - b["t2"]) <= 1e-9 * max(1.0, abs(b["t2"]))
        assert abs(a["e"] - b["e"]) <= 1e-8 * b["e"] + 1e-11 * math.sqrt(n)
    Dg = D.cpu().numpy()
    assert np.linalg.norm(Dg - o["D"]) <= 1e-8 * math.sqrt(n)
    assert np.array_equal(Dg, Dg.T)
    return Dg, r, o


@pytest.mark.parametrize("i,j", PAIRS)
def test_off_centre_256_parity(snf, i, j):
    h = _off_centre()
    Dg, r, o = _compare(snf, h, "snf_pij", (i, j))
    assert r["products"] == ((i + j) // 2 + 1) * r["iterations"] + 1
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert np.linalg.norm(Dg - D_ref) <= 1e-8 * math.sqrt(h.n)
    assert abs(r["trace_err"]) < 1e-8
    print(f"snf_pij P_{i}{j}: {r['iterations']} iterations, {r['products']} products, "
          f"e={r['idem_err']:.2e}")


@pytest.mark.parametrize("i,j", [(3, 1), (1, 5), (5, 3)])
def test_unscaled_parity(snf, i, j):
    _compare(snf, _off_centre(mu=0.3), "pij", (i, j))


@pytest.mark.parametrize("n,n_occ", [(130, 61), (300, 190), (17, 5)])
@pytest.mark.parametrize("pij", [(3, 1), (1, 3), (3, 5)])
def test_ragged_sizes_parity(snf, n, n_occ, pij):
    mu, gap = 0.15, 0.06
    h = H.random_spectrum_hamiltonian(n, n_occ, -1.0, mu - gap / 2, mu + gap / 2, 1.2,
                                      seed=n * 7 + n_occ)
    _compare(snf, h, "snf_pij", pij)


def test_whole_tile_and_split_epilogues_2944(snf):
    """n = 2944: 276 upper-triangle tiles, 256 of them computed whole (the second output from
    the product kernel's own epilogue) and 20 split into k-slices (the second output from the
    fix-up's epilogue); smaller orders split every tile."""
    h = _off_centre(n=2944, seed=7, mu=-0.4, gap=0.04)
    _compare(snf, h, "snf_pij", (3, 1))


@pytest.mark.parametrize("m,ref", [(1, "snf_fixmu"), (3, "snf_fixmu3")])
def test_symmetric_pair_agrees_with_pmm_path(snf, m, ref):
    """i = j through the general evaluation: same counts as the dedicated path and the
    exact projector."""
    h = H.small_gap_256()
    F = torch.tensor(h.F, device="cuda:0")
    D1, r1 = snf.purify_dense(F, "snf_pij", **_kw(h, (m, m)))
    D2, r2 = snf.purify_dense(F, ref, **_kw(h, None))
    assert r1["status"] == r2["status"] == "ok"
    assert r1["iterations"] == r2["iterations"] and r1["products"] == r2["products"]
    for a, b in zip(r1["log"], r2["log"]):
        if b["branch"] is not None:
            assert a["alpha"] == pytest.approx(b["alpha"], rel=1e-12)
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert np.linalg.norm(D1.cpu().numpy() - D_ref) <= 1e-8 * math.sqrt(h.n)
    assert np.linalg.norm(D1.cpu().numpy() - D2.cpu().numpy()) <= 1e-8 * math.sqrt(h.n)


def test_matching_polynomial_is_cheaper_off_centre(snf):
    """mu a quarter of the way up: P_{3,1} (x* = 0.87, room for the long unoccupied part)
    needs fewer products than its mirror P_{1,3}."""
    h = _off_centre(mu=-0.5, gap=0.01)
    F = torch.tensor(h.F, device="cuda:0")
    _, r31 = snf.purify_dense(F, "snf_pij", **_kw(h, (3, 1)))
    _, r13 = snf.purify_dense(F, "snf_pij", **_kw(h, (1, 3)))
    assert r31["status"] == r13["status"] == "ok"
    assert r31["products"] < r13["products"]


def test_rejects_bad_polynomials_modes_and_paths(snf):
    h = _off_centre()
    F = torch.tensor(h.F, device="cuda:0")
    for bad in [(2, 1), (1, 4), (7, 1), (0, 3), None]:
        with pytest.raises(RuntimeError):
            snf.purify_dense(F, "snf_pij", **_kw(h, bad))
    with pytest.raises(RuntimeError):
        snf.purify_dense(F, "snf_pij", "fp32_ref64", **_kw(h, (3, 1)))
    # P_{1,5} puts mu at x* = 0.058; with gamma = 25.9 a gap of 3.5 puts the lower gap edge
    # below 0, outside the unit interval
    kw = _kw(h, (1, 5))
    kw["xi"] = 3.5
    with pytest.raises(RuntimeError):
        snf.purify_dense(F, "snf_pij", **kw)
    srv = snf.Server(64 << 20, max_slots=4)
    try:
        with pytest.raises(RuntimeError):            # served in FP64 only
            srv.submit(h.F, "snf_pij", "fp32_ref64", **_kw(h, (3, 1)))
        with pytest.raises(RuntimeError):            # checked as for the dense path
            srv.submit(h.F, "snf_pij", **_kw(h, (2, 1)))
    finally:
        srv.close()
