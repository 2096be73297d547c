"""GPU parity of the higher-order fixed-mu schemes (P_{3,3}, P_{5,5}; scaled by Eq. 3 and
unscaled) against the CPU oracle, through the C ABI.

The device evaluates P_{m,m}(X_s) in m + 1 products from the point symmetry of P_{m,m} and
solves Eq. 3 by bisection on the incomplete-beta form of the polynomial; the oracle evaluates
the polynomial by Horner's rule in X_s on exact coefficients and solves Eq. 3 by bisection on
the monomial form.  Bars: branch letters, iteration and product counts and status identical;
alpha per iteration within 1e-12 relative and beta within 1e-10 relative (the root-finders
agree to an ulp or two, but near convergence beta_s = alpha (beta - 1/2) + 1/2 is a small
difference of O(1) numbers and P_{m,m} raises it to the power m + 1, so rounding differences
in beta grow by a factor of order m + 1 per iteration); traces and idempotency as for the
other dense schemes; ||D_gpu - D_oracle||_F <= 1e-8 sqrt(n).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense, exact  # noqa: E402
from paper_1101_0265_amd import hamiltonians as H  # noqa: E402

pytestmark = pytest.mark.gpu

HO = ("snf_fixmu3", "snf_fixmu5", "pmm3", "pmm5")


@pytest.fixture(scope="module")
def snf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_0265_amd import snf as s
    s.lib()
    return s


def _kw(h, tol=1e-10, max_iter=120):
    return dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ,
                mu=h.mu, xi=h.xi, tol=tol, max_iter=max_iter)


def _compare(snf, h, scheme, tol=1e-10):
    kw = _kw(h, tol)
    D, r = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), scheme, **kw)
    o = dense.purify(h.F, scheme, **kw)
    n = h.n
    assert r["status"] == o["status"] == "ok", (r["status"], o["status"])
    assert r["branches"] == o["branches"]
    assert r["iterations"] == o["iterations"] and r["products"] == o["products"]
    for a, b in zip(r["log"], o["log"]):
        assert abs(a["beta"] - b["beta"]) <= 1e-10 * b["beta"] + 1e-300
        if "alpha" in b:
            assert abs(a["alpha"] - b["alpha"]) <= 1e-12 * b["alpha"]
        assert abs(a["t1"] - b["t1"]) <= 1e-9 * max(1.0, abs(b["t1"]))
        assert abs(a["t2"] - b["t2"]) <= 1e-9 * max(1.0, abs(b["t2"]))
        assert abs(a["e"] - b["e"]) <= 1e-8 * b["e"] + 1e-11 * math.sqrt(n)
    Dg = D.cpu().numpy()
    assert np.linalg.norm(Dg - o["D"]) <= 1e-8 * math.sqrt(n)
    assert np.array_equal(Dg, Dg.T)
    return Dg, r, o


@pytest.mark.parametrize("scheme", HO)
def test_small_gap_256_parity(snf, scheme):
    h = H.small_gap_256()
    Dg, r, o = _compare(snf, h, scheme)
    m = 3 if scheme.endswith("3") else 5
    assert r["products"] == (m + 1) * r["iterations"] + 1
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert np.linalg.norm(Dg - D_ref) <= 1e-8 * math.sqrt(h.n)
    print(f"\n{scheme}: {r['iterations']} iterations, {r['products']} products, "
          f"e={r['idem_err']:.2e}")


@pytest.mark.parametrize("n,n_occ", [(130, 61), (300, 190), (17, 5)])
@pytest.mark.parametrize("scheme", ["snf_fixmu3", "pmm5", "snf_fixmu5"])
def test_ragged_sizes_parity(snf, n, n_occ, scheme):
    mu, gap = 0.15, 0.06
    h = H.random_spectrum_hamiltonian(n, n_occ, -1.0, mu - gap / 2, mu + gap / 2, 1.2,
                                      seed=n * 7 + n_occ)
    _compare(snf, h, scheme)


def test_scaled_needs_fewer_products_than_unscaled(snf):
    h = H.small_gap_256()
    _, r3 = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), "snf_fixmu3", **_kw(h))
    _, p3 = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), "pmm3", **_kw(h))
    _, a1 = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), "snf_fixmu", **_kw(h))
    assert a1["products"] < r3["products"] < p3["products"]


def test_workspace_growth_between_schemes(snf):
    """A P_{m,m} solve needs a fourth buffer: interleave with three-buffer schemes and a larger
    order so the workspace is re-created while the extra buffer exists."""
    h1 = H.random_spectrum_hamiltonian(200, 90, -1.0, -0.05, 0.05, 1.0, seed=1)
    h2 = H.random_spectrum_hamiltonian(400, 150, -1.0, -0.05, 0.05, 1.0, seed=2)
    for h, scheme in [(h1, "snf_fixmu3"), (h2, "snf_varmu"), (h2, "snf_fixmu5"),
                      (h1, "snf_fixmu")]:
        kw = dict(_kw(h), homo=h.homo, lumo=h.lumo)
        D, r = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), scheme, **kw)
        assert r["status"] == "ok"
        D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
        assert np.linalg.norm(D.cpu().numpy() - D_ref) <= 1e-8 * math.sqrt(h.n)


def test_higher_order_rejects_low_precision(snf):
    h = H.small_gap_256()
    F = torch.tensor(h.F, device="cuda:0")
    with pytest.raises(RuntimeError):
        snf.purify_dense(F, "snf_fixmu3", "fp32_ref64", **_kw(h))
    # (the block-sparse path runs them in FP32: tests/test_gpu_bsr.py; serving in FP64:
    # tests/test_gpu_serve.py)
    srv = snf.Server(64 << 20, max_slots=4)
    try:
        with pytest.raises(RuntimeError):
            srv.submit(h.F, "pmm3", "fp32_ref64", **_kw(h))
    finally:
        srv.close()
