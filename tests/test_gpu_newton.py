"""Subspace correction (SNF_FLAG_SUBSPACE_NEWTON) on the GPU against the CPU oracle.

* FP64 parity: an FP64 solve stopped early (tol 1e-3, so its result is far from a projector
  and the correction has real work to do) is corrected in FP64 on the device; the oracle's
  newton_correct applied to the same uncorrected result (a second call without the flag;
  the path is deterministic) gives the same D within the FP64 parity bar, with the same number
  of correction products.
* FP32 products with FP64 refinement: the correction removes the subspace error that
  refinement by purification leaves (a few percent of it remains at most), and the result stays
  within an FP32 bound of the oracle's correction of the same input:
  ||D - D_oracle||_F <= 4 N u32 sqrt(n) / g0 x ||D~ - D_exact||_F (N response steps, each
  rounding the response to FP32 with an amplification of at most 1 / g0, the initial X-space
  gap).
* Argument checks: the flag needs n_occ and gap edges.
"""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import correction as corr  # noqa: E402
from oracle import exact  # noqa: E402
from paper_1101_0265_amd import hamiltonians as H  # noqa: E402

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def snf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_0265_amd import snf as s
    s.lib()
    return s


def _kw(h, **extra):
    d = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
             lumo=h.lumo, mu=h.mu, xi=h.xi, tol=1e-10, max_iter=120)
    d.update(extra)
    return d


def _okw(h):
    return dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, homo=h.homo, lumo=h.lumo,
                n_occ=h.n_occ)


@pytest.mark.parametrize("n,n_occ,scheme", [(300, 140, "snf_varmu"), (517, 260, "sp2"),
                                            (1000, 480, "tc2")])
def test_fp64_correction_matches_oracle(snf, n, n_occ, scheme):
    h = H.random_spectrum_hamiltonian(n, n_occ, -1.0, -0.02, 0.03, 1.0, seed=n)
    F = torch.tensor(h.F, device="cuda:0")
    Dt, r0 = snf.purify_dense(F, scheme, **_kw(h, tol=1e-3))
    Dt = Dt.cpu().numpy()
    D, r = snf.purify_dense(F, scheme, flags=snf.FLAG_SUBSPACE_NEWTON, **_kw(h, tol=1e-3))
    o = corr.newton_correct(h.F, Dt, tol=1e-3, **_okw(h))
    steps = corr.alg2_steps(h.lambda_min, h.lambda_max, h.homo, h.lumo, 1e-10)
    assert r["status"] == "ok"
    assert r["branches"] == r0["branches"]
    # the correction's products: W, M, then a response product and a square per step, then
    # the refinement's products (the certifying one included)
    assert r["products"] == r0["products"] + r["products_newton"]
    assert r["products_newton"] == 2 + 2 * len(steps) + o["refine_products"]
    err = float(np.linalg.norm(D.cpu().numpy() - o["D"]))
    print(f"\nn={n} {scheme}: {len(steps)} response steps, ||D - D_oracle||_F = {err:.2e}")
    assert err <= 1e-8 * math.sqrt(n)
    # the refinement stops at tol; the eigenvalues of D then lie within ||D^2 - D||_F of 0 or 1
    assert r["idem_err"] <= 1e-3 and abs(r["trace_err"]) <= math.sqrt(n) * 1e-3


@pytest.mark.parametrize("gsw", [0.0, 0.5])
def test_fp32_correction_removes_the_subspace_error(snf, gsw):
    n, n_occ = 640, 300
    h = H.random_spectrum_hamiltonian(n, n_occ, -1.0, 0.0, 0.004, 1.0, seed=77)
    F = torch.tensor(h.F, device="cuda:0")
    kw = _kw(h, gap_switch=gsw, tol=1e-10)
    Dt, r0 = snf.purify_dense(F, "snf_varmu", "fp32_ref64", **kw)
    D, r = snf.purify_dense(F, "snf_varmu", "fp32_ref64", flags=snf.FLAG_SUBSPACE_NEWTON, **kw)
    D_exact = exact.projector(n_occ=n_occ, eigvals=h.eigvals, Q=h.Q)
    before = float(np.linalg.norm(Dt.cpu().numpy() - D_exact))
    after = float(np.linalg.norm(D.cpu().numpy() - D_exact))
    o = corr.newton_correct(h.F, Dt.cpu().numpy(), tol=1e-10, **_okw(h))
    to_oracle = float(np.linalg.norm(D.cpu().numpy() - o["D"]))
    N = len(corr.alg2_steps(h.lambda_min, h.lambda_max, h.homo, h.lumo, 1e-10))
    g0 = (h.lumo - h.homo) / (h.lambda_max - h.lambda_min)
    bound = 4.0 * N * U32 * math.sqrt(n) / g0 * before
    print(f"\nfp32_ref64 gap_switch={gsw}: ||D~ - D||_F = {before:.2e} -> {after:.2e} "
          f"(oracle's correction {np.linalg.norm(o['D'] - D_exact):.2e}); "
          f"||D - D_oracle||_F = {to_oracle:.2e} ({to_oracle / bound:.3f} of the bound)")
    assert r["status"] == "ok" and r["idem_err"] <= 1e-10
    assert abs(r["trace_err"]) <= 1e-8
    assert r["products_lowp"] > r0["products_lowp"]
    assert before > 1e-6                      # there was a subspace error to remove
    assert after <= 0.05 * before
    assert to_oracle <= bound


def test_flag_needs_occupation_and_gap_edges(snf):
    h = H.random_spectrum_hamiltonian(128, 60, -1.0, -0.05, 0.05, 1.0, seed=5)
    F = torch.tensor(h.F, device="cuda:0")
    L = snf.lib()
    D = torch.empty_like(F)
    stream = torch.cuda.current_stream().cuda_stream
    for bad in (dict(n_occ=-1), dict(homo=float("nan"), lumo=float("nan"), mu=float("nan"))):
        kw = _kw(h, flags=snf.FLAG_SUBSPACE_NEWTON)
        kw.update(bad)
        p = snf.make_params(**kw)
        res = snf.Result()
        rc = L.snf_purify_dense(F.data_ptr(), 128, 128, ctypes.byref(p), snf.SCHEMES["tc2"], 0,
                                D.data_ptr(), ctypes.byref(res), None, 0, stream)
        assert rc == snf.EINVAL and res.status == snf.EINVAL, bad
    # fixed-mu schemes: the gap edges come from mu and xi
    Dn, r = snf.purify_dense(F, "snf_fixmu", flags=snf.FLAG_SUBSPACE_NEWTON,
                             **_kw(h, homo=float("nan"), lumo=float("nan")))
    assert r["status"] == "ok" and r["products_newton"] > 0
    D_exact = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert np.linalg.norm(Dn.cpu().numpy() - D_exact) <= 1e-8 * math.sqrt(h.n)


def test_gap1e3_8192_fp32_correction(snf):
    """n = 8192, gap 1e-3 at mu = 0.1 (the precision workload; Haar Q drawn on the device):
    FP32 products from the start with FP64 refinement leave ||D~ - D_exact||_F of a few 1e-3;
    the correction takes it down by at least 100x."""
    n, n_occ = 8192, 4506
    lam = H.two_interval_spectrum(n_occ, n - n_occ, -1.0, 0.0995, 0.1005, 1.0,
                                  np.random.default_rng(4))
    F, Q = H.rotated_spectrum_torch(lam, seed=4)
    qo = Q[:, :n_occ].contiguous()
    D_exact = qo @ qo.T
    del Q, qo
    kw = dict(lambda_min=-1.0, lambda_max=1.0, n_occ=n_occ, homo=0.0995, lumo=0.1005,
              tol=1e-8, max_iter=200, gap_switch=0.0)
    D, r0 = snf.purify_dense(F, "snf_varmu", "fp32_ref64", **kw)
    before = float(torch.linalg.norm(D - D_exact))
    D, r = snf.purify_dense(F, "snf_varmu", "fp32_ref64", out=D, flags=snf.FLAG_SUBSPACE_NEWTON,
                            **kw)
    after = float(torch.linalg.norm(D - D_exact))
    print(f"\nn=8192 gap 1e-3 fp32_ref64: ||D~ - D||_F = {before:.2e} -> {after:.2e} with "
          f"{r['products_newton']} correction products")
    assert r["status"] == "ok" and r["idem_err"] <= 1e-8
    assert before > 1e-4
    assert after <= before / 100.0
