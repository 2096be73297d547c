"""Precision modes (FP32 / BF16 products, FP64 refinement) against the FP64 oracle.

The paper reasons in exact arithmetic; low-precision products leave an error in the occupied
subspace that a refinement by purification cannot remove (it restores idempotency and the
trace only).  So the bars here are: the refined result is idempotent to tol and has the right
trace (like FP64), the phase sequence is FP64 -> low precision -> FP64 refinement, and the
distance to the FP64 oracle's D is *stated* (printed) and kept under a loose ceiling that
catches a broken kernel, not under the FP64 parity tolerance.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense, exact  # noqa: E402
from paper_1101_0265_amd import hamiltonians as H  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_0265_amd import snf as s
    s.lib()
    return s


def _kw(h, tol=1e-9, **extra):
    d = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
             lumo=h.lumo, mu=h.mu, xi=h.xi, tol=tol, max_iter=150)
    d.update(extra)
    return d


def _oracle_kw(kw):
    return {k: v for k, v in kw.items() if k not in ("gap_switch", "lowp_floor")}


def _phases(log):
    seq = []
    for rec in log:
        if not seq or seq[-1] != rec["phase"]:
            seq.append(rec["phase"])
    return seq


@pytest.mark.parametrize("scheme", ["snf_varmu", "snf_fixmu", "sp2", "tc2"])
@pytest.mark.parametrize("prec,gsw,ceiling", [("fp32_ref64", 0.0, 1e-3),
                                              ("fp32_ref64", 0.9, 1e-4),
                                              ("bf16_ref64", 0.5, 0.5),
                                              ("bf16_ref64", 0.9, 0.3)])
def test_refined_modes(snf, scheme, prec, gsw, ceiling):
    h = H.random_spectrum_hamiltonian(384, 170, -1.0, 0.02, 0.07, 1.0, seed=12)
    kw = _kw(h, gap_switch=gsw)
    D, r = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), scheme, prec, **kw)
    assert r["status"] == "ok", r["status"]
    assert r["idem_err"] <= kw["tol"] and abs(r["trace_err"]) <= 1e-8
    assert r["products_lowp"] > 0 and r["products_fp64"] > 0
    assert r["products_lowp"] + r["products_fp64"] == r["products"]
    ph = _phases(r["log"])
    assert ph in ([1, 2], [0, 1, 2]), ph           # (FP64 ->) low precision -> refinement
    lowp = [rec["precision"] for rec in r["log"] if rec["phase"] == 1]
    assert set(lowp) == {1 if prec.startswith("fp32") else 2}
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    o = dense.purify(h.F, scheme, **_oracle_kw(kw))
    err_oracle = float(np.linalg.norm(D.cpu().numpy() - o["D"]))
    err_exact = float(np.linalg.norm(D.cpu().numpy() - D_ref))
    Fd = torch.tensor(h.F, device="cuda:0")
    comm = float(torch.linalg.norm(Fd @ D - D @ Fd))
    print(f"\n{scheme} {prec} gap_switch={gsw}: products {r['products']} "
          f"(lowp {r['products_lowp']}, fp64 {r['products_fp64']}), "
          f"|D-D_oracle|_F={err_oracle:.2e} |D-D_exact|_F={err_exact:.2e} "
          f"|[F,D]|_F={comm:.2e}")
    assert err_oracle <= ceiling


def test_fp32_only_stops_at_floor(snf):
    h = H.random_spectrum_hamiltonian(300, 140, -1.0, 0.0, 0.05, 1.0, seed=3)
    kw = _kw(h, tol=1e-12)
    D, r = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), "snf_varmu", "fp32", **kw)
    assert r["status"] in ("ok_floor", "ok")
    assert r["products_fp64"] == 0
    assert r["idem_err"] <= 1e-3 and abs(r["trace_err"]) <= 1e-2
    o = dense.purify(h.F, "snf_varmu", **_oracle_kw(kw))
    print(f"\nfp32-only: status {r['status']} e={r['idem_err']:.2e} "
          f"|D-D_oracle|_F={np.linalg.norm(D.cpu().numpy() - o['D']):.2e}")


def test_gap_switch_one_is_all_fp64_then_refine(snf):
    """gap_switch = 1: the X-space gap never reaches 1, so every product stays FP64."""
    h = H.random_spectrum_hamiltonian(200, 90, -1.0, 0.0, 0.05, 1.0, seed=5)
    kw = _kw(h, gap_switch=1.0)
    D, r = snf.purify_dense(torch.tensor(h.F, device="cuda:0"), "snf_varmu", "fp32_ref64", **kw)
    o = dense.purify(h.F, "snf_varmu", **_oracle_kw(kw))
    assert r["products_lowp"] == 0
    assert r["branches"] == o["branches"]
    assert np.linalg.norm(D.cpu().numpy() - o["D"]) <= 1e-8 * math.sqrt(h.n)
