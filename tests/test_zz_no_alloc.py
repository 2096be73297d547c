"""snf_purify_dense_noalloc (the entry point that allocates nothing) against snf_purify_dense.

Both are called through the C ABI.  Two calls in a row of the no-allocation entry point, the
second with a smaller order (its buffers then hold the first call's values beyond the second
call's order), must each give what the allocating entry point gives: the same status,
branches and product count, and D bit for bit (same kernels on the same decomposition); D is
also held to the FP64 parity bar against the oracle.  Orders above the limit, other precisions
and the P_{i,j} schemes are rejected without touching D.
"""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense  # noqa: E402
from paper_1101_0265_amd import hamiltonians as H  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_0265_amd import snf as s
    s.lib()
    return s


def _kw(h):
    return dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
                lumo=h.lumo, mu=h.mu, xi=h.xi, tol=1e-10, max_iter=120)


def _call(snf, entry, F, scheme, kw, precision="fp64", ld=None):
    """One call of ``entry`` through the C ABI; F may be a column slice (row stride ld)."""
    L = snf.lib()
    n = F.shape[0]
    ld = F.stride(0) if ld is None else ld
    D_full = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda:0")
    D = D_full[:, :n]
    p = snf.make_params(**kw)
    res = snf.Result()
    logs = (snf.LogRec * snf.LOG_MAX)()
    rc = getattr(L, entry)(F.data_ptr(), n, ld, ctypes.byref(p), snf.SCHEMES[scheme],
                           snf.PRECISIONS[precision], D.data_ptr(), ctypes.byref(res), logs,
                           snf.LOG_MAX, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return rc, D_full, snf.result_dict(res, logs)


def _hamiltonian(n, seed):
    return H.random_spectrum_hamiltonian(n, n // 2 - 3, -1.0, -0.04, 0.04, 1.0, seed)


@pytest.mark.parametrize("scheme", ["snf_varmu", "sp2", "snf_fixmu", "snf_fixmu3"])
def test_two_calls_match_the_allocating_entry_point(snf, scheme):
    # 700 pads to 768 (a launch per step); 200 pads to 256 (the cooperative whole-solve
    # launch, except for P_{3,3}, which launches per step at every order)
    hs = [_hamiltonian(700, 11), _hamiltonian(200, 12)]
    Fs = [torch.tensor(h.F, device="cuda:0") for h in hs]
    got = [_call(snf, "snf_purify_dense_noalloc", F, scheme, _kw(h)) for F, h in zip(Fs, hs)]
    ref = [_call(snf, "snf_purify_dense", F, scheme, _kw(h)) for F, h in zip(Fs, hs)]
    for h, (rc_b, D_b, r_b), (rc_a, D_a, r_a) in zip(hs, got, ref):
        assert rc_b == rc_a == snf.OK, (rc_b, rc_a)
        assert r_b["status"] == r_a["status"] == "ok"
        assert r_b["branches"] == r_a["branches"] and r_b["products"] == r_a["products"]
        assert r_b["iterations"] == r_a["iterations"]
        assert r_b["idem_err"] == r_a["idem_err"] and r_b["trace"] == r_a["trace"]
        assert torch.equal(D_b, D_a)
        o = dense.purify(h.F, scheme, **_kw(h))
        assert r_b["branches"] == o["branches"] and r_b["products"] == o["products"]
        assert np.linalg.norm(D_b.cpu().numpy() - o["D"]) <= 1e-8 * math.sqrt(h.n)
        assert r_b["device_ms"] > 0.0


def test_row_stride_and_maximum_order(snf):
    # the largest accepted order (896) with a row stride larger than n, then a small one
    h = _hamiltonian(896, 21)
    big = torch.zeros((896, 960), dtype=torch.float64, device="cuda:0")
    big[:, :896] = torch.tensor(h.F, device="cuda:0")
    F = big[:, :896]
    rc_b, D_b, r_b = _call(snf, "snf_purify_dense_noalloc", F, "snf_varmu", _kw(h), ld=960)
    rc_a, D_a, r_a = _call(snf, "snf_purify_dense", F, "snf_varmu", _kw(h), ld=960)
    assert rc_b == rc_a == snf.OK
    assert torch.equal(D_b, D_a)
    assert torch.all(D_b[:, 896:] == 7.0)             # the stride's tail is not written
    h2 = _hamiltonian(40, 22)
    F2 = torch.tensor(h2.F, device="cuda:0")
    rc_b, D_b, r_b = _call(snf, "snf_purify_dense_noalloc", F2, "tc2", _kw(h2))
    rc_a, D_a, r_a = _call(snf, "snf_purify_dense", F2, "tc2", _kw(h2))
    assert rc_b == rc_a == snf.OK and torch.equal(D_b, D_a)


def test_rejections_leave_D_untouched(snf):
    h = _hamiltonian(897, 31)                          # pads to 1024 > 896
    F = torch.tensor(h.F, device="cuda:0")
    rc, D, r = _call(snf, "snf_purify_dense_noalloc", F, "snf_varmu", _kw(h))
    assert rc == snf.ESIZE and r["status"] == "esize"
    assert torch.all(D == 7.0)
    assert "maximum" in snf.strerror(snf.ESIZE)
    h = _hamiltonian(300, 32)
    F = torch.tensor(h.F, device="cuda:0")
    for prec in ("fp32", "fp32_ref64", "bf16_ref64"):
        rc, D, _ = _call(snf, "snf_purify_dense_noalloc", F, "snf_varmu", _kw(h), precision=prec)
        assert rc == snf.EINVAL and torch.all(D == 7.0), prec
    kw = dict(_kw(h), poly_ij=(3, 1), mu=0.0, xi=0.08)
    rc, D, _ = _call(snf, "snf_purify_dense_noalloc", F, "snf_pij", kw)
    assert rc == snf.EINVAL and torch.all(D == 7.0)
