"""Block-sparse path (32x32 FP32 blocks, block truncation) against the CPU oracle.

The oracle is the dense FP64 iteration with the same block-truncation rule applied after
every step (`oracle.dense.block_truncation_mask`), on the same (brick/Morton-ordered) matrix.
The GPU computes in FP32 and decides truncation on FP32 block norms, so a block whose norm is
within rounding of the threshold may be kept on one side and dropped on the other; the bars:
* scalar decisions (branch letters) identical -- they depend on the bounds only;
* one step: elementwise within the FP32 dot-product bound, and the kept pattern equal to the
  oracle's except for blocks whose norm is within 1e-4 (relative) of the threshold;
* whole solves: ||D_gpu - D_oracle||_F stated, below 1e-3 sqrt(n) (FP32 + truncation), trace
  and idempotency at the truncation floor.
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


def _dev_bsr(m):
    return (torch.tensor(m.row_ptr, device="cuda:0"), torch.tensor(m.col_idx, device="cuda:0"),
            torch.tensor(m.val, device="cuda:0"))


def _to_dense(rp, ci, va, n, b=32):
    m = H.BSRMatrix(n=n, b=b, row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(),
                    val=va.cpu().numpy())
    return m.to_dense()


def _block_norms(d, b=32):
    nb = d.shape[0] // b
    blk = d.reshape(nb, b, nb, b)
    return np.sqrt(np.einsum("ibjc,ibjc->ij", blk, blk))


@pytest.mark.parametrize("L,tau", [((8, 8, 4), 1e-6), ((8, 8, 4), 1e-2), ((8, 8, 8), 1e-3)])
def test_step_matches_masked_numpy(snf, L, tau):
    m, h = H.lattice_bsr(L, seed=7)
    n = m.n
    Fd = m.to_dense()
    # a symmetric X with the lattice pattern: X_0 of the trace-correcting scheme
    X = (h.lambda_max * np.eye(n) - Fd) / (h.lambda_max - h.lambda_min)
    Xm = H.dense_to_bsr(X, 32)
    # keep F's pattern (dense_to_bsr keeps the same non-zero blocks)
    c2, c1, c0 = -1.44, 2.4, 0.0
    (rp, ci, va), sums, _ = snf.step_bsr(*_dev_bsr(Xm), n, c2, c1, c0, trunc_tau=tau)
    Y = _to_dense(rp, ci, va, n)
    X32 = Xm.to_dense()                      # the FP32 values the GPU used
    P = X32 @ X32
    Yref = c2 * P + c1 * X32 + c0 * np.eye(n)
    norms = _block_norms(Yref)
    nb = n // 32
    keep_ref = (norms >= tau) | np.eye(nb, dtype=bool)
    got = _block_norms(Y) > 0
    got |= np.eye(nb, dtype=bool)
    near = np.abs(norms - tau) <= 1e-4 * tau + 1e-7
    assert np.all((got == keep_ref) | near)
    mask = np.kron(keep_ref & got, np.ones((32, 32), bool))
    bound = (n + 2) * 2.0 ** -24 * (np.abs(X32) @ np.abs(X32)) * abs(c2) + 1e-6
    assert np.all(np.abs(Y - Yref)[mask] <= bound[mask] + 2.0 ** -23 * np.abs(Yref[mask]))
    assert np.array_equal(Y, Y.T)
    assert abs(sums[0] - np.sum((P - X32) ** 2)) <= 1e-4 * np.sum((P - X32) ** 2)
    assert abs(sums[1] - np.trace(Y)) <= 1e-6 * max(1.0, abs(np.trace(Y)))
    assert abs(sums[2] - np.sum(Y * Y)) <= 1e-5 * np.sum(Y * Y)


def test_step_reads_only_upper_blocks(snf):
    """snf_step_bsr reads blocks (I, J) with I <= J and the upper half of diagonal blocks only
    (the documented contract): noise in the lower blocks and in the lower halves of the
    diagonal blocks leaves the result bitwise unchanged."""
    m, h = H.lattice_bsr((8, 8, 4), seed=11)
    n = m.n
    X = (h.lambda_max * np.eye(n) - m.to_dense()) / (h.lambda_max - h.lambda_min)
    Xm = H.dense_to_bsr(X, 32)
    noisy = Xm.val.astype(np.float32).copy()
    rng = np.random.default_rng(5)
    low = np.tril(np.ones((32, 32), bool), -1)
    for i in range(m.nb):
        for p in range(Xm.row_ptr[i], Xm.row_ptr[i + 1]):
            j = Xm.col_idx[p]
            if j < i:
                noisy[p] = rng.standard_normal((32, 32))
            elif j == i:
                noisy[p][low] = rng.standard_normal(int(low.sum()))
    Xn = H.BSRMatrix(n=n, b=32, row_ptr=Xm.row_ptr, col_idx=Xm.col_idx, val=noisy)
    args = (n, -1.44, 2.4, 0.0)
    (rp0, ci0, va0), s0, _ = snf.step_bsr(*_dev_bsr(Xm), *args, trunc_tau=1e-6)
    (rp1, ci1, va1), s1, _ = snf.step_bsr(*_dev_bsr(Xn), *args, trunc_tau=1e-6)
    assert torch.equal(rp0, rp1) and torch.equal(ci0, ci1) and torch.equal(va0, va1)
    assert s0 == s1


@pytest.mark.parametrize("L", [(8, 8, 4), (8, 8, 8), (16, 16, 8)])
@pytest.mark.parametrize("scheme", ["snf_varmu", "sp2", "tc2", "snf_fixmu", "mcweeny"])
def test_purify_bsr_vs_masked_oracle(snf, L, scheme):
    """Algorithm 1 and McWeeny run two products per iteration (S2 = Xs^2, then S2.X); the
    truncation applies to the iteration's result, as the oracle's mask does."""
    tau = 1e-6
    m, h = H.lattice_bsr(L, seed=3)
    n = m.n
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-9, max_iter=60)
    if scheme in ("snf_fixmu", "mcweeny"):
        kw.update(mu=h.mu, xi=h.xi)
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, scheme, trunc_tau=tau, **kw)
    assert r["status"] in ("ok", "ok_floor"), r["status"]
    Dg = _to_dense(rp, ci, va, n)
    Fd = m.to_dense()
    okw = dict(kw)
    okw.update(tol=0.0, max_iter=r["iterations"])
    o = dense.purify(Fd, scheme, mask=dense.block_truncation_mask(32, tau), **okw)
    if scheme != "sp2":
        assert r["branches"] == o["branches"]
    err = float(np.linalg.norm(Dg - o["D"]))
    comm = float(np.linalg.norm(Fd @ Dg - Dg @ Fd))
    print(f"\nBSR {L} {scheme}: status {r['status']} products {r['products']} "
          f"e={r['idem_err']:.2e} blocks {r['nnzb']}/{(n // 32) ** 2} "
          f"|D-D_oracle|_F={err:.2e} |[F,D]|_F={comm:.2e} tr err {r['trace_err']:.2e}")
    assert err <= 1e-3 * math.sqrt(n)
    assert abs(r["trace_err"]) <= 1e-2 and r["idem_err"] <= 1e-3
    assert np.array_equal(Dg, Dg.T)
    if scheme in ("snf_fixmu", "mcweeny"):
        assert r["products"] == 2 * r["iterations"] + 1      # two per iteration + certifying


@pytest.mark.parametrize("L,scheme,pij", [((8, 8, 4), "snf_fixmu3", None),
                                          ((8, 8, 8), "snf_fixmu3", None),
                                          ((8, 8, 4), "snf_fixmu5", None),
                                          ((8, 8, 8), "snf_fixmu5", None),
                                          ((8, 8, 4), "pmm3", None),
                                          ((8, 8, 4), "snf_pij", (1, 3)),
                                          ((8, 8, 8), "snf_pij", (3, 1)),
                                          ((8, 8, 4), "pij", (1, 3))])
def test_purify_bsr_higher_order_vs_masked_oracle(snf, L, scheme, pij):
    """P_{m,m}: W = (a (X - I/2))^2, Horner levels in W, then X.T: m + 1 products per
    iteration on the schedule's buffers, truncation after the last.  P_{i,j}: the first
    product writes W and the top Horner level (two outputs over one candidate pattern), then
    the levels T.W, then X.T: (i + j)/2 + 1 products."""
    tau = 1e-6
    m, h = H.lattice_bsr(L, seed=3)
    n = m.n
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, mu=h.mu,
              xi=h.xi, tol=1e-9, max_iter=60)
    if pij:
        kw["poly_ij"] = pij
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, scheme, trunc_tau=tau, **kw)
    assert r["status"] in ("ok", "ok_floor"), r["status"]
    Dg = _to_dense(rp, ci, va, n)
    Fd = m.to_dense()
    okw = dict(kw)
    okw.update(tol=0.0, max_iter=r["iterations"])
    o = dense.purify(Fd, scheme, mask=dense.block_truncation_mask(32, tau), **okw)
    assert r["branches"] == o["branches"]
    per_it = (pij[0] + pij[1]) // 2 + 1 if pij else (4 if scheme.endswith("3") else 6)
    assert r["products"] == per_it * r["iterations"] + 1
    err = float(np.linalg.norm(Dg - o["D"]))
    print(f"\nBSR {L} {scheme}: status {r['status']} products {r['products']} "
          f"e={r['idem_err']:.2e} |D-D_oracle|_F={err:.2e} tr err {r['trace_err']:.2e}")
    assert err <= 1e-3 * math.sqrt(n)
    assert abs(r["trace_err"]) <= 1e-2 and r["idem_err"] <= 1e-3
    assert np.array_equal(Dg, Dg.T)


def test_bsr_no_truncation_matches_dense_oracle(snf):
    """tau = 0: the block-sparse product is a plain FP32 product of the full pattern."""
    m, h = H.lattice_bsr((8, 8, 4), seed=1)
    n = m.n
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-4, max_iter=60)
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, "snf_varmu", trunc_tau=0.0, **kw)
    o = dense.purify(m.to_dense(), "snf_varmu", **kw)
    assert r["status"] == o["status"] == "ok"
    assert r["branches"] == o["branches"] and r["products"] == o["products"]
    assert np.linalg.norm(_to_dense(rp, ci, va, n) - o["D"]) <= 1e-4 * math.sqrt(n)
    # Algorithm 1: both products of every iteration without truncation
    kw.update(mu=h.mu, xi=h.xi)
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, "snf_fixmu", trunc_tau=0.0, **kw)
    o = dense.purify(m.to_dense(), "snf_fixmu", **kw)
    assert r["status"] == o["status"] == "ok"
    assert r["branches"] == o["branches"] and r["products"] == o["products"]
    assert np.linalg.norm(_to_dense(rp, ci, va, n) - o["D"]) <= 1e-4 * math.sqrt(n)


def test_bsr_invalid_inputs(snf):
    m, h = H.lattice_bsr((8, 8, 4), seed=1)
    n = m.n
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-6, max_iter=40)
    rp, ci, va = _dev_bsr(m)
    with pytest.raises(RuntimeError):            # Algorithm 1 needs mu and xi
        snf.purify_bsr(rp, ci, va, n, "snf_fixmu", **kw)
    with pytest.raises(RuntimeError):            # an error-control budget must be positive
        snf.purify_bsr(rp, ci, va, n, "snf_fixmu", mu=h.mu, xi=h.xi, trunc_tau=0.0,
                       flags=snf.FLAG_TRUNC_ERROR_CONTROL, **kw)
    with pytest.raises(RuntimeError):            # P_{i,j} needs odd i, j
        snf.purify_bsr(rp, ci, va, n, "snf_pij", mu=h.mu, xi=h.xi, poly_ij=(2, 3), **kw)
    # drop one off-diagonal block: the pattern is no longer symmetric
    keep = np.ones(m.nnzb, bool)
    off = next(p for p in range(m.nnzb) if m.col_idx[p] != 0)
    keep[off] = False
    cnt = np.diff(m.row_ptr).copy()
    cnt[0] -= 1
    rp2 = np.concatenate(([0], np.cumsum(cnt))).astype(np.int32)
    bad = H.BSRMatrix(n=n, b=32, row_ptr=rp2, col_idx=m.col_idx[keep], val=m.val[keep])
    with pytest.raises(RuntimeError):
        snf.purify_bsr(*_dev_bsr(bad), n, "snf_varmu", **kw)


def test_bsr_full_lattice_65536(snf):
    """The 32x32x32-site lattice (n = 65536) with tau = 1e-6: runs to the truncation floor.
    No oracle fits at this size; checked: decisions equal the scalar recurrence, trace and
    idempotency at the floor, symmetric pattern, D within [0, 1] spectrum sanity through
    ||D||_F^2 ~ tr D."""
    from oracle import spectral
    m, h = H.lattice_bsr((32, 32, 32), seed=3)
    n = m.n
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-9, max_iter=60)
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, "snf_varmu", trunc_tau=1e-6, **kw)
    assert r["status"] in ("ok", "ok_floor")
    seq = spectral.decision_sequence("snf_varmu", lambda_min=h.lambda_min,
                                     lambda_max=h.lambda_max, homo=h.homo, lumo=h.lumo,
                                     steps=r["iterations"])
    assert r["branches"] == "".join(s[0] for s in seq)
    assert abs(r["trace_err"]) <= 1.0 and r["idem_err"] <= 1e-2
    t2 = float((va.double() ** 2).sum())
    assert abs(t2 - r["trace"]) <= 1e-2 * r["trace"]
    print(f"\nBSR 32^3: {r['status']} products {r['products']} e={r['idem_err']:.2e} "
          f"tr err {r['trace_err']:.2e} blocks {r['nnzb']} ({r['nnzb'] / (n // 32):.0f} per row) "
          f"device {r['device_ms']:.0f} ms")


@pytest.mark.parametrize("scheme,pij", [("tc2", None), ("snf_varmu", None), ("sp2", None),
                                        ("snf_fixmu", None), ("snf_fixmu3", None),
                                        ("snf_pij", (1, 3))])
@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_error_controlled_truncation(snf, scheme, pij, eps):
    """Error-controlled truncation (budget eps for ||D - D_exact||_F) on the 16x8x8-site
    lattice (n = 2048).  Bars: decisions equal the oracle's; ||D_gpu - D_exact||_F within eps
    plus the FP32 floor of the same solve without truncation; stored blocks of D within 5% of
    the oracle's (FP32 block norms near a bin edge may fall on the other side).  The fixed-mu
    schemes truncate each iteration's result, with the gap of its bounds."""
    m, h = H.lattice_bsr((16, 8, 8), seed=3)
    n = m.n
    m64, _ = H.lattice_bsr((16, 8, 8), seed=3, dtype=np.float64)
    Fd = m64.to_dense()
    D_ref = exact.projector(F=Fd, n_occ=h.n_occ)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-9, max_iter=60)
    pkw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, homo=h.homo, lumo=h.lumo)
    if scheme not in ("tc2", "snf_varmu", "sp2"):
        kw.update(mu=h.mu, xi=h.xi, poly_ij=pij)
        pkw.update(mu=h.mu, xi=h.xi, poly_ij=pij)
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, scheme, trunc_tau=eps,
                                      flags=snf.FLAG_TRUNC_ERROR_CONTROL, **kw)
    assert r["status"] in ("ok", "ok_floor"), r["status"]
    (rp0, ci0, va0), r0 = snf.purify_bsr(*_dev_bsr(m), n, scheme, trunc_tau=0.0, **kw)
    floor = float(np.linalg.norm(_to_dense(rp0, ci0, va0, n) - D_ref))
    Dg = _to_dense(rp, ci, va, n)
    err = float(np.linalg.norm(Dg - D_ref))
    N = dense.predicted_iterations(scheme, eps=eps, **pkw)
    mk = dense.ErrorControlledTruncation(32, eps, N)
    okw = dict(kw)
    okw.update(tol=0.0, max_iter=r["iterations"])
    o = dense.purify(Fd, scheme, mask=mk, **okw)
    if scheme != "sp2":
        assert r["branches"] == o["branches"]
    nb = n // 32
    blocks_o = int((np.abs(o["D"]).reshape(nb, 32, nb, 32).sum(axis=(1, 3)) > 0).sum())
    print(f"\nEC {scheme} eps={eps:g}: {r['status']} products {r['products']} "
          f"|D-D_exact|={err:.2e} (no-truncation floor {floor:.2e}, oracle "
          f"{np.linalg.norm(o['D'] - D_ref):.2e}) blocks {r['nnzb']} / oracle {blocks_o} "
          f"/ untruncated {r0['nnzb']}")
    assert err <= eps + floor
    assert abs(r["nnzb"] - blocks_o) <= 0.05 * blocks_o
    # blocks stored over the iterates (the log's spare field): fewer than without truncation
    assert sum(x["phase"] for x in r["log"]) < sum(x["phase"] for x in r0["log"])
    assert np.array_equal(Dg, Dg.T)


def test_error_control_rejects_zero_budget(snf):
    m, h = H.lattice_bsr((8, 8, 4), seed=1)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-6, max_iter=40)
    with pytest.raises(RuntimeError):
        snf.purify_bsr(*_dev_bsr(m), m.n, "snf_varmu", trunc_tau=0.0,
                       flags=snf.FLAG_TRUNC_ERROR_CONTROL, **kw)



@pytest.mark.parametrize("tau_s", [1e-4, 1e-3])
def test_step_screened_matches_oracle(snf, tau_s):
    """Norm screening of one step against the oracle's screened product on the same FP32
    values: a graded X (X_0^4 of the lattice, block norms from 3e-4 to 1.1, so that 26% /
    46% of the block triples fall below the two thresholds); the pattern is the unscreened
    one, the values are those of the screened product within the FP32 dot-product bound,
    while they differ from the unscreened product by far more than that bound."""
    m, h = H.lattice_bsr((8, 8, 4), seed=7)
    n = m.n
    Fd = m.to_dense()
    X0 = (h.lambda_max * np.eye(n) - Fd) / (h.lambda_max - h.lambda_min)
    X1 = X0 @ X0
    Xm = H.dense_to_bsr(X1 @ X1, 32)
    X32 = Xm.to_dense()
    nb = n // 32
    norms = _block_norms(X32)
    terms = (norms[:, :, None] * norms[None, :, :]).ravel()
    assert not np.any(np.abs(terms[terms > 0] / tau_s - 1.0) <= 1e-9)   # no near-ties
    c2, c1, c0 = -1.44, 2.4, 0.0
    (rp, ci, va), sums, _ = snf.step_bsr(*_dev_bsr(Xm), n, c2, c1, c0, trunc_tau=0.0,
                                          screen_tau=tau_s)
    Y = _to_dense(rp, ci, va, n)
    Ps = dense.screened_square(X32, 32, tau_s)
    Yref = c2 * Ps + c1 * X32 + c0 * np.eye(n)
    Yfull = c2 * (X32 @ X32) + c1 * X32 + c0 * np.eye(n)
    pat = (norms > 0).astype(int)
    assert np.array_equal(_block_norms(Y) > 0, ((pat @ pat) > 0) | np.eye(nb, dtype=bool))
    bound = (n + 2) * 2.0 ** -24 * (np.abs(X32) @ np.abs(X32)) * abs(c2) + 1e-6 \
        + 2.0 ** -23 * np.abs(Yref)
    assert np.all(np.abs(Y - Yref) <= bound)
    assert np.max(np.abs(Yfull - Yref) / bound) > 4.0        # the screening is visible
    e2 = np.sum((Ps - X32) ** 2)
    assert abs(sums[0] - e2) <= 1e-4 * e2
    assert np.array_equal(Y, Y.T)


@pytest.mark.parametrize("scheme,pij", [("snf_varmu", None), ("tc2", None),
                                        ("snf_fixmu", None), ("mcweeny", None),
                                        ("snf_fixmu3", None), ("pmm3", None),
                                        ("snf_pij", (1, 3)), ("pij", (3, 1))])
def test_purify_bsr_screened_vs_oracle(snf, scheme, pij):
    """Whole solves with truncation (tau = 1e-6) and norm screening (1e-8) on the 8x8x8-site
    lattice against the oracle with the same truncation rule and the same screening of its
    FP64 iterates: identical decisions, D as close as for truncation alone.  The fixed-mu
    schemes screen every product of an iteration (Algorithm 1's S2.X, the Horner levels
    W.T of P_{m,m} and T.W of P_{i,j}, the last X.T), each with its operands' block norms."""
    tau, tau_s = 1e-6, 1e-8
    m, h = H.lattice_bsr((8, 8, 8), seed=3)
    n = m.n
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-9, max_iter=60)
    if scheme not in ("snf_varmu", "tc2", "sp2"):
        kw.update(mu=h.mu, xi=h.xi)
    if pij is not None:
        kw.update(poly_ij=pij)
    (rp, ci, va), r = snf.purify_bsr(*_dev_bsr(m), n, scheme, trunc_tau=tau,
                                      screen_tau=tau_s, **kw)
    assert r["status"] in ("ok", "ok_floor"), r["status"]
    Dg = _to_dense(rp, ci, va, n)
    Fd = m.to_dense()
    okw = dict(kw)
    okw.update(tol=0.0, max_iter=r["iterations"])
    o = dense.purify(Fd, scheme, mask=dense.block_truncation_mask(32, tau),
                     screen=(32, tau_s), **okw)
    assert r["branches"] == o["branches"]
    err = float(np.linalg.norm(Dg - o["D"]))
    print(f"\nBSR screened {scheme}: status {r['status']} products {r['products']} "
          f"e={r['idem_err']:.2e} |D-D_oracle|_F={err:.2e} tr err {r['trace_err']:.2e}")
    assert err <= 1e-3 * math.sqrt(n)
    assert abs(r["trace_err"]) <= 1e-2 and r["idem_err"] <= 1e-3
    assert np.array_equal(Dg, Dg.T)
    with pytest.raises(RuntimeError):
        snf.purify_bsr(*_dev_bsr(m), n, scheme, trunc_tau=tau, screen_tau=-1.0, **kw)

def test_step_full_lattice_65536_sampled(snf):
    """Two steps at the size of the block-sparse workload (32x32x32 sites, n = 65536, 2048
    block rows), no truncation: X_1 = X_0^2 from the trace scheme's X_0, then a fold-type
    step Y = c2 X_1^2 + c1 X_1.  No dense oracle fits at this size, so: the pattern of sampled
    block rows of Y equals the union of the patterns of the rows it combines (exact); sampled
    blocks equal FP64 sums over the shared blocks within the FP32 dot-product bound; mirror
    blocks are exact transposes; the fused sums equal sums over the returned blocks."""
    m, h = H.lattice_bsr((32, 32, 32), seed=3)
    n, nb, b = m.n, m.nb, 32
    w = h.lambda_max - h.lambda_min
    val = -m.val.astype(np.float64) / w
    for i in range(nb):
        lo, hi = m.row_ptr[i], m.row_ptr[i + 1]
        p = lo + int(np.searchsorted(m.col_idx[lo:hi], i))
        assert m.col_idx[p] == i
        val[p] += np.eye(b) * (h.lambda_max / w)
    X0 = H.BSRMatrix(n=n, b=b, row_ptr=m.row_ptr, col_idx=m.col_idx, val=val.astype(np.float32))
    dev0 = _dev_bsr(X0)
    (rp1, ci1, va1), s1, _ = snf.step_bsr(*dev0, n, 1.0, 0.0, 0.0, trunc_tau=0.0)

    def keys(rp, ci):
        rows = torch.repeat_interleave(torch.arange(nb, device=ci.device),
                                       (rp[1:] - rp[:-1]).long())
        return rows * nb + ci.long()

    # e2 of the first step: ||X_0^2 - X_0||_F^2 over the returned blocks (X_0's pattern is
    # inside X_0^2's: every row holds its diagonal block)
    k1, k0 = keys(rp1, ci1), keys(dev0[0], dev0[1])
    idx = torch.searchsorted(k1, k0)
    assert torch.equal(k1[idx], k0)
    diff = va1.double().clone()
    diff[idx] -= dev0[2].double()
    e2 = float((diff ** 2).sum())
    assert abs(s1[0] - e2) <= 1e-4 * e2

    c2, c1, c0 = -1.69, 2.6, 0.0
    (rp2, ci2, va2), s2, _ = snf.step_bsr(rp1, ci1, va1, n, c2, c1, c0, trunc_tau=0.0)
    rp1h, ci1h = rp1.cpu().numpy(), ci1.cpu().numpy()
    rp2h, ci2h = rp2.cpu().numpy(), ci2.cpu().numpy()

    def row(rp, ci, i):
        return ci[rp[i]:rp[i + 1]]

    rng = np.random.default_rng(65536)
    u32 = 2.0 ** -24
    checked = 0
    for i in rng.choice(nb, size=16, replace=False):
        cols_i = row(rp1h, ci1h, i)
        union = np.unique(np.concatenate([row(rp1h, ci1h, k) for k in cols_i]))
        assert np.array_equal(row(rp2h, ci2h, i), union), i
        Xi = va1[rp1h[i]:rp1h[i + 1]].double().cpu().numpy()
        for j in list(rng.choice(union, size=3, replace=False)) + [i]:
            cols_j = row(rp1h, ci1h, j)
            Xj = va1[rp1h[j]:rp1h[j + 1]].double().cpu().numpy()
            shared, pi, pj = np.intersect1d(cols_i, cols_j, return_indices=True)
            P = np.einsum("kab,kcb->ac", Xi[pi], Xj[pj])            # sum_K X_IK X_JK^T
            A = np.einsum("kab,kcb->ac", np.abs(Xi[pi]), np.abs(Xj[pj]))
            ref = c2 * P + (c0 * np.eye(b) if i == j else 0.0)
            pij = np.searchsorted(cols_i, j)
            if pij < cols_i.size and cols_i[pij] == j:
                ref = ref + c1 * Xi[pij]
            q = rp2h[i] + int(np.searchsorted(row(rp2h, ci2h, i), j))
            got = va2[q].double().cpu().numpy()
            bound = (32 * shared.size + 2) * u32 * abs(c2) * A + 1e-6 + 2.0 ** -23 * np.abs(ref)
            assert np.all(np.abs(got - ref) <= bound), (i, j)
            qm = rp2h[j] + int(np.searchsorted(row(rp2h, ci2h, j), i))
            assert torch.equal(va2[qm], va2[q].T), (i, j)
            checked += 1
    diag = rp2h[:-1] + np.array([np.searchsorted(row(rp2h, ci2h, i), i) for i in range(nb)])
    tr = float(va2[torch.tensor(diag, device=va2.device)].double()
               .diagonal(dim1=1, dim2=2).sum())
    f2 = float((va2.double() ** 2).sum())
    assert abs(s2[1] - tr) <= 1e-6 * max(1.0, abs(tr))
    assert abs(s2[2] - f2) <= 1e-5 * f2
    print(f"\nBSR step at n = {n}: X_1 {ci1.numel() / nb:.0f} blocks per row, Y "
          f"{ci2.numel() / nb:.0f}; {checked} sampled blocks within the FP32 bound")
