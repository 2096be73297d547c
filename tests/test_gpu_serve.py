"""Serving loop (continuous batching) on the GPU.

* a request's D is bitwise the same alone and in a mix of requests of other sizes, schemes
  and precisions submitted before, with and after it;
* results match the FP64 oracle (decisions, products, D within 1e-8 sqrt(n) in FP64 mode);
* admission respects the memory budget: with room for one request at a time, a request is
  admitted only after the previous one has finished (the scheduler has seen the stop flag of
  its last step), so their runs on the device do not overlap; a request larger than the budget
  fails at submit.
"""
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


def _req(n, n_occ, seed, gap=0.04):
    mu = -1.0 + 2.0 * n_occ / n
    return H.random_spectrum_hamiltonian(n, n_occ, -1.0, mu - gap / 2, mu + gap / 2, 1.0, seed)


def _kw(h, tol=1e-10):
    return dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
                lumo=h.lumo, mu=h.mu, xi=h.xi, tol=tol, max_iter=150)


GB = 1 << 30


@pytest.mark.parametrize("scheme,prec", [("snf_varmu", "fp64"), ("snf_fixmu", "fp64"),
                                         ("snf_varmu", "fp32_ref64"), ("sp2", "bf16_ref64")])
def test_alone_equals_mix_bitwise(snf, scheme, prec):
    target = _req(300, 140, seed=42)
    others = [(_req(n, n // 2 + 3, seed=n), s, p) for n, s, p in
              [(64, "sp2", "fp64"), (900, "snf_varmu", "fp32_ref64"), (130, "mcweeny", "fp64"),
               (513, "tc2", "fp64"), (77, "snf_fixmu", "bf16_ref64"), (1000, "snf_varmu", "fp64")]]
    with snf.Server(4 * GB, max_slots=16) as sv:
        t = sv.submit(target.F, scheme, prec, **_kw(target))
        D_alone, r_alone = sv.wait(t)
        D_alone = D_alone.copy()
    with snf.Server(4 * GB, max_slots=16) as sv:
        tickets = [sv.submit(h.F, s, p, **_kw(h)) for h, s, p in others[:3]]
        t = sv.submit(target.F, scheme, prec, **_kw(target))
        tickets += [sv.submit(h.F, s, p, **_kw(h)) for h, s, p in others[3:]]
        D_mix, r_mix = sv.wait(t)
        others_res = [sv.wait(x) for x in tickets]
    assert r_alone["status"] == r_mix["status"] == "ok"
    assert np.array_equal(D_alone, D_mix)
    assert r_alone["products"] == r_mix["products"] and r_alone["branches"] == r_mix["branches"]
    for (h, s, p), (D, r) in zip(others, others_res):
        assert r["status"] == "ok", (h.n, s, p, r["status"])
        assert abs(r["trace_err"]) <= 1e-8
    o = dense.purify(target.F, scheme, **_kw(target))
    err = np.linalg.norm(D_mix - o["D"])
    print(f"\n{scheme} {prec}: |D-D_oracle|_F = {err:.2e}")
    if prec == "fp64":
        assert r_mix["branches"] == o["branches"] and r_mix["products"] == o["products"]
        assert err <= 1e-8 * math.sqrt(target.n)


@pytest.mark.parametrize("scheme,pij", [("snf_fixmu3", None), ("pmm5", None),
                                        ("snf_pij", (1, 3)), ("pij", (3, 1))])
def test_higher_order_schemes_served(snf, scheme, pij):
    """P_{m,m} and P_{i,j} requests (FP64; a fourth iterate buffer per request, and for
    P_{i,j} the grouped product with a second output) alone and in a mix with requests of
    other schemes, sizes and precisions: bitwise the same, with the oracle's decisions,
    product count and D."""
    target = _req(300, 140, seed=43)
    kwt = dict(_kw(target), poly_ij=pij)
    others = [(_req(n, n // 2 + 3, seed=n + 1), s, p, pp) for n, s, p, pp in
              [(200, "snf_pij", "fp64", (3, 1)), (640, "snf_varmu", "fp32_ref64", None),
               (130, "snf_fixmu5", "fp64", None), (257, "sp2", "fp64", None),
               (96, "snf_fixmu", "fp64", None)]]
    with snf.Server(4 * GB, max_slots=16) as sv:
        t = sv.submit(target.F, scheme, "fp64", **kwt)
        D_alone, r_alone = sv.wait(t)
        D_alone = D_alone.copy()
    with snf.Server(4 * GB, max_slots=16) as sv:
        tickets = [sv.submit(h.F, s, p, **dict(_kw(h), poly_ij=pp)) for h, s, p, pp in others[:2]]
        t = sv.submit(target.F, scheme, "fp64", **kwt)
        tickets += [sv.submit(h.F, s, p, **dict(_kw(h), poly_ij=pp)) for h, s, p, pp in others[2:]]
        D_mix, r_mix = sv.wait(t)
        others_res = [sv.wait(x) for x in tickets]
    assert r_alone["status"] == r_mix["status"] == "ok"
    assert np.array_equal(D_alone, D_mix)
    for (h, s, p, pp), (D, r) in zip(others, others_res):
        assert r["status"] == "ok", (h.n, s, p, r["status"])
    o = dense.purify(target.F, scheme, **kwt)
    err = np.linalg.norm(D_mix - o["D"])
    print(f"\nserved {scheme} {pij}: products {r_mix['products']} |D-D_oracle|_F = {err:.2e}")
    assert r_mix["branches"] == o["branches"] and r_mix["products"] == o["products"]
    assert err <= 1e-8 * math.sqrt(target.n)


def test_results_match_oracle_fp64(snf):
    hs = [_req(n, n // 2 - 5, seed=100 + n, gap=0.08) for n in (64, 200, 385, 640)]
    with snf.Server(2 * GB, max_slots=8) as sv:
        tickets = [sv.submit(h.F, "snf_varmu", "fp64", **_kw(h)) for h in hs]
        results = [sv.wait(t) for t in tickets]
    for h, (D, r) in zip(hs, results):
        o = dense.purify(h.F, "snf_varmu", **_kw(h))
        assert r["status"] == o["status"] == "ok"
        assert r["branches"] == o["branches"] and r["products"] == o["products"]
        assert np.linalg.norm(D - o["D"]) <= 1e-8 * math.sqrt(h.n)


def test_budget_serialises_admission(snf):
    n = 500
    one = snf.Server.request_bytes(n, "fp64")
    hs = [_req(n, 240, seed=s) for s in range(4)]
    with snf.Server(int(one * 1.5), max_slots=8) as sv:
        tickets = [sv.submit(h.F, "snf_varmu", "fp64", **_kw(h)) for h in hs]
        for h, t in zip(hs, tickets):
            # each admission reuses the memory the previous request was retired from (the
            # retirement's copy-out and the admission's writes share one stream)
            D, r = sv.wait(t)
            assert r["status"] == "ok"
            o = dense.purify(h.F, "snf_varmu", **_kw(h))
            assert np.linalg.norm(D - o["D"]) <= 1e-8 * math.sqrt(n)
        times = [sv.timing(t) for t in tickets]
        line = [sv.timeline(t) for t in tickets]
        with pytest.raises(RuntimeError):                  # larger than the whole budget
            sv.submit(_req(900, 400, seed=9).F, "snf_varmu", "fp64",
                      **_kw(_req(900, 400, seed=9)))
    for sub, adm, fin, done in line:
        assert sub <= adm <= fin <= done
    # the runs [admitted, finished] follow one another: each request was admitted only after
    # the previous one finished
    for k in range(len(line) - 1):
        assert line[k + 1][1] >= line[k][2], (k, line[k], line[k + 1])
    # queued time grows along the FIFO: each request waited for the previous one
    q = [t[0] for t in times]
    assert q[1] > 0 and q[3] > q[1]


def test_unknown_ticket(snf):
    with snf.Server(GB // 4, max_slots=2) as sv:
        with pytest.raises(KeyError):
            sv.poll(12345)


def test_device_submit_matches_host_submit(snf):
    hs = [_req(n, n // 2 + 1, seed=7 * n, gap=0.05) for n in (96, 300, 700)]
    with snf.Server(GB, max_slots=8) as sv:
        th = [sv.submit(h.F, "snf_varmu", "fp32_ref64", **_kw(h)) for h in hs]
        Fd = [torch.tensor(h.F, device="cuda:0") for h in hs]
        td = [sv.submit_device(F, "snf_varmu", "fp32_ref64", **_kw(h)) for F, h in zip(Fd, hs)]
        host = [sv.wait(t) for t in th]
        devr = [sv.wait(t) for t in td]
    torch.cuda.synchronize()
    for (Dh, rh), (Dd, rd) in zip(host, devr):
        assert rh["status"] == rd["status"] == "ok"
        assert np.array_equal(Dh, Dd.cpu().numpy())


def test_many_small_requests_pinned_staging_cycles(snf):
    """More queued host requests than the pinned staging holds at once: all complete."""
    hs = [_req(512, 250 + (i % 7), seed=500 + i, gap=0.1) for i in range(40)]
    with snf.Server(64 << 20, max_slots=4) as sv:
        ts = [sv.submit(h.F, "sp2", "fp64", **_kw(h, tol=1e-9)) for h in hs]
        rs = [sv.wait(t) for t in ts]
    assert all(r["status"] == "ok" for _, r in rs)
