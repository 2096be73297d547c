"""Degenerate and boundary cases across the entry points (GPU, C ABI), each against the CPU
oracle or an exact answer: order 1 for every scheme, a single-block and a block-diagonal
block-sparse matrix, max_iter exhaustion of the higher-order schemes, all-occupied and
empty occupations rejected or handled, bound estimation at n = 1 and n < steps, and an
order that is not a multiple of the tile for the bound estimators."""
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
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda:0")


@pytest.mark.parametrize("scheme", ["snf_fixmu3", "snf_fixmu5", "pmm3", "pmm5"])
@pytest.mark.parametrize("level", [0.3, 0.9])
def test_order_one_higher_order(snf, scheme, level):
    """n = 1: a single level below (occupied) or above (empty) mu = 0.6."""
    F = np.array([[level]])
    kw = dict(lambda_min=-1.0, lambda_max=1.0, mu=0.6, xi=0.6, tol=1e-12, max_iter=100)
    D, r = snf.purify_dense(_dev(F), scheme, **kw)
    o = dense.purify(F, scheme, **kw)
    assert r["status"] == o["status"] == "ok"
    assert r["products"] == o["products"]
    assert abs(D.item() - (1.0 if level < 0.6 else 0.0)) <= 1e-12


def test_higher_order_max_iter_exhausted(snf):
    h = H.random_spectrum_hamiltonian(64, 30, -1.0, -0.001, 0.001, 1.0, seed=3)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, mu=h.mu,
              xi=h.xi, tol=1e-12, max_iter=2)
    _, r = snf.purify_dense(_dev(h.F), "snf_fixmu3", **kw)
    o = dense.purify(h.F, "snf_fixmu3", **kw)
    assert r["status"] == o["status"] == "noconv"
    assert r["iterations"] == o["iterations"] == 2
    assert r["products"] == o["products"] == 2 * 4 + 1


def _bsr_dev(m):
    return (torch.tensor(m.row_ptr, device="cuda:0"), torch.tensor(m.col_idx, device="cuda:0"),
            torch.tensor(m.val, device="cuda:0"))


def _bsr_dense(snf, D, n):
    rp, ci, va = D
    return H.BSRMatrix(n=n, b=32, row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(),
                       val=va.cpu().numpy()).to_dense()


@pytest.mark.parametrize("scheme", ["snf_varmu", "sp2", "tc2", "snf_fixmu", "mcweeny",
                                    "snf_fixmu3"])
def test_bsr_single_block(snf, scheme):
    """n = 32: the whole matrix is one block (for the fixed-mu schemes every product of an
    iteration is that one block)."""
    h = H.random_spectrum_hamiltonian(32, 13, -1.0, -0.1, 0.1, 1.0, seed=4)
    m = H.dense_to_bsr(h.F, 32)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-5, max_iter=60)
    if scheme in ("snf_fixmu", "mcweeny", "snf_fixmu3"):
        kw.update(mu=h.mu, xi=h.xi)
    D, r = snf.purify_bsr(*_bsr_dev(m), 32, scheme, trunc_tau=0.0, **kw)
    assert r["status"] in ("ok", "ok_floor")
    D_ref = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    assert np.linalg.norm(_bsr_dense(snf, D, 32) - D_ref) <= 1e-4


def test_bsr_block_diagonal(snf):
    """Block-diagonal F (no coupling between blocks): D stays block diagonal, each block the
    projector of its own block of F."""
    rng = np.random.default_rng(5)
    n, nb = 128, 4
    F = np.zeros((n, n))
    blocks = []
    for b in range(nb):
        h = H.random_spectrum_hamiltonian(32, 16, -1.0, -0.2, 0.2, 1.0, seed=10 + b)
        F[32 * b:32 * b + 32, 32 * b:32 * b + 32] = h.F
        blocks.append(h)
    m = H.dense_to_bsr(F, 32)
    assert m.col_idx.size == nb
    kw = dict(lambda_min=-1.0, lambda_max=1.0, n_occ=64, homo=-0.2, lumo=0.2, tol=1e-5,
              max_iter=60)
    D, r = snf.purify_bsr(*_bsr_dev(m), n, "snf_varmu", trunc_tau=1e-7, **kw)
    assert r["status"] in ("ok", "ok_floor") and r["nnzb"] == nb
    Dd = _bsr_dense(snf, D, n)
    for b, h in enumerate(blocks):
        Db = exact.projector(n_occ=16, eigvals=h.eigvals, Q=h.Q)
        assert np.linalg.norm(Dd[32 * b:32 * b + 32, 32 * b:32 * b + 32] - Db) <= 1e-4


def test_bounds_order_one_and_short(snf):
    F = np.array([[0.37]])
    lo, hi, glo, ghi = snf.spectral_bounds(_dev(F), 5)
    assert abs(lo - 0.37) < 1e-12 and abs(hi - 0.37) < 1e-12 and lo <= 0.37 <= hi
    assert glo == ghi == 0.37
    h = H.random_spectrum_hamiltonian(100, 40, -1.0, -0.05, 0.05, 1.0, seed=8)
    v0 = np.random.default_rng(1).standard_normal(100)
    lo, hi, _, _ = snf.spectral_bounds(_dev(h.F), 150, start=_dev(v0))   # steps > n
    assert abs(lo - h.lambda_min) < 1e-11 and abs(hi - h.lambda_max) < 1e-11
    D = exact.projector(n_occ=h.n_occ, eigvals=h.eigvals, Q=h.Q)
    homo, lumo = snf.gap_bounds(_dev(h.F), _dev(D), -1.0, 1.0, 3, start=_dev(v0))
    ohomo, olumo = bounds.gap_bounds(h.F, D, -1.0, 1.0, v0, 3)
    assert abs(homo - ohomo) < 1e-12 and abs(lumo - olumo) < 1e-12
    assert homo <= h.homo and lumo >= h.lumo


def test_dense_rejects_impossible_occupation(snf):
    h = H.random_spectrum_hamiltonian(16, 8, -1.0, -0.1, 0.1, 1.0, seed=2)
    with pytest.raises(RuntimeError):
        snf.purify_dense(_dev(h.F), "sp2", lambda_min=-1.0, lambda_max=1.0, n_occ=17,
                         tol=1e-10)
