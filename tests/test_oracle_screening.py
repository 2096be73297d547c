"""Pins of the norm-screened block product in the CPU oracle (no GPU).

Screening leaves the block product X_IK X_KJ out of (X.X)_IJ when ||X_IK||_F ||X_KJ||_F is
below a threshold (the block-sparse path's use of the decay of the blocks next to
truncation; the paper only says that the schemes combine with such approximations, the rule
is a reading).  Pinned against: the library matrix product when nothing is screened, a
brute-force loop over block triples on tiny inputs (a square and a product of two different,
non-symmetric matrices), the norm bound on what is left out, the empty product above every
norm product, Algorithm 1's printed map for its written-out step, and the unscreened
iteration, which a threshold below every term reproduces.
"""
import math

import numpy as np
import pytest

from fractions import Fraction

from oracle import dense, polynomials, schedule
from paper_1101_0265_amd import hamiltonians as H


def _graded(nb, b, seed):
    """Symmetric matrix whose blocks have norms spread over many decades."""
    rng = np.random.default_rng(seed)
    n = nb * b
    X = rng.standard_normal((n, n))
    scale = 10.0 ** rng.uniform(-9, 0, size=(nb, nb))
    scale = np.sqrt(scale * scale.T)
    X = X * np.kron(scale, np.ones((b, b)))
    return 0.5 * (X + X.T)


def test_threshold_zero_is_the_matrix_product():
    X = _graded(6, 8, 1)
    P = dense.screened_square(X, 8, 0.0)
    assert np.allclose(P, X @ X, rtol=0, atol=1e-13 * np.abs(X).max() ** 2 * X.shape[0])


@pytest.mark.parametrize("tau_s", [1e-8, 1e-5, 1e-3])
def test_brute_force_block_triples(tau_s):
    nb, b = 3, 4
    X = _graded(nb, b, 7)
    blk = lambda I, J: X[I * b:(I + 1) * b, J * b:(J + 1) * b]  # noqa: E731
    P = np.zeros_like(X)
    skipped = 0
    for I in range(nb):
        for J in range(nb):
            acc = np.zeros((b, b))
            for K in range(nb):
                if np.linalg.norm(blk(I, K)) * np.linalg.norm(blk(K, J)) >= tau_s:
                    acc += blk(I, K) @ blk(K, J)
                else:
                    skipped += 1
            P[I * b:(I + 1) * b, J * b:(J + 1) * b] = acc
    assert np.allclose(dense.screened_square(X, b, tau_s), P, rtol=1e-13, atol=1e-300)
    assert 0 < skipped < nb ** 3          # the threshold falls inside the norm range


@pytest.mark.parametrize("tau_s", [1e-7, 1e-4, 1e-2])
def test_left_out_part_within_the_norm_bound(tau_s):
    nb, b = 8, 6
    X = _graded(nb, b, 3)
    blocks = X.reshape(nb, b, nb, b)
    norms = np.sqrt(np.einsum("ibjc,ibjc->ij", blocks, blocks))
    D = (dense.screened_square(X, b, tau_s) - X @ X).reshape(nb, b, nb, b)
    err = np.sqrt(np.einsum("ibjc,ibjc->ij", D, D))
    for I in range(nb):
        for J in range(nb):
            terms = norms[I, :] * norms[:, J]
            bound = terms[terms < tau_s].sum()
            assert err[I, J] <= bound * (1 + 1e-12) + 1e-15 * norms.max() ** 2
            assert bound <= (terms < tau_s).sum() * tau_s


def test_threshold_above_every_term_leaves_nothing():
    X = _graded(4, 5, 11)
    assert not dense.screened_square(X, 5, 1e3 * np.abs(X).max() ** 2 * X.shape[0]).any()


def test_expanded_step_equals_the_printed_maps():
    X = _graded(4, 5, 2)
    X = X / np.abs(np.linalg.eigvalsh(X)).max()
    I = np.eye(X.shape[0])
    for alpha in (0.0, 0.3, 0.9):
        sq = dense.step_expanded(X, X @ X, "S", alpha)
        fo = dense.step_expanded(X, X @ X, "F", alpha)
        Y = (1 + alpha) * X - alpha * I
        assert np.allclose(sq, Y @ Y, atol=1e-13)
        assert np.allclose(fo, 2 * (1 + alpha) * X - (1 + alpha) ** 2 * (X @ X), atol=1e-13)


@pytest.mark.parametrize("scheme", ["snf_varmu", "tc2", "sp2"])
def test_tiny_threshold_reproduces_the_unscreened_iteration(scheme):
    m, h = H.lattice_bsr((4, 4, 4), seed=3, dtype=np.float64)
    F = m.to_dense()
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-10, max_iter=60)
    a = dense.purify(F, scheme, **kw)
    b = dense.purify(F, scheme, screen=(32, 1e-300), **kw)
    assert a["status"] == b["status"] == "ok"
    assert a["branches"] == b["branches"] and a["products"] == b["products"]
    assert np.linalg.norm(a["D"] - b["D"]) <= 1e-11 * math.sqrt(F.shape[0])


def test_screened_iteration_error_grows_with_the_threshold():
    """On the lattice the screened solve stays close to the unscreened one at small
    thresholds and moves away as the threshold grows (the left-out terms act as a
    perturbation of each product)."""
    m, h = H.lattice_bsr((4, 4, 4), seed=3, dtype=np.float64)
    F = m.to_dense()
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-7, max_iter=60)
    ref = dense.purify(F, "snf_varmu", **kw)
    errs = []
    for tau_s in (1e-9, 1e-6, 1e-3):
        r = dense.purify(F, "snf_varmu", screen=(32, tau_s), tol=0.0,
                         max_iter=ref["iterations"],
                         **{k: v for k, v in kw.items() if k not in ("tol", "max_iter")})
        errs.append(float(np.linalg.norm(r["D"] - ref["D"])))
    assert errs[0] <= 1e-7
    assert errs[0] <= errs[1] <= errs[2]


@pytest.mark.parametrize("q", [0.2, 0.5, 0.8])
def test_product_brute_force_block_triples(q):
    """Two different, non-symmetric factors: a transposed operand or the norms of the wrong
    factor would change which triples are kept.  The threshold lies halfway between two
    neighbouring norm products near the q-quantile (no ties), so some triples are kept and
    some left out."""
    nb, b = 3, 4
    A = _graded(nb, b, 17) + 0.3 * _graded(nb, b, 18) @ np.diag(np.arange(1.0, nb * b + 1))
    B = _graded(nb, b, 19) * np.kron(np.triu(np.ones((nb, nb))) + 1e-4, np.ones((b, b)))
    blk = lambda M, I, J: M[I * b:(I + 1) * b, J * b:(J + 1) * b]  # noqa: E731
    prods = [np.linalg.norm(blk(A, I, K)) * np.linalg.norm(blk(B, K, J))
             for I in range(nb) for J in range(nb) for K in range(nb)]
    srt = np.sort(prods)
    k = int(q * len(srt))
    tau_s = float(0.5 * (srt[k] + srt[k + 1]))
    P = np.zeros_like(A)
    skipped = 0
    for I in range(nb):
        for J in range(nb):
            acc = np.zeros((b, b))
            for K in range(nb):
                if np.linalg.norm(blk(A, I, K)) * np.linalg.norm(blk(B, K, J)) >= tau_s:
                    acc += blk(A, I, K) @ blk(B, K, J)
                else:
                    skipped += 1
            P[I * b:(I + 1) * b, J * b:(J + 1) * b] = acc
    assert np.allclose(dense.screened_product(A, B, b, tau_s), P, rtol=1e-13, atol=1e-300)
    assert 0 < skipped < nb ** 3
    assert np.allclose(dense.screened_product(A, B, b, 0.0), A @ B, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("alpha", [0.2, 0.7, 1.0])
def test_alg1_written_out_step_equals_the_printed_map(alpha):
    """3 Xs^2 - 2 Xs^3 with Xs = a (X - I/2) + I/2, from the written-out form (X.X given,
    S2.X formed); a = 1 is McWeeny's 3 X^2 - 2 X^3."""
    X = _graded(4, 5, 23)
    X = 0.5 * np.eye(X.shape[0]) + 0.4 * X / np.abs(np.linalg.eigvalsh(X)).max()
    I = np.eye(X.shape[0])
    Xs = alpha * (X - 0.5 * I) + 0.5 * I
    printed = 3.0 * Xs @ Xs - 2.0 * Xs @ Xs @ Xs
    got = dense.step_expanded_alg1(X, X @ X, alpha, 5, 0.0)
    assert np.allclose(got, printed, rtol=0, atol=1e-14)


@pytest.mark.parametrize("scheme", ["snf_fixmu", "mcweeny"])
def test_tiny_threshold_reproduces_the_unscreened_alg1_iteration(scheme):
    m, h = H.lattice_bsr((4, 4, 4), seed=3, dtype=np.float64)
    F = m.to_dense()
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, mu=h.mu, xi=h.xi, tol=1e-10,
              max_iter=60)
    a = dense.purify(F, scheme, **kw)
    b = dense.purify(F, scheme, screen=(32, 1e-300), **kw)
    assert a["status"] == b["status"] == "ok"
    assert a["branches"] == b["branches"] and a["products"] == b["products"]
    assert np.linalg.norm(a["D"] - b["D"]) <= 1e-11 * math.sqrt(F.shape[0])


def _poly_eval(coeffs, x):
    acc = Fraction(0)
    for c in reversed(coeffs):
        acc = acc * x + c
    return acc


@pytest.mark.parametrize("m", [1, 3, 5])
def test_pmm_shifted_coefficients(m):
    """r_k of P_{m,m}(1/2 + v) = 1/2 + v r(v^2): the closed form c_m C(m, k) (-1)^k
    4^(k-m) / (2k + 1), c_m = (2m+1)! / (m!)^2 (integrating P' = c_m (1/4 - v^2)^m), and the
    polynomial itself at rational points (so no even power of v is lost)."""
    r = dense.pmm_r_exact(m)
    cm = Fraction(math.factorial(2 * m + 1), math.factorial(m) ** 2)
    for k in range(m + 1):
        assert r[k] == cm * math.comb(m, k) * (-1) ** k * Fraction(4) ** (k - m) / (2 * k + 1)
    p = polynomials.p_ij_exact(m, m)
    for v in (Fraction(-2, 5), Fraction(1, 7), Fraction(3, 10)):
        rv = sum(rk * (v * v) ** k for k, rk in enumerate(r))
        assert _poly_eval(p, Fraction(1, 2) + v) == Fraction(1, 2) + v * rv


@pytest.mark.parametrize("ij", [(1, 3), (3, 1), (3, 5), (5, 3), (1, 5)])
def test_pij_shifted_coefficients(ij):
    """q_k of P_{i,j}(x* + v) = x* + v Q(v): the polynomial at points around x* (x* its
    unstable fixed point)."""
    i, j = ij
    xs = schedule.pij_xstar(i, j)
    q = dense.pij_q(i, j, xs)
    p = [float(c) for c in polynomials.p_ij_exact(i, j)]
    assert len(q) == i + j + 1
    for v in np.linspace(-xs, 1.0 - xs, 9):
        lhs = xs + v * sum(qk * v ** k for k, qk in enumerate(q))
        rhs = sum(pk * (xs + v) ** k for k, pk in enumerate(p))
        assert abs(lhs - rhs) <= 1e-13


def _unit_interval_matrix(seed, n=40):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A + A.T
    return 0.5 * np.eye(n) + 0.45 * A / np.abs(np.linalg.eigvalsh(A)).max()


@pytest.mark.parametrize("m,alpha", [(3, 0.6), (3, 1.0), (5, 0.8), (5, 1.0)])
def test_pmm_written_out_step_equals_the_printed_map(m, alpha):
    X = _unit_interval_matrix(31)
    got = dense.step_expanded_pmm(X, X @ X, alpha, m, 8, 0.0)
    want = dense.step(X, schedule.PMM[m], alpha)
    assert np.allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("ij,alpha", [((1, 3), 0.7), ((3, 1), 1.0), ((3, 5), 0.9),
                                      ((5, 1), 0.8)])
def test_pij_written_out_step_equals_the_printed_map(ij, alpha):
    X = _unit_interval_matrix(37)
    st = schedule.SchemeState("snf_pij", -1.0, 1.0, mu=0.1, xi=0.05, poly_ij=ij)
    got = dense.step_expanded_pij(X, X @ X, alpha, ij[0], ij[1], st.xs, 8, 0.0)
    want = dense.step(X, schedule.PIJ, alpha, st)
    assert np.allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("scheme,pij", [("snf_fixmu3", None), ("pmm5", None),
                                        ("snf_pij", (1, 3)), ("pij", (3, 1))])
def test_tiny_threshold_reproduces_the_unscreened_higher_order_iteration(scheme, pij):
    m, h = H.lattice_bsr((4, 4, 4), seed=3, dtype=np.float64)
    F = m.to_dense()
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, mu=h.mu, xi=h.xi, tol=1e-10,
              max_iter=60, poly_ij=pij)
    a = dense.purify(F, scheme, **kw)
    b = dense.purify(F, scheme, screen=(32, 1e-300), **kw)
    assert a["status"] == b["status"] == "ok"
    assert a["branches"] == b["branches"] and a["products"] == b["products"]
    assert np.linalg.norm(a["D"] - b["D"]) <= 1e-10 * math.sqrt(F.shape[0])
