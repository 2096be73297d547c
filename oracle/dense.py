"""Dense FP64 matrix oracle of the purification schemes (test infrastructure only).

Follows the paper's steps on n x n matrices with ``numpy.matmul``:

* Algorithm 2 (varying-mu scale-and-fold) and its alpha = 0 form (unscaled trace-correcting
  scheme with the eigenvalue-based choice): X_0 = (lambda_max I - F)/(lambda_max - lambda_min);
  square branch X <- ((1+a) X - a I)^2, fold branch X <- 2 (1+a) X - (1+a)^2 X^2.
* The trace-based choice ("sp2"): same f_0 and polynomials with a = 0; square iff
  |tr(X^2) - N| < |2 tr X - tr(X^2) - N|.
* Algorithm 1 (fixed-mu scale-and-fold) and its alpha = 1 form (McWeeny):
  X_0 = (mu I - F)/gamma + 0.5 I; X_s = a (X - 0.5 I) + 0.5 I; X <- 3 X_s^2 - 2 X_s^3.
* The same with P_{3,3} or P_{5,5} in place of P_{1,1} (Eq. 2 for odd m): X <- P_{m,m}(X_s),
  evaluated by Horner's rule in X_s on the exact coefficients; the count reported is the
  scheme's m + 1 products per iteration, not the oracle's own.
* P_{i,j} with i, j odd, scaled about its fixed point x*: X_0 = (mu I - F)/gamma + x* I,
  X <- P_{i,j}(a (X - x* I) + x* I), Horner in X_s on the exact coefficients (the schedule
  and its reading are in ``oracle.schedule``); the count is the scheme's (i + j)/2 + 1.

Stopping rule (reading of the open loop length): X_{i-1}^2 is formed, and if
||X_{i-1}^2 - X_{i-1}||_F <= tol the result is D = X_{i-1}.  The scheme's product count
includes that certifying product; Algorithm 1 counts two products per iteration.  The oracle
itself spends extra products (it forms X^2 for the check separately from the step) -- it is
slow on purpose and the count it reports is the scheme's, not its own.

``screen`` (optional): ``(b, tau_s)`` replaces every block product by the norm-screened one
(``screened_product``): X.X in the idempotency check, and in the step the printed polynomial
written out in products, c2 P + c1 X + c0 I for Algorithm 2's maps, for Algorithm 1
S2 = Xs^2 from the screened X.X, then the screened S2.X (``step_expanded_alg1``), for
P_{m,m} and P_{i,j} W = v^2 from the screened X.X, the Horner levels and the last product
with v, each screened (``step_expanded_pmm``, ``step_expanded_pij``).  A screened product
depends on the order of its factors (the norms of A's blocks meet those of B's), so the
written-out steps fix it: W.T for P_{m,m}, T.W for P_{i,j}, X.T last.  Not in the paper: the
screening is the other use of the decay of the blocks next to truncation, and its threshold
rule is a reading.

``mask`` (optional): a callable applied to each new X, used by the block-truncation oracle
(drop blocks below a threshold after every step, the BSR reading).  A mask with
``needs_gap = True`` is called as ``mask(X, gap)`` with the X-space gap beta-bar - beta of
the new iterate (the error-controlled rule) and is not applied to X_0.

Parity: pinned against the exact projector, its invariants and the spectral oracle.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import polynomials as poly
from . import schedule as sch


def f0(F: np.ndarray, scheme: str, lambda_min: float, lambda_max: float,
       mu: float = None, st: "sch.SchemeState" = None) -> np.ndarray:
    n = F.shape[0]
    I = np.eye(n)
    if scheme in ("sp2", "tc2", "snf_varmu"):
        return (lambda_max * I - F) / (lambda_max - lambda_min)       # Algorithm 2, f_0
    if scheme in sch.GENERAL:                                          # mu onto x*
        return (mu * I - F) / st.gamma + st.xs * I
    gamma = sch.alg1_gamma(lambda_min, lambda_max, mu)
    return (mu * I - F) / gamma + 0.5 * I                              # Algorithm 1, X_0


def step(X: np.ndarray, branch: str, alpha: float, st: "sch.SchemeState" = None) -> np.ndarray:
    """One purification transformation f_i, as printed."""
    I = np.eye(X.shape[0])
    if branch == sch.PIJ:                      # P_{i,j}(a (X - x* I) + x* I), Horner in X_s
        Xs = alpha * (X - st.xs * I) + st.xs * I
        c = [float(v) for v in poly.p_ij_exact(st.i, st.j)]
        Y = c[-1] * I
        for k in range(len(c) - 2, -1, -1):
            Y = Y @ Xs + c[k] * I
        return Y
    if branch == sch.SQUARE:
        Y = (1.0 + alpha) * X - alpha * I
        return Y @ Y
    if branch == sch.FOLD:
        return 2.0 * (1.0 + alpha) * X - (1.0 + alpha) ** 2 * (X @ X)
    Xs = alpha * (X - 0.5 * I) + 0.5 * I
    if branch == sch.MCW:
        Xs2 = Xs @ Xs
        Xs3 = Xs2 @ Xs
        return 3.0 * Xs2 - 2.0 * Xs3
    m = 3 if branch == sch.PMM[3] else 5
    c = [float(v) for v in poly.p_ij_exact(m, m)]
    Y = c[-1] * I
    for k in range(len(c) - 2, -1, -1):
        Y = Y @ Xs + c[k] * I
    return Y


def screened_product(A: np.ndarray, B: np.ndarray, b: int, tau_s: float) -> np.ndarray:
    """A.B with every block product A_IK B_KJ whose factors have Frobenius norms with
    product below ``tau_s`` left out of block (I, J): P = sum over block columns K of the
    outer product of block column K of A and block row K of B, each block (I, J) of it kept
    iff ||A_IK||_F ||B_KJ||_F >= tau_s.  Each term left out has norm below tau_s
    (||AB||_F <= ||A||_F ||B||_F).  tau_s = 0 keeps every term."""
    n = A.shape[0]
    nb = n // b

    def block_norms(M):
        blocks = M.reshape(nb, b, nb, b)
        return np.sqrt(np.einsum("ibjc,ibjc->ij", blocks, blocks))

    na, nbn = block_norms(A), block_norms(B)
    P = np.zeros_like(A)
    for K in range(nb):
        col = A[:, K * b:(K + 1) * b]
        row = B[K * b:(K + 1) * b, :]
        keep = np.outer(na[:, K], nbn[K, :]) >= tau_s
        P += np.kron(keep, np.ones((b, b))) * (col @ row)
    return P


def screened_square(X: np.ndarray, b: int, tau_s: float) -> np.ndarray:
    """X.X norm-screened as in ``screened_product``."""
    return screened_product(X, X, b, tau_s)


def step_expanded(X: np.ndarray, P: np.ndarray, branch: str, alpha: float) -> np.ndarray:
    """Algorithm 2's two maps written out in powers of X, with P standing for X^2:
    ((1+a) X - a I)^2 = (1+a)^2 P - 2 a (1+a) X + a^2 I and
    2 (1+a) X - (1+a)^2 X^2 = 2 (1+a) X - (1+a)^2 P."""
    I = np.eye(X.shape[0])
    if branch == sch.SQUARE:
        return (1.0 + alpha) ** 2 * P - 2.0 * alpha * (1.0 + alpha) * X + alpha ** 2 * I
    if branch == sch.FOLD:
        return 2.0 * (1.0 + alpha) * X - (1.0 + alpha) ** 2 * P
    raise ValueError("the expanded step covers the one-product schemes only")


def step_expanded_alg1(X: np.ndarray, P: np.ndarray, alpha: float, b: int,
                       tau_s: float) -> np.ndarray:
    """Algorithm 1's step 3 Xs^2 - 2 Xs^3 (Xs = a X + c I, c = (1 - a)/2) written out with P
    standing for X^2: S2 = Xs^2 = a^2 P + 2 a c X + c^2 I, Xs^3 = a S2.X + c S2, so
    X_new = (3 - 2c) S2 - 2 a R with R = S2.X, the second product screened at tau_s."""
    I = np.eye(X.shape[0])
    c = 0.5 * (1.0 - alpha)
    S2 = alpha * alpha * P + 2.0 * alpha * c * X + c * c * I
    R = screened_product(S2, X, b, tau_s)
    return (3.0 - 2.0 * c) * S2 - 2.0 * alpha * R


def pmm_r_exact(m: int) -> list:
    """r_0..r_m (``Fraction``) of P_{m,m}(1/2 + v) = 1/2 + v r(v^2), from the exact monomial
    coefficients of P_{m,m} shifted to v = x - 1/2 (the odd powers of v)."""
    p = poly.p_ij_exact(m, m)
    c = [Fraction(0)] * len(p)
    for deg, pd in enumerate(p):
        for t in range(deg + 1):
            c[t] += pd * math.comb(deg, t) * Fraction(1, 2) ** (deg - t)
    return [c[2 * k + 1] for k in range(m + 1)]


def pij_q(i: int, j: int, xs: float) -> list:
    """q_0..q_(i+j) (FP64) of P_{i,j}(x* + v) = x* + v Q(v), Q(v) = sum_k q_k v^k: P's exact
    monomial coefficients shifted to v = x - x*."""
    p = [float(v) for v in poly.p_ij_exact(i, j)]
    d = len(p) - 1
    c = [sum(p[deg] * math.comb(deg, t) * xs ** (deg - t) for deg in range(t, d + 1))
         for t in range(d + 1)]
    return c[1:]


def step_expanded_pmm(X: np.ndarray, P: np.ndarray, alpha: float, m: int, b: int,
                      tau_s: float) -> np.ndarray:
    """P_{m,m}(Xs) = I/2 + V r(W), V = a (X - I/2), W = V^2 = a^2 (P - X + I/4) with P
    standing for X^2; r(W) by Horner's rule from the top, the first level from W.W, then
    T <- W.T + r_k I; last V.T = a X.T - (a/2) T.  Products screened at tau_s."""
    I = np.eye(X.shape[0])
    r = [float(v) for v in pmm_r_exact(m)]
    a2 = alpha * alpha
    W = a2 * P - a2 * X + 0.25 * a2 * I
    T = r[m] * screened_product(W, W, b, tau_s) + r[m - 1] * W + r[m - 2] * I
    for k in range(m - 3, -1, -1):
        T = screened_product(W, T, b, tau_s) + r[k] * I
    return alpha * screened_product(X, T, b, tau_s) - 0.5 * alpha * T + 0.5 * I


def step_expanded_pij(X: np.ndarray, P: np.ndarray, alpha: float, i: int, j: int, xs: float,
                      b: int, tau_s: float) -> np.ndarray:
    """P_{i,j}(Xs) = x* I + V Q(V), V = a (X - x* I), W = V^2 = a^2 (P - 2 x* X + x*^2 I) with
    P standing for X^2, Q(V) = sum_k (q_2k I + q_(2k+1) V) W^k (h = (i + j)/2 levels): top
    level T = q_2h W + q_(2h-1) V + q_(2h-2) I, then T <- T.W + q_(2k+1) V + q_2k I, last
    V.T = a X.T - a x* T.  Products screened at tau_s."""
    I = np.eye(X.shape[0])
    q = pij_q(i, j, xs)
    h = (i + j) // 2
    a2 = alpha * alpha
    W = a2 * P - 2.0 * a2 * xs * X + a2 * xs * xs * I
    V = alpha * (X - xs * I)
    T = q[2 * h] * W + q[2 * h - 1] * V + q[2 * h - 2] * I
    for k in range(h - 2, -1, -1):
        T = screened_product(T, W, b, tau_s) + q[2 * k + 1] * V + q[2 * k] * I
    return alpha * screened_product(X, T, b, tau_s) - alpha * xs * T + xs * I


def purify(F: np.ndarray, scheme: str, *, lambda_min: float, lambda_max: float,
           n_occ: int = None, homo: float = None, lumo: float = None, mu: float = None,
           xi: float = None, tol: float = 1e-10, max_iter: int = 200, mask=None,
           force_branches: str = None, poly_ij=None, screen=None) -> dict:
    """Purify the dense symmetric ``F``.

    Returns dict(status, D, iterations, products, branches, log, e_final, trace) with the
    same meaning as ``oracle.spectral.purify_spectrum``.  ``force_branches`` replays a given
    branch string for the trace-based scheme (used when an FP64 near-tie of the trace rule is
    resolved the other way by another implementation).
    """
    if F.ndim != 2 or F.shape[0] != F.shape[1]:
        raise ValueError("F must be square")
    st = sch.SchemeState(scheme, lambda_min, lambda_max, homo=homo, lumo=lumo, mu=mu, xi=xi,
                         poly_ij=poly_ij)
    X = f0(np.asarray(F, dtype=np.float64), scheme, lambda_min, lambda_max, mu, st)
    gap_mask = mask is not None and getattr(mask, "needs_gap", False)
    if mask is not None and not gap_mask:
        X = mask(X)
    per_it = sch.products_per_iteration(scheme, poly_ij)
    log, branches = [], []
    products = 0
    status = "noconv"
    for it in range(max_iter + 1):
        X2 = X @ X if screen is None else screened_square(X, *screen)
        products += 1
        e = float(np.linalg.norm(X2 - X))
        t1 = float(np.trace(X))
        t2 = float(np.trace(X2))
        rec = dict(i=it, e=e, t1=t1, t2=t2, beta=st.beta, betabar=st.betabar)
        if not math.isfinite(e):
            status = "nonfinite"
            log.append(rec)
            break
        if e <= tol:
            status = "ok"
            log.append(rec)
            break
        if it == max_iter:
            log.append(rec)
            break
        branch, alpha = st.choose(t1, t2, n_occ)
        if force_branches is not None and it < len(force_branches):
            branch = force_branches[it]
        rec.update(branch=branch, alpha=alpha,
                   margin=(sch.trace_margin(t1, t2, n_occ) if scheme == "sp2" else None))
        log.append(rec)
        branches.append(branch)
        if screen is None:
            X = step(X, branch, alpha, st)
        elif branch == sch.MCW:
            X = step_expanded_alg1(X, X2, alpha, *screen)
        elif branch in sch.PMM.values():
            X = step_expanded_pmm(X, X2, alpha, 3 if branch == sch.PMM[3] else 5, *screen)
        elif branch == sch.PIJ:
            X = step_expanded_pij(X, X2, alpha, st.i, st.j, st.xs, *screen)
        else:
            X = step_expanded(X, X2, branch, alpha)
        st.advance(branch, alpha)
        if gap_mask:
            X = mask(X, st.betabar - st.beta)
        elif mask is not None:
            X = mask(X)
        products += per_it - 1
    if n_occ is not None and status == "ok" and abs(float(np.trace(X)) - n_occ) >= 0.5:
        status = "mixed"
    return dict(status=status, D=X, iterations=len(branches), products=products,
                branches="".join(branches), log=log, e_final=log[-1]["e"],
                trace=float(np.trace(X)))


def block_truncation_mask(b: int, tau: float):
    """Mask for the block-truncated iteration: after each step drop block (I,J) together with
    its mirror (J,I) when the Frobenius norm of block (I,J), I < J, is below ``tau``; diagonal
    blocks are never dropped.  (The paper leaves the truncation rule open; this is the reading
    used for the block-sparse path.)"""

    def apply(X: np.ndarray) -> np.ndarray:
        n = X.shape[0]
        nb = n // b
        blocks = X.reshape(nb, b, nb, b)
        norms = np.sqrt(np.einsum("ibjc,ibjc->ij", blocks, blocks))
        keep = norms >= tau
        keep = np.triu(keep, 1)
        keep = keep | keep.T | np.eye(nb, dtype=bool)
        return (blocks * keep[:, None, :, None]).reshape(n, n)

    return apply


# ---- error-controlled block truncation ------------------------------------------------
#
# The paper expects the schemes, being of the form of Eq. 1, to combine with forward-error
# control of the truncation, and fewer iterations to allow more aggressive truncation each
# (sparsity paragraph after the bounds paragraph).  The rule used here (a reading; the paper
# gives none): a symmetric perturbation E of an iterate whose X-space gap is g turns its
# occupied subspace by at most ~||E||_F / g (Davis-Kahan), and later iterations keep that
# subspace, so the error of D is bounded to first order by sum_i sqrt(2) ||E_i||_F / g_i.
# With N iterations predicted by the scalar recurrence and a budget eps for ||D~ - D||_F,
# iteration i may drop blocks of total Frobenius norm eps_i = eps g_i / (sqrt(2) N).
# Dropped blocks are chosen on a quarter-octave grid of block norms (half-octaves of the
# squared norm s): bin(s) = floor(2 log2 s), decided exactly from the binary exponent and
# the mantissa against fl(sqrt 2), clamped to [BIN_MIN, BIN_MAX]; each bin is charged
# count * 2^((j+1)/2) (its upper edge), mirror blocks included; the lowest bins are dropped
# while their charge stays within eps_i^2.  Diagonal blocks are never dropped.

BIN_MIN, BIN_MAX = -160, 40
SQRT2 = math.sqrt(2.0)


def half_octave_bin(s: np.ndarray) -> np.ndarray:
    """floor(2 log2 s) for s > 0 (exact), clamped to [BIN_MIN, BIN_MAX]; s = 0 -> BIN_MIN."""
    s = np.asarray(s, dtype=np.float64)
    m, e = np.frexp(s)                 # s = m 2^e, m in [0.5, 1)
    m2, e2 = 2.0 * m, e - 1            # s = m2 2^e2, m2 in [1, 2)
    j = 2 * e2 + (m2 >= SQRT2).astype(np.int64)
    j = np.where(s > 0.0, j, BIN_MIN)
    return np.clip(j, BIN_MIN, BIN_MAX)


def drop_bin_limit(bins: np.ndarray, weights: np.ndarray, eps_i: float) -> int:
    """Largest k such that the blocks with bin < k may be dropped: sum over bins j < k of
    weight * 2^((j+1)/2) <= eps_i^2.  Returns BIN_MIN if not even the lowest bin fits."""
    budget = eps_i * eps_i
    charge = 0.0
    k = BIN_MIN
    for j in range(BIN_MIN, BIN_MAX + 1):
        w = float(np.sum(weights[bins == j]))
        if w == 0.0:
            k = j + 1
            continue
        c = w * 2.0 ** ((j + 1) / 2.0)
        if charge + c > budget:
            return j
        charge += c
        k = j + 1
    return k


def predicted_iterations(scheme: str, *, lambda_min: float, lambda_max: float,
                         homo: float = None, lumo: float = None, eps: float,
                         max_iter: int = 200, mu: float = None, xi: float = None,
                         poly_ij=None) -> int:
    """Iterations the scalar recurrence takes until its a-priori bound (max(beta, 1 - beta-bar),
    for P_{i,j} max(a, a')) is at most eps (the trace scheme, whose choice needs the matrix,
    is predicted by its alpha = 0 recurrence).  The fixed-mu schemes take mu and xi."""
    sch_name = "tc2" if scheme == "sp2" else scheme
    st = sch.SchemeState(sch_name, lambda_min, lambda_max, homo=homo, lumo=lumo, mu=mu, xi=xi,
                         poly_ij=poly_ij)
    for it in range(max_iter):
        if st.bound() <= eps:
            return max(it, 1)
        branch, alpha = st.choose()
        st.advance(branch, alpha)
    return max_iter


class ErrorControlledTruncation:
    """Mask for the error-controlled block truncation (rule above); call as mask(X, gap)."""

    needs_gap = True

    def __init__(self, b: int, eps: float, n_iter: int):
        self.b, self.eps, self.n_iter = b, eps, max(int(n_iter), 1)
        self.history = []              # (eps_i, k, dropped Frobenius^2) per call

    def __call__(self, X: np.ndarray, gap: float) -> np.ndarray:
        n, b = X.shape[0], self.b
        nb = n // b
        blocks = X.reshape(nb, b, nb, b)
        s = np.einsum("ibjc,ibjc->ij", blocks, blocks)
        present = np.any(blocks != 0.0, axis=(1, 3))
        upper = np.triu(present, 1)
        eps_i = self.eps * gap / (SQRT2 * self.n_iter)
        bins = half_octave_bin(s)
        k = drop_bin_limit(bins[upper], np.full(int(upper.sum()), 2.0), eps_i)
        drop = upper & (bins < k)
        drop = drop | drop.T
        self.history.append((eps_i, k, float(np.sum(s[drop]))))
        return (blocks * (~drop)[:, None, :, None]).reshape(n, n)
