"""Spectral oracle: the purification schemes applied to eigenvalues (test infrastructure only).

Every f_i of Eq. 1 is a polynomial, so X_i = Q p_i(Lambda) Q^T and the iteration acts on each
eigenvalue of X_0 independently.  This is also the paper's own argument for testing on
diagonal Hamiltonians (remark following Fig. 3: results for a given gap and chemical potential
hold for any Hamiltonian with that gap and potential).  Per iteration it gives, at O(n) cost:
tr X = sum p, ||X||_F^2 = tr X^2 = sum p^2, ||X^2 - X||_F = sqrt(sum (p^2 - p)^2), the branch
and alpha sequence, and the product count.

Stopping rule (the algorithms leave the loop length open; reading used throughout): before
applying f_i, the product X_{i-1}^2 is formed; if ||X_{i-1}^2 - X_{i-1}||_F <= tol the result is
D = X_{i-1} and that certifying product is counted.  Algorithm 1 spends two products per
iteration (X_s^2 and X_s^3), the other schemes one.

Parity: pinned against the dense oracle and the eigendecomposition (tests).
"""
from __future__ import annotations

import math

import numpy as np

from . import polynomials as poly
from . import schedule as sch


def f0_eigs(eigvals: np.ndarray, scheme: str, lambda_min: float, lambda_max: float,
            mu: float = None, st: "sch.SchemeState" = None) -> np.ndarray:
    """Eigenvalues of X_0 = f_0(F) (Algorithm 2 / trace scheme, or Algorithm 1; the P_{i,j}
    schemes centre mu on their fixed point x* with the scale ``st.gamma``)."""
    lam = np.asarray(eigvals, dtype=np.float64)
    if scheme in ("sp2", "tc2", "snf_varmu"):
        return (lambda_max - lam) / (lambda_max - lambda_min)
    if scheme in sch.GENERAL:
        return (mu - lam) / st.gamma + st.xs
    gamma = sch.alg1_gamma(lambda_min, lambda_max, mu)
    return (mu - lam) / gamma + 0.5


def apply_branch(p: np.ndarray, branch: str, alpha: float,
                 st: "sch.SchemeState" = None) -> np.ndarray:
    """One f_i on eigenvalues, written as the paper's transformation."""
    if branch == sch.SQUARE:                 # P_{1,0}((1+a) x - a), Eq. 4
        y = (1.0 + alpha) * p - alpha
        return y * y
    if branch == sch.FOLD:                   # P_{0,1}((1+a) x), Eq. 5
        z = (1.0 + alpha) * p
        return 2.0 * z - z * z
    if branch == sch.PIJ:                    # P_{i,j}(a (x - x*) + x*)
        return poly.pij(st.i, st.j, alpha * (p - st.xs) + st.xs)
    xs = alpha * (p - 0.5) + 0.5             # P_{m,m}(a (x - 1/2) + 1/2), Eq. 2
    if branch == sch.MCW:
        return 3.0 * xs * xs - 2.0 * xs * xs * xs
    return poly.pmm(3 if branch == sch.PMM[3] else 5, xs)


products_per_iteration = sch.products_per_iteration


def purify_spectrum(eigvals: np.ndarray, scheme: str, *, lambda_min: float,
                    lambda_max: float, n_occ: int = None, homo: float = None,
                    lumo: float = None, mu: float = None, xi: float = None,
                    tol: float = 1e-10, max_iter: int = 200, poly_ij=None,
                    force_branches: str = None) -> dict:
    """Run ``scheme`` on the spectrum; returns the final eigenvalues of D and the log.

    Returned keys: status ("ok" | "noconv" | "nonfinite"), p (eigenvalues of D), iterations,
    products, branches (string of S/F/M), log (list of per-iteration dicts with i, branch,
    alpha, beta, betabar, e, t1, t2 of X_{i-1} before the step, and for the trace scheme the
    margin of its choice), e_final, trace.  ``force_branches`` replays a given branch string
    for the trace scheme (an FP64 near-tie of the trace rule resolved the other way by another
    implementation).
    """
    st = sch.SchemeState(scheme, lambda_min, lambda_max, homo=homo, lumo=lumo, mu=mu, xi=xi,
                         poly_ij=poly_ij)
    p = f0_eigs(eigvals, scheme, lambda_min, lambda_max, mu, st)
    per_it = products_per_iteration(scheme, poly_ij)
    log, branches = [], []
    products = 0
    status = "noconv"
    for it in range(max_iter + 1):
        t1 = float(np.sum(p))
        t2 = float(np.sum(p * p))
        e = math.sqrt(float(np.sum((p * p - p) ** 2)))
        products += 1                              # the product X_{i-1}^2
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
        p = apply_branch(p, branch, alpha, st)
        st.advance(branch, alpha)
        products += per_it - 1                     # Algorithm 1's second product
    return dict(status=status, p=p, iterations=len(branches), products=products,
                branches="".join(branches), log=log, e_final=log[-1]["e"],
                trace=float(np.sum(p)))


def decision_sequence(scheme: str, *, lambda_min: float, lambda_max: float, homo: float,
                      lumo: float, mu: float = None, xi: float = None,
                      steps: int = 64, poly_ij=None) -> list:
    """(branch, alpha, beta, betabar) for the first ``steps`` iterations of the scalar
    recurrence alone (Algorithms 1 and 2 decide without looking at X)."""
    st = sch.SchemeState(scheme, lambda_min, lambda_max, homo=homo, lumo=lumo, mu=mu, xi=xi,
                         poly_ij=poly_ij)
    out = []
    for _ in range(steps):
        branch, alpha = st.choose()
        out.append((branch, alpha, st.beta, st.betabar))
        st.advance(branch, alpha)
    return out


def products_to_accuracy(scheme: str, mu01: float, xi: float, acc: float = 1e-9,
                         max_iter: int = 200) -> int:
    """Products needed until the eigenvalue error bound max(beta, 1 - beta-bar) <= acc for a
    spectrum in [0, 1] with a gap of width xi centred at mu01 and exact bounds (the setting of
    Fig. 3; with exact bounds this bound equals ||D~ - D||_2 of a diagonal test matrix).

    The unscaled trace scheme ("sp2") is not covered: its choice needs the whole spectrum.
    """
    homo, lumo = mu01 - 0.5 * xi, mu01 + 0.5 * xi
    # (Algorithm 1 maps mu onto 0.5; the level nearest 0.5 is xi/2 away in F-space)
    kw = dict(lambda_min=0.0, lambda_max=1.0, homo=homo, lumo=lumo, mu=mu01, xi=xi)
    st = sch.SchemeState(scheme, **kw)
    per_it = products_per_iteration(scheme)
    prods = 0
    for _ in range(max_iter):
        if st.bound() <= acc:
            return prods
        branch, alpha = st.choose()
        st.advance(branch, alpha)
        prods += per_it
    raise RuntimeError("did not reach the requested accuracy")


def products_to_accuracy_pij(poly_ij, *, lambda_min: float, lambda_max: float, mu: float,
                             xi: float, acc: float = 1e-9, scaled: bool = True,
                             max_iter: int = 200) -> int:
    """Products of the P_{i,j} fixed-mu scheme until max(a, a-bar) <= acc, for a spectrum in
    [lambda_min, lambda_max] with a gap of width xi centred at mu and exact bounds."""
    st = sch.SchemeState("snf_pij" if scaled else "pij", lambda_min, lambda_max, mu=mu, xi=xi,
                         poly_ij=poly_ij)
    per_it = products_per_iteration(st.scheme, poly_ij)
    prods = 0
    for _ in range(max_iter):
        if st.bound() <= acc:
            return prods
        branch, alpha = st.choose()
        st.advance(branch, alpha)
        prods += per_it
    raise RuntimeError("did not reach the requested accuracy")
