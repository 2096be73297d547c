"""Write fig3_counts.txt: the product counts of the setting of Fig. 3, from the oracle.

The paper shows Fig. 3 as plots only (no printed values), so this table is the oracle's:
multiplications until ||D~ - D||_2 <= 1e-9 for Hamiltonians with spectral width 1 and exact
bounds -- panel (a) gap 0.01 at several chemical potentials, panel (b) mu = 0.5 (the middle of
the spectrum) at several gaps -- for the regular schemes (McWeeny, i.e. Algorithm 1 with
alpha = 1, and the alpha = 0 form of Algorithm 2) and the scaled ones (Algorithms 1 and 2).
With exact bounds the error of a diagonal test matrix after k products equals the scalar
bound max(beta, 1 - beta-bar), which ``oracle.spectral.products_to_accuracy`` iterates.

Run from the repository root: python tests/golden/make_fig3_counts.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import spectral  # noqa: E402

MU_GRID = (0.05, 0.1, 0.2, 0.25, 0.3, 0.4, 0.5, 0.6, 0.75, 0.9, 0.95)
XI_GRID = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)
SCHEMES = ("mcweeny", "snf_fixmu", "tc2", "snf_varmu")


def rows():
    out = []
    for mu in MU_GRID:
        out.append(("a", mu, 0.01) + tuple(spectral.products_to_accuracy(s, mu, 0.01)
                                           for s in SCHEMES))
    for xi in XI_GRID:
        out.append(("b", 0.5, xi) + tuple(spectral.products_to_accuracy(s, 0.5, xi)
                                          for s in SCHEMES))
    return out


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig3_counts.txt")
    with open(path, "w") as fh:
        fh.write("# Fig. 3 setting (spectral width 1, exact bounds, ||D~ - D||_2 <= 1e-9):\n")
        fh.write("# multiplications per scheme; panel a: gap 0.01, varying mu; panel b: mu 0.5,\n")
        fh.write("# varying gap.  Written by tests/golden/make_fig3_counts.py from the oracle\n")
        fh.write("# (the paper plots these counts; it prints no values).\n")
        fh.write("# panel mu xi " + " ".join(SCHEMES) + "\n")
        for r in rows():
            fh.write(f"{r[0]} {r[1]:g} {r[2]:g} " + " ".join(str(v) for v in r[3:]) + "\n")


if __name__ == "__main__":
    main()
