"""Seeded synthetic Hamiltonians shared by the tests, the benchmark and the oracle checks.

This module only *makes inputs*: symmetric matrices F, their known spectra and eigenvectors
where the construction fixes them, the occupation count and spectral bounds.  It holds none
of the purification arithmetic (no f0, no polynomial step, no schedule); both the HIP path and
the CPU oracle consume what it returns.

Workloads (the paper's test matrices are diagonal Hamiltonians with a prescribed gap and
chemical potential, Fig. 3; by the rotation-invariance remark that follows Fig. 3, any
Hamiltonian with the same gap and chemical potential behaves the same, so rotated spectra
stand in for them):

* ``random_spectrum_hamiltonian`` -- F = Q diag(lam) Q^T with Q Haar-orthogonal (QR of a
  standard-normal matrix with the sign of diag(R) folded into Q's columns) and lam drawn
  uniformly in an occupied and an unoccupied interval, the four interval edges included
  exactly.
* ``lattice_hamiltonian`` -- two-orbital cubic tight-binding lattice, periodic, orbital 0 at
  +0.5 and orbital 1 at -0.5 on-site energy plus uniform disorder, hopping -0.1 between all
  four orbital pairs of nearest-neighbour sites (the gapped reading of the lattice workload).
* ``lattice_bsr`` -- the same lattice in 32x32 block-sparse row form, sites grouped in
  4x2x2 bricks ordered by the Morton code of the brick coordinates.
* ``serving_trace`` -- a stream of independent purification requests of mixed size.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Hamiltonian:
    """A symmetric test Hamiltonian and the inputs a purification call needs.

    ``eigvals`` / ``Q`` are set when the construction fixes the spectrum exactly
    (rotated random spectra); lattice inputs carry eigenvalues from a dense symmetric
    eigensolver (used only to place the bounds) and ``Q = None``.
    """

    name: str
    F: np.ndarray                 # (n, n) float64, row-major, exactly symmetric
    n_occ: int
    lambda_min: float             # bounds of the whole spectrum (outer)
    lambda_max: float
    homo: float                   # bounds of the gap edges passed to the method
    lumo: float
    mu: float                     # chemical potential (middle of the gap)
    xi: float                     # gap width used by the fixed-mu schemes
    eigvals: Optional[np.ndarray] = None
    Q: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.F.shape[0])


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix (QR of a Gaussian matrix, sign-fixed)."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def two_interval_spectrum(n_occ: int, n_unocc: int, lo: float, homo: float, lumo: float,
                          hi: float, rng: np.random.Generator) -> np.ndarray:
    """Ascending eigenvalues: n_occ in [lo, homo], n_unocc in [lumo, hi], edges exact."""
    if n_occ < 1 or n_unocc < 1:
        raise ValueError("need at least one occupied and one unoccupied level")
    parts = []
    for cnt, a, b, edge in ((n_occ, lo, homo, homo), (n_unocc, lumo, hi, lumo)):
        if cnt == 1:
            parts.append(np.array([edge]))   # a lone level sits on the gap edge
            continue
        inner = rng.uniform(a, b, size=cnt - 2)
        parts.append(np.sort(np.concatenate(([a], inner, [b]))))
    return np.concatenate(parts)


def rotate_spectrum(eigvals: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """F = Q diag(eigvals) Q^T, then symmetrised so F is exactly symmetric in FP64."""
    f = (Q * eigvals[None, :]) @ Q.T
    return 0.5 * (f + f.T)


def random_spectrum_hamiltonian(n: int, n_occ: int, lo: float, homo: float, lumo: float,
                                hi: float, seed: int, name: str = "random",
                                rotate: bool = True) -> Hamiltonian:
    """Rotated two-interval random spectrum with exactly known edges.

    The bounds handed to the method are the exact interval edges; ``mu`` is the middle of
    the gap and ``xi`` its width (the gap is symmetric about ``mu`` by construction).
    With ``rotate=False`` F is the diagonal matrix itself (the paper's diagonal tests).
    """
    rng = np.random.default_rng(seed)
    lam = two_interval_spectrum(n_occ, n - n_occ, lo, homo, lumo, hi, rng)
    if rotate:
        Q = haar_orthogonal(n, rng)
        F = rotate_spectrum(lam, Q)
    else:
        Q = np.eye(n)
        F = np.diag(lam).astype(np.float64)
    return Hamiltonian(name=name, F=np.ascontiguousarray(F), n_occ=n_occ,
                       lambda_min=float(lo), lambda_max=float(hi), homo=float(homo),
                       lumo=float(lumo), mu=0.5 * (homo + lumo), xi=float(lumo - homo),
                       eigvals=lam, Q=Q)


# ----------------------------------------------------------------------------------------
# The named workloads
# ----------------------------------------------------------------------------------------

def small_gap_256(seed: int = 1101) -> Hamiltonian:
    """n=256: 128 levels uniform in [-1,-0.025], 128 in [0.025,1]; gap 0.05 about mu=0."""
    return random_spectrum_hamiltonian(256, 128, -1.0, -0.025, 0.025, 1.0, seed,
                                       name="dense-n256-gap0.05")


def tiny_gap_8192(seed: int = 4, n: int = 8192) -> Hamiltonian:
    """Spectrum in [-1,1] with a 1e-3 gap centred at mu=0.1, N_occ=4506 (n=8192).

    For smaller ``n`` the occupied fraction is kept (N_occ = round(n*4506/8192)).
    """
    n_occ = 4506 if n == 8192 else int(round(n * 4506 / 8192))
    return random_spectrum_hamiltonian(n, n_occ, -1.0, 0.0995, 0.1005, 1.0, seed,
                                       name=f"dense-n{n}-gap1e-3")


def fig3_diagonal(n: int, mu01: float, xi: float, seed: int = 0,
                  rotate: bool = False) -> Hamiltonian:
    """Diagonal test Hamiltonian of the paper's Fig. 3: spectral width 1, spectrum [0,1],
    chemical potential ``mu01`` in ]0,1[, gap ``xi`` centred on it.

    The number of occupied levels follows the position of the gap (about n*mu01, at least 1
    on each side).
    """
    homo = mu01 - 0.5 * xi
    lumo = mu01 + 0.5 * xi
    n_occ = min(max(int(round(n * mu01)), 1), n - 1)
    return random_spectrum_hamiltonian(n, n_occ, 0.0, homo, lumo, 1.0, seed,
                                       name=f"diag-mu{mu01}-xi{xi}", rotate=rotate)


# ----------------------------------------------------------------------------------------
# Two-orbital cubic tight-binding lattice
# ----------------------------------------------------------------------------------------

ONSITE = 0.5
DISORDER = 0.05
HOPPING = -0.1


def _lattice_onsite(L: tuple, seed: int) -> np.ndarray:
    """On-site energies indexed [x, y, z, orbital]."""
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = L
    base = np.empty((Lx, Ly, Lz, 2))
    base[..., 0] = ONSITE
    base[..., 1] = -ONSITE
    return base + rng.uniform(-DISORDER, DISORDER, size=base.shape)


def _neighbour_pairs(L: tuple):
    """Yield (site_a, site_b) index arrays for +x, +y, +z periodic bonds (site = (x,y,z))."""
    Lx, Ly, Lz = L
    x, y, z = np.meshgrid(np.arange(Lx), np.arange(Ly), np.arange(Lz), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    for dx, dy, dz in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        yield (x, y, z), ((x + dx) % Lx, (y + dy) % Ly, (z + dz) % Lz)


def lattice_hamiltonian(L: tuple = (16, 16, 8), seed: int = 2, with_bounds: bool = True,
                        pad: float = 1e-12) -> Hamiltonian:
    """Dense two-orbital lattice Hamiltonian, orbital index 2*site + o, site lexicographic.

    Half filling (N_occ = n/2).  Bounds come from a dense symmetric eigensolver, widened
    outwards by ``pad``: lambda_min/max outside the spectrum, homo below the highest
    occupied level and lumo above the lowest unoccupied one.
    """
    Lx, Ly, Lz = L
    nsite = Lx * Ly * Lz
    n = 2 * nsite
    onsite = _lattice_onsite(L, seed)
    F = np.zeros((n, n))
    sid = lambda x, y, z: (x * Ly + y) * Lz + z  # noqa: E731
    F[np.arange(n), np.arange(n)] = onsite.reshape(-1)
    for a, b in _neighbour_pairs(L):
        sa, sb = sid(*a), sid(*b)
        for oa in range(2):
            for ob in range(2):
                np.add.at(F, (2 * sa + oa, 2 * sb + ob), HOPPING)
                np.add.at(F, (2 * sb + ob, 2 * sa + oa), HOPPING)
    n_occ = n // 2
    h = Hamiltonian(name=f"lattice-{Lx}x{Ly}x{Lz}", F=F, n_occ=n_occ, lambda_min=0.0,
                    lambda_max=0.0, homo=0.0, lumo=0.0, mu=0.0, xi=0.0)
    if with_bounds:
        ev = np.linalg.eigvalsh(F)
        set_bounds_from_eigvals(h, ev, pad)
    return h


def set_bounds_from_eigvals(h: Hamiltonian, ev: np.ndarray, pad: float = 1e-12) -> None:
    """Outer bounds: [lambda_min, lambda_max] contains the spectrum and [homo, lumo]
    contains the gap, each widened by ``pad``; mu mid-gap, xi = twice the distance from mu
    to the nearer widened edge."""
    ev = np.sort(ev)
    h.eigvals = ev
    h.lambda_min = float(ev[0] - pad)
    h.lambda_max = float(ev[-1] + pad)
    h.homo = float(ev[h.n_occ - 1] - pad)
    h.lumo = float(ev[h.n_occ] + pad)
    h.mu = 0.5 * (h.homo + h.lumo)
    h.xi = h.lumo - h.homo


def lattice_clean_band_edges(L: tuple) -> tuple:
    """Band edges of the disorder-free lattice, E = eps +- sqrt(eps^2 + 0.25) with
    eps(k) = 2*HOPPING*sum_d cos k_d over the periodic k-grid.  Returns
    (lambda_min, homo, lumo, lambda_max) of the clean spectrum."""
    ks = [2.0 * np.pi * np.arange(l) / l for l in L]
    cx, cy, cz = (np.cos(k) for k in ks)
    eps = 2.0 * HOPPING * (cx[:, None, None] + cy[None, :, None] + cz[None, None, :])
    root = np.sqrt(eps * eps + ONSITE * ONSITE)
    lower, upper = eps - root, eps + root
    return float(lower.min()), float(lower.max()), float(upper.min()), float(upper.max())


# ---- block-sparse (BSR) form --------------------------------------------------------------

BRICK = (4, 2, 2)  # sites per brick along x, y, z; 16 sites x 2 orbitals = 32 rows


def _morton3(bx: np.ndarray, by: np.ndarray, bz: np.ndarray, bits: int) -> np.ndarray:
    code = np.zeros_like(bx, dtype=np.int64)
    for b in range(bits):
        code |= ((bx >> b) & 1).astype(np.int64) << (3 * b)
        code |= ((by >> b) & 1).astype(np.int64) << (3 * b + 1)
        code |= ((bz >> b) & 1).astype(np.int64) << (3 * b + 2)
    return code


def lattice_orbital_order(L: tuple) -> np.ndarray:
    """perm[site*2+o] = row index in brick/Morton order (bricks 4x2x2 sites, orbitals within
    a brick ordered by (local x, local y, local z, orbital))."""
    Lx, Ly, Lz = L
    bx_, by_, bz_ = BRICK
    if Lx % bx_ or Ly % by_ or Lz % bz_:
        raise ValueError("lattice extent must be a multiple of the 4x2x2 brick")
    NBx, NBy, NBz = Lx // bx_, Ly // by_, Lz // bz_
    bbx, bby, bbz = np.meshgrid(np.arange(NBx), np.arange(NBy), np.arange(NBz), indexing="ij")
    bits = int(max(NBx, NBy, NBz) - 1).bit_length() or 1
    code = _morton3(bbx.ravel(), bby.ravel(), bbz.ravel(), bits)
    brick_rank = np.empty(code.size, dtype=np.int64)
    brick_rank[np.argsort(code, kind="stable")] = np.arange(code.size)
    brick_rank = brick_rank.reshape(NBx, NBy, NBz)
    x, y, z = np.meshgrid(np.arange(Lx), np.arange(Ly), np.arange(Lz), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    rank = brick_rank[x // bx_, y // by_, z // bz_]
    local = ((x % bx_) * by_ + (y % by_)) * bz_ + (z % bz_)
    per_brick = 2 * bx_ * by_ * bz_
    perm = np.empty(2 * x.size, dtype=np.int64)
    for o in range(2):
        perm[2 * np.arange(x.size) + o] = rank * per_brick + 2 * local + o
    return perm


@dataclasses.dataclass
class BSRMatrix:
    """Host-side block-sparse row matrix: square blocks of side ``b``, each row-major."""

    n: int
    b: int
    row_ptr: np.ndarray   # int32 (nb+1,)
    col_idx: np.ndarray   # int32 (nnzb,), ascending within each block row
    val: np.ndarray       # float32 or float64 (nnzb, b, b)

    @property
    def nb(self) -> int:
        return self.n // self.b

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.size)

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=np.float64)
        b = self.b
        for i in range(self.nb):
            for p in range(self.row_ptr[i], self.row_ptr[i + 1]):
                j = self.col_idx[p]
                d[i * b:(i + 1) * b, j * b:(j + 1) * b] = self.val[p]
        return d


def dense_to_bsr(d: np.ndarray, b: int, dtype=np.float32) -> BSRMatrix:
    """Keep every block with at least one non-zero entry (structural pattern of ``d``)."""
    n = d.shape[0]
    if n % b:
        raise ValueError("n must be a multiple of the block size")
    nb = n // b
    blocks = d.reshape(nb, b, nb, b).transpose(0, 2, 1, 3)
    mask = np.any(blocks != 0.0, axis=(2, 3))
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(nb + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    val = np.ascontiguousarray(blocks[rows, cols].astype(dtype))
    return BSRMatrix(n=n, b=b, row_ptr=row_ptr, col_idx=cols.astype(np.int32), val=val)


def lattice_bsr(L: tuple = (32, 32, 32), seed: int = 3, b: int = 32,
                dtype=np.float32) -> tuple:
    """Lattice Hamiltonian in brick/Morton-ordered BSR form, built without a dense n x n.

    Returns (BSRMatrix, Hamiltonian-with-F=None-equivalent bounds).  Bounds are rigorous:
    the clean band edges (analytic) moved outward by the disorder amplitude (Weyl), i.e. a
    lower bound of the highest occupied level and an upper bound of the lowest unoccupied one.
    """
    if b != 2 * BRICK[0] * BRICK[1] * BRICK[2]:
        raise ValueError("block size must equal the 4x2x2-site brick (32)")
    Lx, Ly, Lz = L
    nsite = Lx * Ly * Lz
    n = 2 * nsite
    perm = lattice_orbital_order(L)
    onsite = _lattice_onsite(L, seed).reshape(-1)
    sid = lambda x, y, z: (x * Ly + y) * Lz + z  # noqa: E731
    rows = [perm[np.arange(n)]]
    cols = [perm[np.arange(n)]]
    vals = [onsite]
    for a, bb in _neighbour_pairs(L):
        sa, sb = sid(*a), sid(*bb)
        for oa in range(2):
            for ob in range(2):
                ia, ib = perm[2 * sa + oa], perm[2 * sb + ob]
                rows += [ia, ib]
                cols += [ib, ia]
                vals += [np.full(ia.size, HOPPING), np.full(ia.size, HOPPING)]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    nb = n // b
    br, bc = r // b, c // b
    key = br * nb + bc
    ukey, inv = np.unique(key, return_inverse=True)
    val = np.zeros((ukey.size, b, b), dtype=np.float64)
    np.add.at(val, (inv, r % b, c % b), v)
    urow, ucol = ukey // nb, ukey % nb
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(row_ptr, urow + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    m = BSRMatrix(n=n, b=b, row_ptr=row_ptr, col_idx=ucol.astype(np.int32),
                  val=np.ascontiguousarray(val.astype(dtype)))
    lmin, homo, lumo, lmax = lattice_clean_band_edges(L)
    h = Hamiltonian(name=f"lattice-bsr-{Lx}x{Ly}x{Lz}", F=np.zeros((0, 0)), n_occ=n // 2,
                    lambda_min=lmin - DISORDER, lambda_max=lmax + DISORDER,
                    homo=homo - DISORDER, lumo=lumo + DISORDER, mu=0.5 * (homo + lumo),
                    xi=(lumo + DISORDER) - (homo - DISORDER))
    return m, h


# ----------------------------------------------------------------------------------------
# Serving trace
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    arrival_s: float
    n: int
    n_occ: int
    xi: float
    seed: int


def serving_trace(count: int = 512, rate_per_s: float = 100.0, seed: int = 5,
                  n_lo: int = 64, n_hi: int = 2048, xi_lo: float = 1e-3,
                  xi_hi: float = 1e-1) -> list:
    """Poisson arrivals at ``rate_per_s``; n log-uniform in [n_lo, n_hi]; gap log-uniform
    in [xi_lo, xi_hi]; N_occ = round(n/2 * (1 + U(-0.1, 0.1)))."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        xi = float(math.exp(rng.uniform(math.log(xi_lo), math.log(xi_hi))))
        n_occ = int(round(0.5 * n * (1.0 + rng.uniform(-0.1, 0.1))))
        n_occ = min(max(n_occ, 1), n - 1)
        out.append(Request(arrival_s=t, n=n, n_occ=n_occ, xi=xi, seed=seed * 100003 + k))
    return out


def request_hamiltonian(req: Request) -> Hamiltonian:
    """Spectrum uniform on [-1,1] with a gap of width xi placed so exactly N_occ levels lie
    below it (edges included), rotated by a Haar Q seeded per request."""
    n, k, xi = req.n, req.n_occ, req.xi
    # Place the gap where a uniform density on [-1, 1] would put the k-th level.
    centre = -1.0 + 2.0 * k / n
    centre = min(max(centre, -1.0 + xi), 1.0 - xi)
    homo, lumo = centre - 0.5 * xi, centre + 0.5 * xi
    return random_spectrum_hamiltonian(n, k, -1.0, homo, lumo, 1.0, req.seed,
                                       name=f"req-n{n}")


def request_hamiltonian_torch(req: Request, device: str = "cuda:0",
                              keep_on_device: bool = False) -> Hamiltonian:
    """As ``request_hamiltonian`` but with the Haar rotation drawn and applied on the GPU
    (torch, seeded per request), for traces too large for host QR.  F is returned on the
    host, or as the device tensor with ``keep_on_device``.
    """
    import torch

    n, k, xi = req.n, req.n_occ, req.xi
    centre = -1.0 + 2.0 * k / n
    centre = min(max(centre, -1.0 + xi), 1.0 - xi)
    homo, lumo = centre - 0.5 * xi, centre + 0.5 * xi
    rng = np.random.default_rng(req.seed)
    lam = two_interval_spectrum(k, n - k, -1.0, homo, lumo, 1.0, rng)
    g = torch.Generator(device=device)
    g.manual_seed(int(req.seed))
    z = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
    q, r = torch.linalg.qr(z)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    q = q * d[None, :]
    f = (q * torch.tensor(lam, device=device)[None, :]) @ q.T
    f = 0.5 * (f + f.T)
    return Hamiltonian(name=f"req-n{n}", F=f.contiguous() if keep_on_device else f.cpu().numpy(),
                       n_occ=k, lambda_min=-1.0,
                       lambda_max=1.0, homo=float(homo), lumo=float(lumo),
                       mu=0.5 * (homo + lumo), xi=float(lumo - homo), eigvals=lam, Q=None)


def rotated_spectrum_torch(eigvals: np.ndarray, seed: int, device: str = "cuda:0") -> tuple:
    """(F, Q) as device tensors: F = Q diag(eigvals) Q^T symmetrised, Q Haar-orthogonal drawn
    on the GPU (QR of a seeded Gaussian, sign-fixed).  For orders where host QR is slow."""
    import torch

    n = eigvals.size
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    z = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
    q, r = torch.linalg.qr(z)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    q = q * d[None, :]
    f = (q * torch.tensor(eigvals, device=device)[None, :]) @ q.T
    return (0.5 * (f + f.T)).contiguous(), q
