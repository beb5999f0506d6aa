"""Generators for the seeded test and benchmark workloads.

Every workload is Hp = Q diag(lam) Q^T (symmetrised in float64) where

* Q is Haar-orthogonal: the Q factor of a QR of a seeded standard Gaussian
  matrix, with column signs fixed by sign(diag R).  Above ``KRON_ABOVE`` rows a
  dense QR costs minutes on a few host cores, so Q is instead the Kronecker
  product of two Haar factors of size about sqrt(N) (still dense and exactly
  orthogonal to rounding), and the eigenvalues are placed on a seeded random
  permutation of its columns so that the occupied subspace has no Kronecker
  structure.
* lam is drawn from the recipes below, one per benchmark configuration.

The paper's own synthetic matrix (Sec. IV, Results) is ``paper_e1_matrix``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

KRON_ABOVE = 8192


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix (QR of a Gaussian, signs fixed)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


def _kron_split(n: int) -> tuple[int, int]:
    """Factor n = a*b with a <= b and a as close to sqrt(n) as possible."""
    a = int(math.isqrt(n))
    while a > 1 and n % a:
        a -= 1
    return a, n // a


# ----------------------------------------------------------------------------
# spectra (sorted ascending unless stated; all values in Hartree)
# ----------------------------------------------------------------------------

def spectrum_gapped_uniform(n: int, n_occ: int, occ_range, virt_range,
                            rng: np.random.Generator) -> np.ndarray:
    """n_occ eigenvalues uniform in occ_range, the rest uniform in virt_range.
    The top occupied value is pinned to occ_range[1] and the bottom virtual
    one to virt_range[0], so the gap is exactly virt_range[0]-occ_range[1]."""
    occ = np.sort(rng.uniform(occ_range[0], occ_range[1], n_occ))
    vir = np.sort(rng.uniform(virt_range[0], virt_range[1], n - n_occ))
    if n_occ:
        occ[-1] = occ_range[1]
    if n - n_occ:
        vir[0] = virt_range[0]
    return np.concatenate([occ, vir])


def _set_gap(lam: np.ndarray, n_occ: int, gap: float) -> np.ndarray:
    lam = np.sort(lam)
    if 0 < n_occ < lam.size:
        homo, lumo = lam[n_occ - 1], lam[n_occ]
        lam[n_occ:] -= (lumo - homo) - gap
    return lam


def spectrum_bands(n: int, n_occ: int, gap: float, rng: np.random.Generator,
                   nbands: int = 20, lo: float = -1.5, hi: float = 1.5,
                   sigma: float = 0.01) -> np.ndarray:
    """nbands Gaussian bands (width sigma) centred on linspace(lo, hi), n/nbands
    states each (the remainder goes to the top bands); then every state from
    index n_occ up is shifted down so that LUMO - HOMO == gap exactly."""
    centres = np.linspace(lo, hi, nbands)
    counts = np.full(nbands, n // nbands)
    counts[nbands - (n - counts.sum()):] += 1 if n % nbands else 0
    lam = np.concatenate([c + sigma * rng.standard_normal(k)
                          for c, k in zip(centres, counts)])
    return _set_gap(lam, n_occ, gap)


def spectrum_bands_outliers(n: int, n_occ: int, gap: float,
                            rng: np.random.Generator, frac: float = 0.01,
                            out_lo: float = 1.5, out_hi: float = 5.0) -> np.ndarray:
    """The band recipe above with a fraction ``frac`` of the unoccupied band
    states replaced by outliers uniform in [out_lo, out_hi]; gap set last."""
    lam = np.sort(spectrum_bands(n, n_occ, gap, rng))
    k = int(round(frac * n))
    idx = n_occ + rng.choice(n - n_occ, size=k, replace=False)
    lam[idx] = rng.uniform(out_lo, out_hi, k)
    return _set_gap(lam, n_occ, gap)


def spectrum_uniform(n: int, lo: float, hi: float, rng: np.random.Generator) -> np.ndarray:
    return np.sort(rng.uniform(lo, hi, n))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One seeded problem.  ``lam[k]`` is the eigenvalue of column k of Q."""

    name: str
    n: int
    n_occ: float
    kT: float
    tol: float
    lam: np.ndarray                      # eigenvalue per column of Q
    hp: np.ndarray                       # n x n float64, symmetric
    q: Optional[np.ndarray] = None       # explicit Q (Haar) ...
    q_factors: Optional[tuple] = None    # ... or (Qa, Qb, perm): Q = (Qa (x) Qb)[:, perm]

    def q_rows(self, rows) -> np.ndarray:
        """Explicit rows of Q (shape len(rows) x n)."""
        rows = np.atleast_1d(np.asarray(rows, dtype=np.int64))
        if self.q is not None:
            return self.q[rows]
        qa, qb, perm = self.q_factors
        b = qb.shape[0]
        full = (qa[rows // b][:, :, None] * qb[rows % b][:, None, :]).reshape(rows.size, -1)
        return full[:, perm]

    def q_full(self) -> np.ndarray:
        if self.q is not None:
            return self.q
        return self.q_rows(np.arange(self.n))


def _hp_from_kron(qa, qb, lam_grid):
    """Hp = (Qa (x) Qb) diag(lam) (Qa (x) Qb)^T with lam indexed [k1, k2]."""
    a, b = qa.shape[0], qb.shape[0]
    # T[k1] = Qb diag(lam[k1]) Qb^T   (a x b x b)
    t = np.einsum('ik,ck,jk->cij', qb, lam_grid, qb, optimize=True)
    # W[i1, j1, k1] = Qa[i1,k1] Qa[j1,k1]
    w = (qa[:, None, :] * qa[None, :, :]).reshape(a * a, a)
    h = (w @ t.reshape(a, b * b)).reshape(a, a, b, b)      # [i1, j1, i2, j2]
    h = np.ascontiguousarray(h.transpose(0, 2, 1, 3)).reshape(a * b, a * b)
    return h


def make_workload(name: str, lam: np.ndarray, n_occ: float, kT: float, tol: float,
                  seed: int, kron: Optional[bool] = None) -> Workload:
    """Hp = Q diag(lam) Q^T for a seeded Q (Haar, or Kronecker-Haar when large)."""
    n = lam.size
    rng = np.random.default_rng(seed)
    if kron is None:
        kron = n > KRON_ABOVE
    if not kron:
        q = haar_orthogonal(n, rng)
        hp = (q * lam[None, :]) @ q.T
        hp = 0.5 * (hp + hp.T)
        return Workload(name, n, n_occ, kT, tol, lam.copy(), hp, q=q)
    a, b = _kron_split(n)
    qa = haar_orthogonal(a, rng)
    qb = haar_orthogonal(b, rng)
    perm = rng.permutation(n)               # column perm[k] of (Qa(x)Qb) holds lam[k]
    grid = np.empty(n)
    grid[perm] = lam
    hp = _hp_from_kron(qa, qb, grid.reshape(a, b))
    hp = 0.5 * (hp + hp.T)
    return Workload(name, n, n_occ, kT, tol, lam.copy(), hp, q_factors=(qa, qb, perm))


KT_500K = 0.0016  # Ha; 500 K is 1.583e-3 Ha, rounded as in the benchmark definition

# The standard workloads: the recipes of the gapped small case, the 20-band
# case, the gapless uniform finite-temperature case and the band case with
# outliers, at their full sizes (smaller n keeps the recipe).
WORKLOADS = {
    "gapped": dict(name="gapped-n256", n=256, n_occ=64, kT=0.0, tol=1e-10, seed=1000),
    "bands": dict(name="bands-n4000-gap0.02", n=4000, n_occ=1000, kT=0.0, tol=1e-8, seed=2000),
    "uniform": dict(name="uniform-n12000-kT0.0016", n=12000, n_occ=3000, kT=KT_500K, tol=1e-8,
                    seed=3000),
    "outliers": dict(name="bands-outliers-n30000-gap0.05", n=30000, n_occ=7500, kT=0.0, tol=1e-8,
                     seed=4000),
}


def standard_workload(kind: str, n: Optional[int] = None,
                      seed_base: Optional[int] = None) -> Workload:
    """One of the standard workloads ("gapped": 64 of 256 states in
    [-1, -0.2] and the rest in [0, 1.5], gap 0.2 Ha; "bands": 20 Gaussian
    bands, gap 0.02 Ha at N/4; "uniform": uniform [-1, 1] at kT = 0.0016 Ha;
    "outliers": bands plus 1% outliers in [1.5, 5], gap 0.05 Ha), optionally
    at a smaller n with the same recipe (n_occ = n/4)."""
    cfg = WORKLOADS[kind]
    n = cfg["n"] if n is None else int(n)
    seed = cfg["seed"] if seed_base is None else seed_base
    rng = np.random.default_rng(seed + 2)
    if kind == "gapped":
        n_occ = max(1, n // 4) if n > 1 else 0
        lam = spectrum_gapped_uniform(n, n_occ, (-1.0, -0.2), (0.0, 1.5), rng)
    elif kind == "bands":
        n_occ = n // 4
        lam = spectrum_bands(n, n_occ, 0.02, rng)
    elif kind == "uniform":
        n_occ = n // 4
        lam = spectrum_uniform(n, -1.0, 1.0, rng)
    else:
        n_occ = n // 4
        lam = spectrum_bands_outliers(n, n_occ, 0.05, rng)
    name = cfg["name"] if n == cfg["n"] else f"{cfg['name']}@n{n}"
    return make_workload(name, lam, float(n_occ), cfg["kT"], cfg["tol"], seed + 1)


def serving_requests(count: int, n_lo: int = 500, n_hi: int = 16000, seed: int = 4_999_999,
                     rate: float = 1.0):
    """Request descriptors for the serving workload: log-uniform N in
    [n_lo, n_hi], n_occ = N // 4, even requests gapped (0.1 Ha gap, kT = 0),
    odd requests metallic (uniform [-1, 1], kT = 0.0016 Ha); Poisson arrivals
    with the given rate (requests per second).  Returns a list of dicts; the
    matrices are built lazily with ``make_workload`` from each request's seed."""
    rng = np.random.default_rng(seed)
    ns = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(int)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(count):
        n = int(ns[r])
        reqs.append(dict(id=r, n=n, n_occ=n // 4, kT=0.0 if r % 2 == 0 else KT_500K,
                         arrival=float(t[r]), seed=5_000_000 + r))
    return reqs


def serving_workload(req: dict) -> Workload:
    rng = np.random.default_rng(req["seed"])
    n, n_occ = req["n"], req["n_occ"]
    if req["kT"] == 0.0:
        lam = _set_gap(rng.uniform(-1.0, 1.0, n), n_occ, 0.1)
    else:
        lam = np.sort(rng.uniform(-1.0, 1.0, n))
    return make_workload(f"serve-{req['id']}-n{n}", lam, float(n_occ), req["kT"], 1e-8,
                         req["seed"] + 7)


def paper_e1_matrix(n: int) -> np.ndarray:
    """The paper's synthetic projected Hamiltonian (Sec. IV): entries
    exp(-0.5 |i-j|) sin(i+1), read with 0-based i = min(row, col) so that the
    matrix is symmetric as the paper states."""
    i = np.arange(n)
    lo = np.minimum(i[:, None], i[None, :])
    return np.exp(-0.5 * np.abs(i[:, None] - i[None, :])) * np.sin(lo + 1.0)


def paper_e1_band(n: int, bandwidth: int = 80) -> np.ndarray:
    """The paper's matrix (see paper_e1_matrix) in LAPACK upper band storage:
    ab[bandwidth - d, j] = H[j - d, j] for d = 0..bandwidth (entries further
    out are below exp(-40) and left out)."""
    bw = min(bandwidth, n - 1)
    ab = np.zeros((bw + 1, n))
    for d in range(bw + 1):
        j = np.arange(d, n)
        ab[bw - d, d:] = np.exp(-0.5 * np.abs(float(d))) * np.sin(np.minimum(j - d, j) + 1.0)
    return ab


def paper_e1_rows(n: int, r0: int, r1: int) -> np.ndarray:
    """Rows r0..r1-1 of paper_e1_matrix(n) (same arithmetic, so large matrices
    can be built a block of rows at a time)."""
    i = np.arange(r0, r1)[:, None]
    j = np.arange(n)[None, :]
    return np.exp(-0.5 * np.abs(i - j)) * np.sin(np.minimum(i, j) + 1.0)
