"""Density-matrix definitions and accuracy metrics (oracle; test use only).

Sec. II.A of the paper defines the zero-temperature density matrix as the
projector theta(mu I - H) onto the N_occ lowest eigenvectors (occupancies 0 or
1) and the finite-temperature one as the Fermi operator
[exp(beta (H - mu I)) + I]^-1 with beta = 1/(k_B T_e) (occupancies in [0, 1]).
Both are written out here from eigenpairs: D = sum_i f_i q_i q_i^T.
Sec. III.C defines the relative errors eps1 (Frobenius) and eps2 (band
energy Tr(D Hp)).
"""
from __future__ import annotations

import numpy as np

from .eig import jacobi_eigh


def occupations_zero_t(lam: np.ndarray, n_occ: int) -> np.ndarray:
    """f_i = 1 for the n_occ lowest eigenvalues, 0 otherwise (Sec. II.A).
    Raises if the n_occ-th and (n_occ+1)-th eigenvalues coincide: the
    projector is then not defined."""
    lam = np.asarray(lam, dtype=np.float64)
    n_occ = int(round(n_occ))
    order = np.argsort(lam, kind="stable")
    f = np.zeros(lam.size)
    f[order[:n_occ]] = 1.0
    if 0 < n_occ < lam.size and not lam[order[n_occ]] > lam[order[n_occ - 1]]:
        raise ValueError("no gap at n_occ: zero-temperature density matrix undefined")
    return f


def fermi_dirac(lam: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """Occupancies 1 / (exp((lam - mu)/kT) + 1), evaluated in the overflow-free
    form 1/2 (1 - tanh((lam - mu) / (2 kT)))."""
    return 0.5 * (1.0 - np.tanh((np.asarray(lam) - mu) / (2.0 * kT)))


def chemical_potential(lam: np.ndarray, n_occ: float, kT: float, tol: float = 1e-13) -> float:
    """The unique mu with sum_i f_i(mu) = n_occ, by bisection (the sum is
    strictly increasing in mu for kT > 0)."""
    lam = np.asarray(lam, dtype=np.float64)
    if not 0.0 < n_occ < lam.size:
        raise ValueError("n_occ must lie strictly between 0 and N at finite temperature")
    lo = lam.min() - 50.0 * kT
    hi = lam.max() + 50.0 * kT
    while fermi_dirac(lam, lo, kT).sum() > n_occ:
        lo -= (hi - lo)
    while fermi_dirac(lam, hi, kT).sum() < n_occ:
        hi += (hi - lo)
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        s = fermi_dirac(lam, mid, kT).sum()
        if abs(s - n_occ) <= tol or mid in (lo, hi):
            return mid
        if s < n_occ:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def occupations(lam: np.ndarray, n_occ: float, kT: float):
    """(f, mu): zero-temperature occupations for kT == 0 (mu = midgap),
    Fermi-Dirac occupations with the canonical mu otherwise."""
    lam = np.asarray(lam, dtype=np.float64)
    if kT == 0.0:
        f = occupations_zero_t(lam, n_occ)
        s = np.sort(lam)
        k = int(round(n_occ))
        mu = 0.5 * (s[k - 1] + s[k]) if 0 < k < s.size else (s[-1] if k else s[0])
        return f, mu
    mu = chemical_potential(lam, n_occ, kT)
    return fermi_dirac(lam, mu, kT), mu


def density_from_eig(q: np.ndarray, lam: np.ndarray, f: np.ndarray):
    """D = Q diag(f) Q^T and E_band = sum_i f_i lam_i (= Tr(D H))."""
    d = (q * f[None, :]) @ q.T
    return 0.5 * (d + d.T), float(np.dot(f, lam))


def eigh_lapack(h: np.ndarray):
    """Eigenpairs of symmetric h by LAPACK's dense symmetric eigensolver (a
    library routine, used where the plain Jacobi sweep is too slow: N in the
    thousands), sorted ascending.  Returns (w, V) with h ~= V diag(w) V^T."""
    w, v = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    return w, v


def density_matrix(h: np.ndarray, n_occ: float, kT: float = 0.0):
    """Reference density matrix of symmetric h by Jacobi eigendecomposition.
    Returns (D, E_band, mu, eigenvalues)."""
    lam, q = jacobi_eigh(h)
    f, mu = occupations(lam, n_occ, kT)
    d, e = density_from_eig(q, lam, f)
    return d, e, mu, lam


def density_rows(q_rows, n: int, f: np.ndarray, rows, chunk: int = 4096) -> np.ndarray:
    """Full rows D[rows, :] = Q[rows] diag(f) Q^T, built from row blocks of Q."""
    qr = q_rows(np.asarray(rows)) * f[None, :]
    out = np.empty((len(rows), n))
    for c0 in range(0, n, chunk):
        idx = np.arange(c0, min(n, c0 + chunk))
        out[:, c0:c0 + idx.size] = qr @ q_rows(idx).T
    return out


# ---------------------------------------------------------------------------
# metrics (Sec. III.C, plus the absolute checks used as gates)
# ---------------------------------------------------------------------------

def eps1(d: np.ndarray, d_ref: np.ndarray) -> float:
    """Relative Frobenius error ||D - D_ref||_F / ||D_ref||_F."""
    return float(np.linalg.norm(d - d_ref) / np.linalg.norm(d_ref))


def eps2(e: float, e_ref: float) -> float:
    """Signed relative band-energy error (Tr(D H) - Tr(D_ref H)) / Tr(D_ref H)."""
    return float((e - e_ref) / e_ref)


def band_energy(h: np.ndarray, d: np.ndarray) -> float:
    """Tr(D H) = sum_ij H_ij D_ij for symmetric H and D."""
    return float(np.sum(h * d))


def idempotency(d: np.ndarray) -> float:
    """||D^2 - D||_F."""
    return float(np.linalg.norm(d @ d - d))


def commutator(h: np.ndarray, d: np.ndarray) -> float:
    """||H D - D H||_F."""
    return float(np.linalg.norm(h @ d - d @ h))


def banded_eigenvalues(h: np.ndarray, bandwidth: int) -> np.ndarray:
    """Eigenvalues of a symmetric matrix whose entries vanish (to rounding)
    beyond `bandwidth` diagonals, by LAPACK's banded symmetric eigensolver
    (a library routine); used for the paper's synthetic matrix, whose
    entries decay like exp(-0.5 |i - j|)."""
    n = h.shape[0]
    bw = min(bandwidth, n - 1)
    ab = np.zeros((bw + 1, n))
    for d in range(bw + 1):
        ab[bw - d, d:] = np.diag(h, d)
    return band_storage_eigenvalues(ab)


def band_storage_eigenvalues(ab: np.ndarray) -> np.ndarray:
    """Eigenvalues (ascending) of the symmetric matrix held in LAPACK upper
    band storage ab[bw - d, j] = H[j - d, j], by the banded eigensolver."""
    from scipy.linalg import eig_banded
    return np.sort(eig_banded(ab, lower=False, eigvals_only=True))


def reference_energy(lam: np.ndarray, n_occ: float, kT: float):
    """(E_band, mu, occupations) from the eigenvalues alone: E = sum f_i lam_i."""
    f, mu = occupations(lam, n_occ, kT)
    return float(np.dot(f, lam)), mu, f
