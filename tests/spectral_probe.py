"""Test inputs that defeat a Krylov estimate of the spectral bounds.

The library's Lanczos estimate starts from a fixed pseudo-random unit vector
(an integer hash of the row index, mapped to (-1/2, 1/2) and normalised).  A
symmetric matrix with an isolated eigenvalue whose eigenvector is orthogonal
to that vector keeps the eigenvalue out of the Krylov space (up to rounding,
which a few steps do not amplify enough), so the estimate misses it.  The
functions here build such a matrix and replay the 16-step Lanczos estimate in
numpy, to show on the CPU that the estimate misses the eigenvalue before the
library is run on it.  No part of the method's arithmetic lives here."""
import numpy as np


def lanczos_start_vector(n: int) -> np.ndarray:
    """The fixed start vector: x_i = (h(i) >> 8 + 1/2) / 2^24 - 1/2 with the
    32-bit hash h(i) = mix(i * 2654435761 + 0x9e3779b9), normalised."""
    i = np.arange(n, dtype=np.uint64)
    m = np.uint64(0xFFFFFFFF)
    h = (i * np.uint64(2654435761) + np.uint64(0x9E3779B9)) & m
    h ^= h >> np.uint64(15)
    h = (h * np.uint64(2246822519)) & m
    h ^= h >> np.uint64(13)
    x = ((h >> np.uint64(8)).astype(np.float64) + 0.5) / 16777216.0 - 0.5
    return x / np.linalg.norm(x)


def lanczos_estimate(h: np.ndarray, k: int = 16):
    """k plain Lanczos steps (three-term recursion, no reorthogonalisation)
    from the fixed start vector; returns the interval the extreme Ritz
    values give after widening by their residual bounds |beta_k s_k| and by
    1% of the Ritz width."""
    n = h.shape[0]
    v = lanczos_start_vector(n)
    vprev = np.zeros(n)
    alpha, beta = [], []
    b_prev = 0.0
    for _ in range(k):
        w = h @ v - b_prev * vprev
        a = float(w @ v)
        w = w - a * v
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        vprev, v, b_prev = v, w / b, b
    t = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    th, s = np.linalg.eigh(t)
    r_lo, r_hi = abs(beta[-1] * s[-1, 0]), abs(beta[-1] * s[-1, -1])
    margin = 0.01 * (th[-1] - th[0])
    return th[0] - r_lo - margin, th[-1] + r_hi + margin


def hidden_outlier_workload(n: int, n_occ: int, lam_out: float, seed: int = 5):
    """Hp = lam_out z z^T + Q diag(lam) Q^T with z a unit vector orthogonal to
    the start vector and Q (n x n-1) orthonormal columns orthogonal to z
    (QR of a seeded Gaussian with z projected out); lam: n_occ values uniform
    in [-1, -0.1], the rest uniform in [0, 1] (gap 0.1 Ha at n_occ), and
    lam_out unoccupied (> 0).  Returns (hp, eigenvalues, eigenvectors as
    columns, the eigenvalue order being the columns')."""
    rng = np.random.default_rng(seed)
    v0 = lanczos_start_vector(n)
    z = rng.standard_normal(n)
    z -= (z @ v0) * v0
    z /= np.linalg.norm(z)
    z -= (z @ v0) * v0        # a second pass leaves z . v0 at rounding level
    z /= np.linalg.norm(z)
    g = rng.standard_normal((n, n - 1))
    g -= np.outer(z, z @ g)
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    q -= np.outer(z, z @ q)   # reorthogonalise against z
    q, _ = np.linalg.qr(q)
    lam = np.concatenate([rng.uniform(-1.0, -0.1, n_occ), rng.uniform(0.0, 1.0, n - 1 - n_occ)])
    lam[n_occ - 1] = -0.1
    lam[n_occ] = 0.0
    hp = (q * lam) @ q.T + lam_out * np.outer(z, z)
    hp = 0.5 * (hp + hp.T)
    vecs = np.concatenate([q, z[:, None]], axis=1)
    vals = np.concatenate([lam, [lam_out]])
    return hp, vals, vecs
