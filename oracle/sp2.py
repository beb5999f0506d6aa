"""Zero-temperature recursive Fermi-operator expansion (oracle; test use only).

Written from Sec. II.B.1 and Eq. (1) of the paper: starting from the
Hamiltonian, repeatedly apply one of the two second-order projection
polynomials F(X) = X^2 or F(X) = 2X - X^2, the sign chosen so that the trace of
the next iterate approaches N_occ.  Sec. III.B computes Tr(A^2) as the squared
Frobenius norm of the symmetric iterate, so both candidate traces are known
before the product.  Sec. II.C says the expansion needs spectral bounds of H;
Gershgorin discs provide them here.

Readings where the paper is silent (each is listed in the design notes):
* start: X_0 = (e_max I - H) / (e_max - e_min), which puts the spectrum in
  [0, 1] with occupied states near 1 (the paper writes X_0 = H);
* branch: X^2 iff |Tr X^2 - N_occ| <= |Tr(2X - X^2) - N_occ| (ties -> X^2);
* stop: when ||X_n^2 - X_n||_F <= tol and |Tr X_n - N_occ| <= tol the
  iterate X_n is returned (its square is the product that measured the
  idempotency), else after max_iter products;
* McWeeny refinement X <- 3X^2 - 2X^3 for the final steps of the mixed forms.
"""
from __future__ import annotations

import numpy as np


def gershgorin_bounds(h: np.ndarray):
    """(e_min, e_max) = (min_i h_ii - r_i, max_i h_ii + r_i) with
    r_i = sum_{j != i} |h_ij|: every eigenvalue lies in [e_min, e_max]."""
    n = h.shape[0]
    lo = np.inf
    hi = -np.inf
    for i in range(n):
        r = np.abs(h[i]).sum() - abs(h[i, i])
        lo = min(lo, h[i, i] - r)
        hi = max(hi, h[i, i] + r)
    return float(lo), float(hi)


def initial_iterate(h: np.ndarray, e_min: float, e_max: float) -> np.ndarray:
    """X_0 = (e_max I - H) / (e_max - e_min)."""
    n = h.shape[0]
    return (e_max * np.eye(n) - h) / (e_max - e_min)


def choose_square(trace: float, frob2: float, n_occ: float) -> bool:
    """True for X^2 (trace Tr X^2 = ||X||_F^2), False for 2X - X^2 (trace 2 Tr X - ||X||_F^2)."""
    return abs(frob2 - n_occ) <= abs(2.0 * trace - frob2 - n_occ)


def sp2(h: np.ndarray, n_occ: float, tol: float = 1e-10, max_iter: int = 100,
        bounds=None, x0=None, reltr_stop=None):
    """Plain float64 SP2.  Returns (D, info) with info holding the iteration
    count, the branch sequence (1 = X^2), the idempotency history and the
    bounds.  ``x0`` (optional) replaces the scaled start.  With
    ``reltr_stop`` the paper's criterion (Sec. III.A) replaces the
    idempotency stop: the first iterate X_{n+1} whose relative trace change
    |Tr X_{n+1} - Tr X_n| / |Tr X_n| is at most reltr_stop is returned, and
    info["iterations"] counts the products that produced it."""
    e_min, e_max = gershgorin_bounds(h) if bounds is None else bounds
    x = initial_iterate(h, e_min, e_max) if x0 is None else np.array(x0, dtype=np.float64)
    branches = []
    idem = []
    traces = []
    converged = False
    n_done = 0
    for n_done in range(max_iter):
        t = float(np.trace(x))
        s = float(np.sum(x * x))
        traces.append(t)
        sq = choose_square(t, s, n_occ)
        p = x @ x
        e = float(np.linalg.norm(p - x))
        idem.append(e)
        if reltr_stop is None and e <= tol and abs(t - n_occ) <= tol:
            converged = True
            break
        branches.append(1 if sq else 0)
        x = p if sq else 2.0 * x - p
        if reltr_stop is not None and abs(float(np.trace(x)) - t) / abs(t) <= reltr_stop:
            converged = True
            n_done += 1
            traces.append(float(np.trace(x)))
            break
    info = dict(iterations=n_done, converged=converged, branches=branches, idempotency=idem,
                traces=traces, bounds=(e_min, e_max))
    return x, info


def mcweeny(x: np.ndarray, tol: float, max_steps: int = 8, n_occ=None):
    """X <- 3X^2 - 2X^3 until ||X^2 - X||_F <= tol (and, when n_occ is given,
    |Tr X - n_occ| <= tol as in the SP2 stop rule).  Returns (X, steps, history)."""
    hist = []
    for k in range(max_steps + 1):
        p = x @ x
        e = float(np.linalg.norm(p - x))
        hist.append(e)
        ok = e <= tol and (n_occ is None or abs(float(np.trace(x)) - n_occ) <= tol)
        if ok or k == max_steps:
            return x, k, hist
        x = 3.0 * p - 2.0 * (p @ x)
    return x, max_steps, hist


def rel_trace(traces):
    """RelTr_n = |Tr X_n - Tr X_{n-1}| / |Tr X_{n-1}| (Sec. III.A)."""
    t = np.asarray(traces, dtype=np.float64)
    return np.abs(np.diff(t)) / np.abs(t[:-1])
