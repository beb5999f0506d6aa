"""Truncated zero-temperature expansion used as a smeared step, T-RFOE
(oracle; test use only).

Sec. II.B.3 and Eq. (2) of the paper: for finite temperature an intermediate
iterate of the zero-temperature expansion of Sec. II.B.1 -- the SP2 maps
F(X) = X^2 or 2X - X^2 with the branch steering the trace towards the
electron count -- taken before it has converged to a projector, G_m(H) =
F_m(...F_0(H)), serves as a smeared step function.  The paper says only that
a lower temperature needs more steps m.  The reading used here (listed with
the other readings in the design notes): m is the smallest depth whose slope
at the Fermi level reaches the Fermi function's slope beta/4 per Hartree.
Near the Fermi level the trace-steered iteration follows the unstable
2-cycle of the two maps, the points (3 - sqrt 5)/2 and (sqrt 5 - 1)/2, where
each map has derivative sqrt(5) - 1; X_0 has slope 1 / (e_max - e_min).

Two forms: ``scalar`` applies the steps to the eigenvalues (a diagonal H),
``dense`` to the matrix.  Both take the branch from the traces exactly as
Z-RFOE does; D = X_m.  The result is pinned against itself (the dense
iteration against the spectral form) and against properties of the maps; the
depth rule has no counterpart in the paper.
"""
from __future__ import annotations

import math

import numpy as np

from .sp2 import choose_square, gershgorin_bounds, initial_iterate

GROWTH = math.sqrt(5.0) - 1.0   # derivative of x^2 at (sqrt 5 - 1)/2 and of 2x - x^2 at (3 - sqrt 5)/2


def depth(kT: float, e_min: float, e_max: float) -> int:
    """Smallest m with GROWTH^m >= (e_max - e_min) / (4 kT) (at least 1)."""
    need = (e_max - e_min) / (4.0 * kT)
    return max(1, int(math.ceil(math.log(need) / math.log(GROWTH)))) if need > 1.0 else 1


def scalar(lam, n_occ: float, kT: float, e_min: float, e_max: float, m=None):
    """Occupations g_i = G_m(lam_i) of the truncated expansion on the
    eigenvalues.  Returns (g, info) with the branches (1 = X^2) and m."""
    m = depth(kT, e_min, e_max) if m is None else int(m)
    x = (e_max - np.asarray(lam, dtype=np.float64)) / (e_max - e_min)
    branches = []
    for _ in range(m):
        t, s = float(x.sum()), float((x * x).sum())
        sq = choose_square(t, s, n_occ)
        branches.append(1 if sq else 0)
        x = x * x if sq else 2.0 * x - x * x
    return x, dict(branches=branches, depth=m)


def dense(h: np.ndarray, n_occ: float, kT: float, bounds=None, m=None):
    """The same expansion on the matrix: X_0 = (e_max I - H)/(e_max - e_min)
    (Gershgorin bounds unless given), m SP2 products with trace-chosen
    branches.  Returns (D, info)."""
    e_min, e_max = gershgorin_bounds(h) if bounds is None else bounds
    m = depth(kT, e_min, e_max) if m is None else int(m)
    x = initial_iterate(h, e_min, e_max)
    branches = []
    for _ in range(m):
        t, s = float(np.trace(x)), float(np.sum(x * x))
        sq = choose_square(t, s, n_occ)
        branches.append(1 if sq else 0)
        p = x @ x
        x = p if sq else 2.0 * x - p
    return x, dict(branches=branches, depth=m, bounds=(e_min, e_max))
