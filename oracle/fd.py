"""Finite-temperature recursion (oracle; test use only).

Sec. II.A defines the finite-temperature density matrix as the Fermi operator
[exp(beta(H - mu I)) + I]^-1; Sec. II.B.3 approximates it by composing
projection maps.  The GPU path uses the composition that reproduces the Fermi
operator exactly in the limit: with y = 1/2 - x the SP2-style map
x -> x^2 / (x^2 + (1 - x)^2) becomes y -> 2y / (1 + 4y^2), i.e.
(1/2) tanh(a) -> (1/2) tanh(2a).  Starting from Y_0 = beta (H - mu I) / 2^(m+2)
and applying it m times gives

    D_m = 1/2 I - Y_m,   f_m(e) = 1/2 - 1/2 tanh(2^m atanh(beta (e - mu) / 2^(m+1))),

which tends to the Fermi function as m grows.  Here the recursion runs in
float64 with an exact linear solve for the inverse; ``closed_form`` is f_m.
"""
from __future__ import annotations

import math

import numpy as np


def depth(beta: float, e_min: float, e_max: float, mu: float, extra: int = 6) -> int:
    """m = ceil(log2(beta * max(e_max - mu, mu - e_min))) + extra (>= 1)."""
    r = beta * max(e_max - mu, mu - e_min, 1e-300)
    return max(1, int(math.ceil(math.log2(r))) + extra)


def closed_form(e, mu: float, beta: float, m: int):
    """f_m(e) = 1/2 - 1/2 tanh(2^m atanh(beta (e - mu) / 2^(m+1)))."""
    z = beta * (np.asarray(e, dtype=np.float64) - mu) / 2.0 ** (m + 1)
    return 0.5 - 0.5 * np.tanh(2.0 ** m * np.arctanh(z))


def doubling(h: np.ndarray, mu: float, beta: float, m: int) -> np.ndarray:
    """D_m by the matrix recursion Y <- 2 Y (I + 4 Y^2)^-1 (exact solve)."""
    n = h.shape[0]
    eye = np.eye(n)
    y = beta * (h - mu * eye) / 2.0 ** (m + 2)
    for _ in range(m):
        a = eye + 4.0 * (y @ y)
        y = np.linalg.solve(a, 2.0 * y)
        y = 0.5 * (y + y.T)
    return 0.5 * eye - y
