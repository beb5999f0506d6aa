"""Accelerated zero-temperature expansion, A-Z-RFOE (oracle; test use only).

Written from Sec. II.B.2 of the paper: the SP2 projection polynomials of
Eq. (1) are shifted and scaled, the choice made from the HOMO and LUMO
eigenvalues, so that each step pushes the eigenvalues towards 0 or 1 faster
than X^2 or 2X - X^2 do.  The paper gives no formulas; the reading used here
(listed with the other readings in the design notes):

* X_0 = (e_max I - H) / (e_max - e_min) as in the plain expansion.  A caller's
  bounds homo >= eps_HOMO and lumo <= eps_LUMO (homo < lumo) then say that the
  unoccupied eigenvalues of X_0 lie in [0, l_0] and the occupied ones in
  [h_0, 1], with l_0 = (e_max - lumo) / W and h_0 = (e_max - homo) / W.
* Each step squares the larger of the two errors e_u = l and e_o = 1 - h,
  after shifting the vertex of the parabola to half of it, so that the two
  ends of that interval land on the same value (the interval is folded onto
  itself):
      e_u >= e_o:  p(x) = ((x - s) / (1 - s))^2,          s = e_u / 2
      e_u <  e_o:  p(x) = 1 - ((1 - s - x) / (1 - s))^2,  s = e_o / 2
  s = 0 gives back X^2 and 2X - X^2.  The images of the interval ends are the
  next bounds: e.g. for the first form l' = (s / (1 - s))^2 and
  h' = ((h - s) / (1 - s))^2.  The bounds evolve independently of X, so the
  whole sequence of polynomials is fixed by (l_0, h_0).
* Stop as in the plain expansion: when ||X_n^2 - X_n||_F <= tol and
  |Tr X_n - N_occ| <= tol, X_n is returned (its square is the product that
  measured the idempotency).
"""
from __future__ import annotations

import numpy as np

from .sp2 import gershgorin_bounds, initial_iterate


def start_bounds(e_min: float, e_max: float, homo: float, lumo: float):
    """(l_0, h_0): the unoccupied eigenvalues of X_0 lie in [0, l_0], the
    occupied ones in [h_0, 1]."""
    w = e_max - e_min
    return (e_max - lumo) / w, (e_max - homo) / w


def step_polynomial(l: float, h: float):
    """One accelerated step for the bounds (l, h).  Returns the polynomial as
    coefficients (a, b, c) of a x^2 + b x + c, the branch (1 = the X^2 form),
    the shift s, and the next bounds (l', h')."""
    e_u, e_o = l, 1.0 - h
    if e_u >= e_o:
        s = 0.5 * e_u
        k = 1.0 / (1.0 - s) ** 2
        # k (x - s)^2
        coef = (k, -2.0 * k * s, k * s * s)
        l_next = k * max(s, e_u - s) ** 2
        h_next = k * (h - s) ** 2
        return coef, 1, s, l_next, h_next
    s = 0.5 * e_o
    k = 1.0 / (1.0 - s) ** 2
    u = 1.0 - s
    # 1 - k (u - x)^2
    coef = (-k, 2.0 * k * u, 1.0 - k * u * u)
    l_next = 1.0 - k * (u - l) ** 2
    h_next = 1.0 - k * max(s, e_o - s) ** 2
    return coef, 0, s, l_next, h_next


def schedule(l0: float, h0: float, steps: int):
    """The first ``steps`` polynomials from (l_0, h_0) with the bounds they
    produce: a list of (coef, branch, s, l_after, h_after)."""
    out = []
    l, h = l0, h0
    for _ in range(steps):
        coef, br, s, l, h = step_polynomial(l, h)
        out.append((coef, br, s, l, h))
    return out


def azrfoe(h: np.ndarray, n_occ: float, homo: float, lumo: float, tol: float = 1e-10,
           max_iter: int = 100, bounds=None):
    """Float64 A-Z-RFOE.  ``homo`` must bound eps_HOMO from above and ``lumo``
    eps_LUMO from below, homo < lumo.  Returns (D, info) with the iteration
    count, branches (1 = X^2 form), shifts, idempotency history and bounds."""
    if not lumo > homo:
        raise ValueError("A-Z-RFOE needs homo < lumo")
    e_min, e_max = gershgorin_bounds(h) if bounds is None else bounds
    n = h.shape[0]
    x = initial_iterate(h, e_min, e_max)
    l, hb = start_bounds(e_min, e_max, homo, lumo)
    branches, shifts, idem, traces, intervals = [], [], [], [], [(l, hb)]
    converged = False
    n_done = 0
    eye = np.eye(n)
    for n_done in range(max_iter):
        t = float(np.trace(x))
        traces.append(t)
        p = x @ x
        e = float(np.linalg.norm(p - x))
        idem.append(e)
        if e <= tol and abs(t - n_occ) <= tol:
            converged = True
            break
        (a, b, c), br, s, l, hb = step_polynomial(l, hb)
        branches.append(br)
        shifts.append(s)
        intervals.append((l, hb))
        x = a * p + b * x + c * eye
    info = dict(iterations=n_done, converged=converged, branches=branches, shifts=shifts,
                idempotency=idem, traces=traces, intervals=intervals, bounds=(e_min, e_max))
    return x, info


def scalar_iterations(lam: np.ndarray, n_occ: int, tol: float, e_min: float, e_max: float,
                      homo=None, lumo=None, max_iter: int = 200, reltr_stop=None) -> int:
    """Iteration count of the expansion on a known spectrum (a diagonal H):
    with ``homo``/``lumo`` the accelerated polynomials, without them the plain
    trace-chosen X^2 / 2X - X^2.  Same stop rule as ``azrfoe``, or with
    ``reltr_stop`` the paper's relative-trace criterion (Sec. III.A): the
    count of products up to the first iterate whose trace changed by at most
    reltr_stop relative to the previous one."""
    x = (e_max - np.asarray(lam, dtype=np.float64)) / (e_max - e_min)
    acc = homo is not None
    if acc:
        l, hb = start_bounds(e_min, e_max, homo, lumo)
    for it in range(max_iter):
        p = x * x
        if (reltr_stop is None and float(np.sqrt(np.sum((p - x) ** 2))) <= tol
                and abs(float(x.sum()) - n_occ) <= tol):
            return it
        t = float(x.sum())
        if acc:
            (a, b, c), _, _, l, hb = step_polynomial(l, hb)
            x = a * p + b * x + c
        else:
            s = float(p.sum())
            x = p if abs(s - n_occ) <= abs(2.0 * t - s - n_occ) else 2.0 * x - p
        if reltr_stop is not None and abs(float(x.sum()) - t) / abs(t) <= reltr_stop:
            return it + 1
    return -1
