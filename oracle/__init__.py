"""CPU oracle for the density-matrix solver -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct float64 implementations of what the GPU path
computes, written from the paper (arXiv 2301.04642):

* ``density``: the definitions of Sec. II.A -- the zero-temperature density
  matrix theta(mu I - H) and the Fermi-Dirac matrix [exp(beta(H - mu I)) + I]^-1
  -- built from an eigendecomposition (plain C Jacobi in ``jacobi.c``, or a
  known eigenbasis), plus the accuracy metrics of Sec. III.C.
* ``sp2``: the zero-temperature recursive expansion of Sec. II.B.1, Eq. (1),
  in the paper's order, with Gershgorin spectral bounds (Sec. II.C) and
  McWeeny refinement.
* ``fd``: the finite-temperature doubling recursion and its closed form.
* ``azrfoe``: the accelerated zero-temperature expansion of Sec. II.B.2
  (shifted and scaled SP2 polynomials chosen from HOMO/LUMO bounds).
* ``trfoe``: the truncated zero-temperature expansion used as a smeared step
  at finite temperature (Sec. II.B.3, Eq. (2)).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never calls it.
"""
from . import azrfoe, density, fd, sp2, trfoe  # noqa: F401
