"""Writes the golden fixtures in this folder.  Calls only the oracle package
and the input generators; run from the repository root:

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import density as den  # noqa: E402
from workloads import paper_e1_band, paper_e1_matrix  # noqa: E402


def write(name, header, rows):
    with open(os.path.join(HERE, name), "w") as fh:
        for line in header:
            fh.write("# " + line + "\n")
        for k, v in rows:
            vals = " ".join(repr(float(x)) for x in np.atleast_1d(v))
            fh.write(f"{k} {vals}\n")


def main():
    n = 8
    h = paper_e1_matrix(n)
    # zero temperature, about 90% occupied (Sec. IV): N_occ = 7 of 8
    d, e, mu, lam = den.density_matrix(h, 7, 0.0)
    write("e1_n8_zero_t.txt",
          ["Paper's synthetic Hp (Sec. IV, Results): H_ij = exp(-0.5|i-j|) sin(min(i,j)+1), N = 8",
           "zero temperature, N_occ = 7 (about 90% occupied, Sec. IV)",
           "written by tests/golden/make_golden.py from the oracle (Jacobi eigenpairs)"],
          [("eigenvalues", lam), ("band_energy", e), ("d_diag", np.diag(d)), ("d_row0", d[0])])
    # finite temperature, 85% occupied, kT = 0.0016 Ha (500 K, Sec. IV)
    d, e, mu, lam = den.density_matrix(h, 0.85 * n, 0.0016)
    write("e1_n8_finite_t.txt",
          ["Paper's synthetic Hp (Sec. IV), N = 8, N_occ = 6.8 (85%), kT = 0.0016 Ha (about 500 K)",
           "written by tests/golden/make_golden.py from the oracle (Jacobi eigenpairs, bisection mu)"],
          [("mu", mu), ("band_energy", e), ("d_diag", np.diag(d)), ("d_row0", d[0])])


def large(n):
    """The paper's matrix at one of its sizes (Sec. IV): reference energies
    from the banded eigensolver on the band storage (entries beyond 80
    diagonals are below exp(-40))."""
    lam = den.band_storage_eigenvalues(paper_e1_band(n, 80))
    k = int(0.9 * n)
    e0, _, _ = den.reference_energy(lam, k, 0.0)
    e1, mu, _ = den.reference_energy(lam, 0.85 * n, 0.0016)
    write(f"e1_n{n}.txt",
          [f"Paper's synthetic Hp (Sec. IV), N = {n}: H_ij = exp(-0.5|i-j|) sin(min(i,j)+1)",
           f"zero temperature: N_occ = {k} (90%); finite temperature: N_occ = {0.85 * n} (85%), "
           "kT = 0.0016 Ha",
           "written by tests/golden/make_golden.py --large from the oracle (banded eigensolver)"],
          [("n", n), ("lambda_min_max", [lam[0], lam[-1]]), ("zero_t_n_occ", k),
           ("homo_lumo", [lam[k - 1], lam[k]]), ("zero_t_band_energy", e0),
           ("finite_t_mu", mu), ("finite_t_band_energy", e1)])


if __name__ == "__main__":
    if "--large" in sys.argv:
        sizes = [int(a) for a in sys.argv[2:]] or [16384, 32768]
        for n in sizes:
            large(n)
    else:
        main()
