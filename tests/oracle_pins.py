"""Pins of the CPU oracle against closed forms, invariants and a library
routine.  Each check raises AssertionError on failure; the tests call them on
the real oracle and, with planted mistakes, on mutated copies."""
from __future__ import annotations

import math

import numpy as np

from oracle import density as den
from oracle import azrfoe as az
from oracle import fd, sp2, trfoe
from oracle.eig import jacobi_eigh
import workloads


def check_jacobi_2x2(eigh=jacobi_eigh):
    rng = np.random.default_rng(11)
    for _ in range(20):
        a, b, c = rng.uniform(-2, 2, 3)
        h = np.array([[a, b], [b, c]])
        w, v = eigh(h)
        r = math.sqrt(((a - c) / 2) ** 2 + b * b)
        exact = np.array([(a + c) / 2 - r, (a + c) / 2 + r])
        assert np.allclose(w, exact, atol=1e-14, rtol=0), (w, exact)
        assert np.allclose(v @ np.diag(w) @ v.T, h, atol=1e-14)


def check_jacobi_toeplitz(eigh=jacobi_eigh, n=30, a=0.3, b=-0.7):
    """Tridiagonal Toeplitz: eigenvalues a + 2b cos(k pi/(n+1)), eigenvectors
    sin(j k pi/(n+1)) (closed form)."""
    h = a * np.eye(n) + b * (np.eye(n, k=1) + np.eye(n, k=-1))
    w, v = eigh(h)
    k = np.arange(1, n + 1)
    exact = np.sort(a + 2 * b * np.cos(k * np.pi / (n + 1)))
    assert np.allclose(w, exact, atol=1e-13, rtol=0), np.abs(w - exact).max()
    j = np.arange(1, n + 1)
    # eigenvector of the lowest eigenvalue (b < 0 -> k = 1)
    u = np.sin(j * 1 * np.pi / (n + 1))
    u /= np.linalg.norm(u)
    assert abs(abs(np.dot(u, v[:, 0])) - 1) < 1e-12


def check_jacobi_known_spectrum(eigh=jacobi_eigh, n=48):
    rng = np.random.default_rng(5)
    lam = np.sort(rng.uniform(-2, 2, n))
    wl = workloads.make_workload("pin", lam, n // 4, 0.0, 1e-10, 17)
    w, v = eigh(wl.hp)
    assert np.allclose(w, lam, atol=1e-13, rtol=0), np.abs(w - lam).max()
    assert np.allclose(v.T @ v, np.eye(n), atol=1e-13)
    assert np.allclose((v * w) @ v.T, wl.hp, atol=1e-13)


def check_jacobi_vs_lapack(eigh=jacobi_eigh, n=64):
    rng = np.random.default_rng(9)
    g = rng.standard_normal((n, n))
    h = 0.5 * (g + g.T)
    w, v = eigh(h)
    wl, vl = np.linalg.eigh(h)
    assert np.allclose(w, wl, atol=1e-12, rtol=0)
    # compare spectral projectors of the lowest 20 (robust to eigenvector sign)
    p = v[:, :20] @ v[:, :20].T
    pl = vl[:, :20] @ vl[:, :20].T
    assert np.abs(p - pl).max() < 1e-11


def check_density_invariants(density_matrix=den.density_matrix, n=64):
    wl = workloads.standard_workload("gapped", n=n)
    d, e, mu, lam = density_matrix(wl.hp, wl.n_occ, 0.0)
    assert np.linalg.norm(d @ d - d) < 1e-11
    assert abs(np.trace(d) - wl.n_occ) < 1e-11
    assert np.linalg.norm(wl.hp @ d - d @ wl.hp) < 1e-11
    lowest = np.sort(wl.lam)[: int(wl.n_occ)].sum()
    assert abs(e - lowest) < 1e-11
    assert abs(den.band_energy(wl.hp, d) - lowest) < 1e-11


def check_density_vs_construction(density_matrix=den.density_matrix, n=80, kT=0.0):
    wl = workloads.standard_workload("gapped" if kT == 0.0 else "uniform", n=n)
    d, e, mu, lam = density_matrix(wl.hp, wl.n_occ, kT)
    f, mu2 = den.occupations(wl.lam, wl.n_occ, kT)
    d_ref = (wl.q * f) @ wl.q.T
    assert np.abs(d - d_ref).max() < 1e-12, np.abs(d - d_ref).max()
    assert abs(e - float(np.dot(f, wl.lam))) < 1e-11
    assert abs(mu - mu2) < 1e-9


def check_shift_scale_and_permutation(density_matrix=den.density_matrix, n=40):
    wl = workloads.standard_workload("gapped", n=n)
    d, *_ = density_matrix(wl.hp, wl.n_occ, 0.0)
    d2, *_ = density_matrix(2.5 * wl.hp - 0.7 * np.eye(n), wl.n_occ, 0.0)
    assert np.abs(d - d2).max() < 1e-12
    perm = np.random.default_rng(3).permutation(n)
    d3, *_ = density_matrix(wl.hp[np.ix_(perm, perm)], wl.n_occ, 0.0)
    assert np.abs(d3 - d[np.ix_(perm, perm)]).max() < 1e-12


def check_fd_two_level(fermi=den.fermi_dirac, chem=den.chemical_potential):
    """Two levels at -a and +a with one electron: mu = 0 by symmetry and the
    occupancies are 1/(1 + exp(-+a/kT)) (the Fermi function of Sec. II.A)."""
    a, kT = 0.003, 0.0016
    lam = np.array([-a, a])
    mu = chem(lam, 1.0, kT)
    assert abs(mu) < 1e-12
    f = fermi(lam, mu, kT)
    exact = 1.0 / (np.exp(lam / kT) + 1.0)
    assert np.allclose(f, exact, atol=1e-15, rtol=0)
    # a rotated 2x2: D = f(H) by the 2x2 closed form
    th = 0.37
    q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    h = (q * lam) @ q.T
    d, e, mu3, _ = den.density_matrix(h, 1.0, kT)
    d_exact = (q * exact) @ q.T
    assert np.abs(d - d_exact).max() < 1e-14
    assert abs(e - np.dot(exact, lam)) < 1e-15


def check_fd_symmetric_mu(chem=den.chemical_potential):
    lam = np.linspace(-1, 1, 101)
    assert abs(chem(lam, 50.5, 0.0016)) < 1e-12
    lam = np.concatenate([-np.linspace(0.1, 1, 50), np.linspace(0.1, 1, 50)])
    assert abs(chem(lam, 50.0, 0.01)) < 1e-12


def check_fd_low_t_limit(n=64):
    wl = workloads.standard_workload("gapped", n=n)
    d0, e0, *_ = den.density_matrix(wl.hp, wl.n_occ, 0.0)
    d1, e1, *_ = den.density_matrix(wl.hp, wl.n_occ, 1e-4)   # gap 0.2 Ha >> kT
    assert np.abs(d0 - d1).max() < 1e-12
    assert abs(e0 - e1) < 1e-11


def check_gershgorin(bounds=sp2.gershgorin_bounds):
    d = np.diag([0.5, -1.25, 3.0, 0.0])
    assert bounds(d) == (-1.25, 3.0)
    a, b, c = 0.4, -0.3, 1.1
    assert np.allclose(bounds(np.array([[a, b], [b, c]])), (a - abs(b), c + abs(b)))
    h = np.array([[1.0, 0.5, -0.25], [0.5, -2.0, 1.0], [-0.25, 1.0, 0.0]])
    assert np.allclose(bounds(h), (-3.5, 1.75))
    wl = workloads.standard_workload("bands", n=200)
    lo, hi = bounds(wl.hp)
    assert lo <= wl.lam.min() and hi >= wl.lam.max()


def check_sp2_diagonal(sp2fn=sp2.sp2):
    """On a diagonal H every eigenvalue follows the scalar maps x -> x^2 or
    2x - x^2 under the same branch sequence, from (e_max - h)/(e_max - e_min)."""
    rng = np.random.default_rng(21)
    n, n_occ = 24, 9
    lam = np.concatenate([rng.uniform(-1, -0.3, n_occ), rng.uniform(0.1, 1, n - n_occ)])
    h = np.diag(lam)
    x, info = sp2fn(h, n_occ, tol=1e-12)
    lo, hi = lam.min(), lam.max()           # Gershgorin is exact on a diagonal matrix
    s = (hi - lam) / (hi - lo)
    for br in info["branches"]:
        s = s * s if br else 2 * s - s * s
    assert np.allclose(np.diag(x), s, atol=1e-15, rtol=0)
    assert np.abs(x - np.diag(np.diag(x))).max() == 0.0
    assert np.allclose(np.diag(x), (lam < 0).astype(float), atol=1e-6)


def check_sp2_matches_definition(sp2fn=sp2.sp2, sizes=(4, 16, 64, 256)):
    for n in sizes:
        wl = workloads.standard_workload("gapped", n=n)
        x, info = sp2fn(wl.hp, wl.n_occ, tol=1e-11)
        f, _ = den.occupations(wl.lam, wl.n_occ, 0.0)
        d_ref, e_ref = den.density_from_eig(wl.q, wl.lam, f)
        assert info["converged"], n
        assert np.linalg.norm(x - d_ref) < 1e-10, (n, np.linalg.norm(x - d_ref))
        assert abs(den.band_energy(wl.hp, x) - e_ref) < 1e-10
        assert abs(np.trace(x) - wl.n_occ) < 1e-10


def check_mcweeny(mcw=sp2.mcweeny):
    x = np.diag([0.02, 0.97, 0.999, 0.0, 1.0, 0.05])
    y, steps, hist = mcw(x.copy(), 1e-12)
    s = np.diag(x).copy()
    for _ in range(steps):
        s = 3 * s ** 2 - 2 * s ** 3
    assert np.allclose(np.diag(y), s, atol=1e-15)
    assert np.allclose(np.diag(y), [0, 1, 1, 0, 1, 0], atol=1e-12)


def check_fd_recursion_closed_form(doubling=fd.doubling):
    lam = np.linspace(-1, 1, 33)
    mu, beta = 0.013, 625.0
    m = fd.depth(beta, -1.0, 1.0, mu)
    d = doubling(np.diag(lam), mu, beta, m)
    assert np.allclose(np.diag(d), fd.closed_form(lam, mu, beta, m), atol=1e-13, rtol=0)
    # the closed form tends to the Fermi function: the atanh series gives an
    # argument error s^3 / (3 * 2^(2m+3)), so |f_m - f| shrinks 4x per step
    f = den.fermi_dirac(lam, mu, 1.0 / beta)
    err = [np.abs(fd.closed_form(lam, mu, beta, mm) - f).max() for mm in (m - 2, m - 1, m)]
    assert err[2] < 2.0 ** -(2 * m + 1), err
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5, err


def check_fd_recursion_dense(doubling=fd.doubling, n=64):
    wl = workloads.standard_workload("uniform", n=n)
    kT = 0.0016
    f, mu = den.occupations(wl.lam, wl.n_occ, kT)
    d_ref, _ = den.density_from_eig(wl.q, wl.lam, f)
    m = fd.depth(1.0 / kT, wl.lam.min(), wl.lam.max(), mu)
    d = doubling(wl.hp, mu, 1.0 / kT, m)
    assert np.linalg.norm(d - d_ref) < 1e-11, np.linalg.norm(d - d_ref)


def check_banded_eigenvalues(banded=den.banded_eigenvalues):
    """The banded solver on the paper's matrix agrees with Jacobi (and so
    with the dense definition) once the band holds every non-negligible
    diagonal; the reference energy is the sum of the lowest eigenvalues."""
    h = workloads.paper_e1_matrix(96)
    w = banded(h, 80)
    wj, _ = jacobi_eigh(h)
    assert np.abs(w - wj).max() < 1e-13
    e, mu, f = den.reference_energy(w, 86, 0.0)
    assert abs(e - np.sort(wj)[:86].sum()) < 1e-12
    # truncating the band visibly changes the spectrum (the pin is sensitive)
    assert np.abs(banded(h, 3) - wj).max() > 1e-3


def check_azrfoe_fold(step=az.step_polynomial):
    """Each accelerated polynomial keeps the converged end fixed (1 -> 1 for
    the squaring form, 0 -> 0 for the other), folds the squared interval so
    its two ends meet, maps both assumed intervals into [0, 1], and reports
    the images of the interval ends as the next bounds."""
    rng = np.random.default_rng(31)
    for _ in range(200):
        l, h = np.sort(rng.uniform(0.0, 1.0, 2))
        (a, b, c), br, s, l2, h2 = step(l, h)
        p = lambda x: a * x * x + b * x + c  # noqa: E731
        if br == 1:
            assert abs(p(1.0) - 1.0) < 1e-12 and abs(p(0.0) - p(l)) < 1e-12
        else:
            assert abs(p(0.0)) < 1e-12 and abs(p(1.0) - p(h)) < 1e-12
        xs_u = np.linspace(0.0, l, 101)
        xs_o = np.linspace(h, 1.0, 101)
        assert abs(p(xs_u).max() - l2) < 1e-12 and p(xs_u).min() >= -1e-12
        assert abs(p(xs_o).min() - h2) < 1e-12 and p(xs_o).max() <= 1.0 + 1e-12
        # the squared error shrinks at least 4x faster than under X^2 / 2X - X^2
        if br == 1:
            assert l2 <= l * l / 4.0 * (1.0 + 1e-12) / (1.0 - l / 2.0) ** 2
        else:
            assert 1.0 - h2 <= (1.0 - h) ** 2 / 4.0 * (1.0 + 1e-12) / (1.0 - (1.0 - h) / 2.0) ** 2


def check_azrfoe_diagonal(azfn=az.azrfoe):
    """On a diagonal H with exact bounds, every eigenvalue follows the scalar
    polynomial sequence, and the recorded bounds are attained: the largest
    unoccupied image equals l_n and the smallest occupied image equals h_n."""
    rng = np.random.default_rng(23)
    n, n_occ = 30, 11
    lam = np.sort(np.concatenate([rng.uniform(-1, -0.25, n_occ), rng.uniform(0.05, 1, n - n_occ)]))
    x, info = azfn(np.diag(lam), n_occ, lam[n_occ - 1], lam[n_occ], tol=1e-12)
    assert info["converged"]
    lo, hi = lam.min(), lam.max()
    v = (hi - lam) / (hi - lo)
    occ = np.arange(n) < n_occ
    for k, (br, s) in enumerate(zip(info["branches"], info["shifts"])):
        l_k, h_k = info["intervals"][k]
        assert abs(v[~occ].max() - l_k) < 1e-12 and abs(v[occ].min() - h_k) < 1e-12, k
        v = ((v - s) / (1 - s)) ** 2 if br else 1 - ((1 - s - v) / (1 - s)) ** 2
    assert np.allclose(np.diag(x), v, atol=1e-14, rtol=0)
    assert np.abs(x - np.diag(np.diag(x))).max() == 0.0
    assert np.allclose(np.diag(x), occ.astype(float), atol=1e-6)


def check_azrfoe_matches_definition(azfn=az.azrfoe, sizes=(16, 64, 256), shrink=(0.0, 0.4)):
    """Dense H: the accelerated expansion reaches the definition theta(mu - H)
    with exact HOMO/LUMO bounds and with bounds that understate the gap."""
    for n in sizes:
        wl = workloads.standard_workload("gapped", n=n)
        k = int(wl.n_occ)
        lam = np.sort(wl.lam)
        gap = lam[k] - lam[k - 1]
        f, _ = den.occupations(wl.lam, wl.n_occ, 0.0)
        d_ref, e_ref = den.density_from_eig(wl.q, wl.lam, f)
        for c in shrink:
            x, info = azfn(wl.hp, wl.n_occ, lam[k - 1] + c * gap / 2, lam[k] - c * gap / 2,
                           tol=1e-11)
            assert info["converged"], (n, c)
            assert np.linalg.norm(x - d_ref) < 1e-10, (n, c, np.linalg.norm(x - d_ref))
            assert abs(den.band_energy(wl.hp, x) - e_ref) < 1e-10


def check_azrfoe_paper_counts(count=az.scalar_iterations):
    """Sec. IV: on the paper's matrix the plain expansion takes about 50
    products and the accelerated one about 30.  On the exact spectrum of the
    N = 8192 matrix (banded solver), with the extreme eigenvalues as spectral
    bounds, 90% occupation and the HOMO/LUMO eigenvalues as the accelerated
    form's bounds, the two counts land there."""
    n = 8192
    lam = den.banded_eigenvalues(workloads.paper_e1_matrix(n), 80)
    lo, hi = lam[0], lam[-1]
    k = int(0.9 * n)
    plain = count(lam, k, 1e-8, lo, hi)
    acc = count(lam, k, 1e-8, lo, hi, lam[k - 1], lam[k])
    assert 45 <= plain <= 55, plain
    assert 24 <= acc <= 34, acc


def check_sp2_stop_rule(sp2fn=sp2.sp2):
    """The stop rule asks for both ||X^2 - X||_F <= tol and |Tr X - N_occ| <=
    tol.  On a diagonal H with two clusters (+-0.1, n/4 occupied) and bounds
    (-1, 1) every eigenvalue follows the scalar maps, so the first iterate
    meeting both conditions is known; there the idempotency alone is met one
    step earlier while the trace is still 1.8e-8 off."""
    n, k, tol = 256, 64, 1e-8
    lam = np.concatenate([np.full(k, -0.1), np.full(n - k, 0.1)])
    x, info = sp2fn(np.diag(lam), k, tol=tol, bounds=(-1.0, 1.0))
    s = (1.0 - lam) / 2.0
    first = None
    for it in range(100):
        t, q = s.sum(), (s * s).sum()
        p = s * s
        if np.sqrt(((p - s) ** 2).sum()) <= tol and abs(t - k) <= tol:
            first = it
            break
        s = p if abs(q - k) <= abs(2 * t - q - k) else 2 * s - p
    assert info["converged"] and info["iterations"] == first, (info["iterations"], first)
    assert abs(np.trace(x) - k) <= tol and np.linalg.norm(x @ x - x) <= tol
    assert np.allclose(np.diag(x), s, atol=1e-15, rtol=0)


def check_density_rows(rows_fn=den.density_rows, n=64):
    """Rows of D = Q diag(f) Q^T built from row blocks of the eigenbasis equal
    the rows of the Jacobi density matrix (an independent eigendecomposition),
    at zero and finite temperature, with a block size that leaves a ragged
    tail."""
    for kind, kT in (("gapped", 0.0), ("uniform", 0.0016)):
        wl = workloads.standard_workload(kind, n=n)
        f, _ = den.occupations(wl.lam, wl.n_occ, kT)
        d_jac, *_ = den.density_matrix(wl.hp, wl.n_occ, kT)
        rows = np.array([0, 5, 17, n - 1])
        got = rows_fn(wl.q_rows, n, f, rows, chunk=24)
        assert got.shape == (rows.size, n)
        assert np.abs(got - d_jac[rows]).max() < 1e-12, np.abs(got - d_jac[rows]).max()


def check_kron_workload(make=workloads.make_workload):
    """The Kronecker-Haar construction used above 8192 rows: Q orthogonal,
    each column of Q an eigenvector of Hp with its eigenvalue, rows of Q by
    q_rows equal to rows of the full matrix, and Jacobi recovers the
    spectrum (n = 12 = 3 x 4 and n = 30 = 5 x 6)."""
    for n in (12, 30):
        rng = np.random.default_rng(n)
        lam = rng.uniform(-1.0, 1.0, n)
        wl = make("kron-pin", lam, n // 4, 0.0, 1e-10, 100 + n, kron=True)
        assert wl.q is None and wl.q_factors is not None
        q = wl.q_full()
        assert np.abs(q.T @ q - np.eye(n)).max() < 1e-13
        assert np.abs(wl.hp @ q - q * wl.lam[None, :]).max() < 1e-13
        rows = np.array([0, 3, n - 1])
        assert np.array_equal(wl.q_rows(rows), q[rows])
        w, _ = jacobi_eigh(wl.hp)
        assert np.abs(w - np.sort(lam)).max() < 1e-13


def check_paper_e1_band(band=workloads.paper_e1_band):
    """Band storage of the paper's matrix holds its diagonals (n = 200), and
    the banded eigensolver on it gives the Jacobi spectrum of the dense
    matrix (n = 96)."""
    n, bw = 200, 80
    h = workloads.paper_e1_matrix(n)
    ab = band(n, bw)
    assert ab.shape == (bw + 1, n)
    for d in range(bw + 1):
        assert np.array_equal(ab[bw - d, d:], np.diag(h, d)), d
        assert np.all(ab[bw - d, :d] == 0.0)
    w = den.band_storage_eigenvalues(band(96, bw))
    wj, _ = jacobi_eigh(workloads.paper_e1_matrix(96))
    assert np.abs(w - wj).max() < 1e-13


def check_eps_metrics(e1=den.eps1, e2=den.eps2):
    """Sec. III.C: eps1 = ||D - D_ref||_F / ||D_ref||_F, eps2 signed
    (Tr(D H) - Tr(D_ref H)) / Tr(D_ref H).  Hand-computed cases."""
    d_ref = np.diag([1.0, 1.0, 0.0])
    d = np.diag([1.0, 0.9, 0.1])
    assert abs(e1(d, d_ref) - 0.1) < 1e-15              # sqrt(0.02) / sqrt(2)
    assert abs(e2(-9.9, -10.0) - (-0.01)) < 1e-15       # (-9.9 + 10) / -10
    assert abs(e2(2.2, 2.0) - 0.1) < 1e-15


def check_lapack_eigh(eigh=den.eigh_lapack, n=64):
    """The library eigensolver used for references at large N agrees with
    the plain Jacobi sweep and with a known spectrum."""
    rng = np.random.default_rng(13)
    g = rng.standard_normal((n, n))
    h = 0.5 * (g + g.T)
    w, v = eigh(h)
    wj, vj = jacobi_eigh(h)
    assert np.abs(w - wj).max() < 1e-12
    assert np.abs(v[:, :20] @ v[:, :20].T - vj[:, :20] @ vj[:, :20].T).max() < 1e-11
    wl = workloads.standard_workload("bands", n=n)
    w, v = eigh(wl.hp)
    assert np.abs(w - np.sort(wl.lam)).max() < 1e-13
    assert np.abs((v * w) @ v.T - wl.hp).max() < 1e-13


def check_sp2_reltr_stop(sp2fn=sp2.sp2):
    """The relative-trace stop (Sec. III.A): on a diagonal H the dense
    iteration follows the scalar maps, and the returned iterate is the first
    whose trace changed by at most the threshold; both SP2 branches change
    the trace by Tr(X - X^2), so RelTr of X_{n+1} is (t - s)/t at X_n."""
    rng = np.random.default_rng(31)
    rng.uniform(size=40)
    n, k = 120, 90
    lam = np.sort(np.concatenate([rng.uniform(-1, -0.2, k), rng.uniform(0.1, 1, n - k)]))
    for thr in (5e-3, 5e-4, 5e-8):
        x, info = sp2fn(np.diag(lam), k, reltr_stop=thr, bounds=(lam[0], lam[-1]))
        s = (lam[-1] - lam) / (lam[-1] - lam[0])
        for it in range(1, 200):
            t, q = s.sum(), (s * s).sum()
            s = s * s if abs(q - k) <= abs(2 * t - q - k) else 2 * s - s * s
            if (t - q) / t <= thr:
                break
        assert info["iterations"] == it, (info["iterations"], it)
        assert np.allclose(np.diag(x), s, atol=1e-15, rtol=0)


def check_reltr_paper_count(count=az.scalar_iterations):
    """Sec. IV: stopped at RelTr 5e-8, the plain expansion takes about 50
    products on the paper's matrix (here its exact N = 8192 spectrum, 90%
    occupied, bounds at the extreme eigenvalues)."""
    n = 8192
    lam = den.banded_eigenvalues(workloads.paper_e1_matrix(n), 80)
    c = count(lam, int(0.9 * n), 1e-8, lam[0], lam[-1], reltr_stop=5e-8)
    assert 45 <= c <= 55, c


def check_trfoe_dense_vs_spectral(dense=trfoe.dense, scal=trfoe.scalar, n=64):
    """The truncated expansion is a matrix function: the dense iteration on
    Hp = Q diag(lam) Q^T equals Q diag(G_m(lam)) Q^T, with the same
    trace-chosen branches, at 85% and 25% filling."""
    wl = workloads.standard_workload("uniform", n=n)
    bounds = sp2.gershgorin_bounds(wl.hp)
    for frac in (0.85, 0.25):
        nocc = frac * n
        x, info = dense(wl.hp, nocc, 0.0016, bounds=bounds)
        g, sinfo = scal(wl.lam, nocc, 0.0016, *bounds)
        assert info["branches"] == sinfo["branches"]
        assert np.abs(x - (wl.q * g) @ wl.q.T).max() < 1e-12


def check_trfoe_properties(scal=trfoe.scalar):
    """Occupations lie in [0, 1] and fall with the energy (both maps are
    increasing on [0, 1]); with a gap and many steps the truncated expansion
    becomes the zero-temperature projector (Z-RFOE); the depth grows as the
    temperature falls."""
    lam = np.linspace(-1, 1, 301)
    g, info = scal(lam, 120.3, 0.0016, -1.0, 1.0)
    assert g.min() >= 0.0 and g.max() <= 1.0
    assert np.all(np.diff(g) <= 1e-15)
    lam2 = np.concatenate([np.linspace(-1, -0.3, 40), np.linspace(0.2, 1, 60)])
    g2, _ = scal(lam2, 40, 0.0016, -1.0, 1.0, m=60)
    assert np.abs(g2 - (lam2 < 0)).max() < 1e-12
    assert trfoe.depth(0.0016, -1, 1) > trfoe.depth(0.01, -1, 1) > trfoe.depth(0.05, -1, 1)


def check_trfoe_slope(scal=trfoe.scalar):
    """The depth rule's intent: the smeared step's slope at its half-way
    point is within a factor 2 of the Fermi function's beta/4 (measured on a
    fine uniform spectrum at 30%, 50% and 85% filling, kT = 0.0016 and
    0.01 Ha)."""
    lam = np.linspace(-1, 1, 4001)
    for frac in (0.3, 0.5, 0.85):
        for kT in (0.0016, 0.01):
            g, _ = scal(lam, frac * lam.size, kT, -1.0, 1.0)
            i = int(np.argmin(np.abs(g - 0.5)))
            slope = -(g[i + 1] - g[i - 1]) / (lam[i + 1] - lam[i - 1])
            ratio = slope / (0.25 / kT)
            assert 0.5 <= ratio <= 2.0, (frac, kT, ratio)


ALL_PINS = [
    check_jacobi_2x2, check_jacobi_toeplitz, check_jacobi_known_spectrum, check_jacobi_vs_lapack,
    check_density_invariants, check_density_vs_construction, check_shift_scale_and_permutation,
    check_fd_two_level, check_fd_symmetric_mu, check_fd_low_t_limit, check_gershgorin,
    check_sp2_diagonal, check_sp2_matches_definition, check_mcweeny,
    check_fd_recursion_closed_form, check_fd_recursion_dense, check_banded_eigenvalues,
    check_azrfoe_fold, check_azrfoe_diagonal, check_azrfoe_matches_definition,
    check_azrfoe_paper_counts, check_sp2_stop_rule, check_density_rows, check_kron_workload,
    check_paper_e1_band, check_eps_metrics, check_lapack_eigh, check_sp2_reltr_stop,
    check_reltr_paper_count, check_trfoe_dense_vs_spectral, check_trfoe_properties,
    check_trfoe_slope,
]
