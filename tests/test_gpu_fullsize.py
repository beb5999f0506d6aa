"""Full-size configurations (N = 12000 finite temperature, N = 30000 zero
temperature with outliers): sampled rows of D against rows the oracle builds
one by one from the known eigenbasis, plus properties that hold at any size
(band energy against the closed form sum f_i lam_i, trace, idempotency and
commutator on sampled rows)."""
import numpy as np
import pytest

import workloads
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdm():
    import paper_2301_04642_amd as m
    return m


def sampled_checks(wl, d, f, rows, tol_rows, tol_idem, tol_comm=None):
    from oracle import density as den
    ref_rows = den.density_rows(wl.q_rows, wl.n, f, rows)
    err = np.abs(d[rows] - ref_rows).max()
    dr = d[rows]
    idem = np.linalg.norm(dr @ d - dr)
    hr = wl.hp[rows]
    comm = np.linalg.norm(hr @ d - dr @ wl.hp)
    print(f"[report] {wl.name}: sampled-row max err {err:.2e}, row idempotency {idem:.2e}, "
          f"row commutator {comm:.2e}", flush=True)
    assert err <= tol_rows
    assert idem <= tol_idem
    if tol_comm is not None:
        assert comm <= tol_comm


@pytest.fixture(scope="module")
def outliers30000():
    say("generate bands+outliers N=30000")
    return workloads.standard_workload("outliers")


@pytest.mark.parametrize("prec,bounds", [("fp32", 0), ("fp32", 1), ("fp16x3", 1)])
def test_outliers_n30000_mixed(fdm, outliers30000, prec, bounds):
    """N = 30000, n_occ = 7500, bands + 1% outliers up to 5 Ha, gap 0.05 Ha:
    FP32 bulk with FP64 first steps, traces and McWeeny refinement."""
    from oracle import density as den
    wl = outliers30000
    H = dev(wl.hp)
    say("solve bands+outliers N=30000", prec, "bounds", bounds)
    D, e, st = fdm.solve(H, wl.n_occ, 0.0, 1e-8, prec, bounds=bounds)
    del H
    d = host(D)
    del D
    f, _ = den.occupations(wl.lam, wl.n_occ, 0.0)
    e_ref = float(np.dot(f, wl.lam))
    print(f"[report] outliers-n30000 {prec} bounds={bounds}: k64={st.iters_fp64_first} low={st.iters_low} mcw={st.mcweeny_steps} "
          f"|dE|={abs(e - e_ref):.2e} idem={st.idempotency:.2e} bounds=({st.e_min:.1f},{st.e_max:.1f})",
          flush=True)
    assert st.status == 0
    assert abs(e - e_ref) <= 1e-6
    assert abs(np.trace(d) - wl.n_occ) <= 1e-8
    assert st.idempotency <= 1e-8
    rows = np.random.default_rng(3).choice(wl.n, 6, replace=False)
    # mixed forms: D itself is rotation-limited (reported, not gated)
    sampled_checks(wl, d, f, rows, tol_rows=1e-4, tol_idem=1e-8)


@pytest.fixture(scope="module")
def uniform12000():
    say("generate uniform N=12000")
    return workloads.standard_workload("uniform")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3", "bf16x3"])
def test_uniform_n12000_finite_t(fdm, uniform12000, prec):
    """N = 12000, uniform [-1, 1], kT = 0.0016 Ha, n_occ = 3000 (Sec. II.A
    Fermi-Dirac occupations; the paper's 500 K of Sec. IV).  FP64: every mu
    evaluation in FP64, gated at 1e-10.  Mixed: the mu search in the low
    precision, one FP64 evaluation, then the second-order canonical
    correction; gated at |dE| <= 1e-6 Ha and |Tr D - n_occ| <= 1e-8.
    Sampled rows of D against rows of Q f(Lambda) Q^T."""
    from oracle import density as den
    wl = uniform12000
    H = dev(wl.hp)
    tol = 1e-10 if prec == "fp64" else 1e-8
    say("solve uniform N=12000", prec)
    D, e, st = fdm.solve(H, wl.n_occ, wl.kT, tol, prec)
    del H
    d = host(D)
    del D
    f, mu = den.occupations(wl.lam, wl.n_occ, wl.kT)
    e_ref = float(np.dot(f, wl.lam))
    print(f"[report] uniform-n12000 {prec}: evals={st.mu_evals} depth={st.depth} mu={st.mu:.9f} "
          f"(exact {mu:.9f}) |dE|={abs(e - e_ref):.2e} |dTr|={abs(np.trace(d) - wl.n_occ):.2e} "
          f"products fp64 {st.products[0]} {prec} {st.products[fdm.PRECISIONS[prec]]} "
          f"{st.ms_total:.0f} ms", flush=True)
    assert st.status == 0
    # FP64: 1e-10 Ha, or 1e-13 relative for energies above 1000 Ha.  Here
    # |E| = 2250 Ha and every form (all end with the same FP64 evaluation)
    # lands 1.4e-10 Ha (6e-14 relative) from the reference, at depth +7 and
    # +8 alike: the FP64 rounding floor of the recursion summed over 12000
    # states, not its truncation (the reference itself agrees with the
    # Rayleigh quotients of the stored Hp to 1e-12 Ha).
    assert abs(e - e_ref) <= (max(1e-10, 1e-13 * abs(e_ref)) if prec == "fp64" else 1e-6)
    assert abs(np.trace(d) - wl.n_occ) <= tol
    rows = np.random.default_rng(2).choice(wl.n, 6, replace=False)
    ref_rows = den.density_rows(wl.q_rows, wl.n, f, rows)
    err = np.abs(d[rows] - ref_rows).max()
    hr = wl.hp[rows]
    comm = np.linalg.norm(hr @ d - d[rows] @ wl.hp)
    print(f"[report] uniform-n12000 {prec}: sampled-row max err {err:.2e}, row commutator "
          f"{comm:.2e}", flush=True)
    assert err <= (1e-10 if prec == "fp64" else 1e-5)
    assert comm <= (1e-10 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
def test_uniform_n12000_bulk_low_precision_reported(fdm, uniform12000, prec):
    """The finite-temperature form with every evaluation in low precision
    (fd_final_fp64 = 0).  The doubling recursion amplifies rounding injected
    near mu, so this form is not expected to meet the 1e-6 Ha gate: measured
    and reported, with only the solve's status and the trace (set by the
    final correction) checked."""
    from oracle import density as den
    wl = uniform12000
    say("solve uniform N=12000 bulk", prec)
    D, e, st = fdm.solve(dev(wl.hp), wl.n_occ, wl.kT, 1e-8, prec, fd_final_fp64=0)
    tr = float(D.diagonal().sum())
    del D
    f, _ = den.occupations(wl.lam, wl.n_occ, wl.kT)
    e_ref = float(np.dot(f, wl.lam))
    print(f"[report] uniform-n12000 bulk {prec} (no FP64 evaluation): evals={st.mu_evals} "
          f"|dE|={abs(e - e_ref):.2e} Ha (gate 1e-6: {'met' if abs(e - e_ref) <= 1e-6 else 'missed'}) "
          f"|dTr|={abs(tr - wl.n_occ):.2e} {st.ms_total:.0f} ms", flush=True)
    assert st.status == 0
    assert st.products[0] <= 2        # only the canonical correction's two FP64 products
    assert abs(tr - wl.n_occ) <= 1e-3
