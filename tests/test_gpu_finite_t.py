"""Finite temperature on the GPU against the oracle: one evaluation of the
doubling recursion against its closed form f_m (diagonal H) and against the
oracle recursion (dense H); full solves against the exact Fermi-Dirac density
matrix of the definition (Sec. II.A)."""
import numpy as np
import pytest

import workloads
from gpu_util import dev, host, reference, say

pytestmark = pytest.mark.gpu

KT = 0.0016


@pytest.fixture(scope="module")
def fdm():
    import paper_2301_04642_amd as m
    return m


def test_operator_closed_form_diagonal(fdm):
    import torch
    from oracle import fd
    lam = np.linspace(-1.0, 1.0, 97)
    mu = 0.0123
    H = dev(np.diag(lam))
    D = torch.empty_like(H)
    say("fermi operator diagonal")
    tr, trdd, m = fdm.fdm_fermi_operator(H, mu, KT, D, depth=0)
    ref = fd.closed_form(lam, mu, 1.0 / KT, m)
    d = host(D)
    assert np.abs(np.diag(d) - ref).max() < 1e-13
    assert np.abs(d - np.diag(np.diag(d))).max() < 1e-15
    assert abs(tr - ref.sum()) < 1e-12
    assert abs(trdd - (ref - ref ** 2).sum()) < 1e-12
    assert m == fd.depth(1.0 / KT, -1.0 - 0.0, 1.0, mu, extra=7)


@pytest.mark.parametrize("n", [64, 129, 300])
def test_operator_dense_matches_oracle_recursion(fdm, n):
    import torch
    from oracle import fd
    wl = workloads.standard_workload("uniform", n=n)
    mu = -0.41
    H = dev(wl.hp)
    D = torch.empty_like(H)
    say("fermi operator dense", n)
    tr, trdd, m = fdm.fdm_fermi_operator(H, mu, KT, D, depth=0)
    ref = fd.doubling(wl.hp, mu, 1.0 / KT, m)
    assert np.abs(host(D) - ref).max() < 1e-12
    # and the recursion is the Fermi operator to its truncation error
    from oracle import density as den
    f = den.fermi_dirac(wl.lam, mu, KT)
    d_exact = (wl.q * f) @ wl.q.T
    assert np.linalg.norm(host(D) - d_exact) < 1e-10


@pytest.mark.parametrize("prec", ["fp32", "fp16x3"])
def test_operator_low_precision(fdm, prec):
    import torch
    from oracle import fd
    wl = workloads.standard_workload("uniform", n=200)
    mu = -0.5
    H = dev(wl.hp)
    D = torch.empty_like(H)
    say("fermi operator", prec)
    tr, trdd, m = fdm.fdm_fermi_operator(H, mu, KT, D, depth=0, precision=prec)
    ref = fd.doubling(wl.hp, mu, 1.0 / KT, m)
    # near-mu errors double per step (u beta rho / 4 floor): ~1e-4 in FP32
    assert np.abs(host(D) - ref).max() < 5e-3
    assert abs(tr - np.trace(ref)) < 0.05


def check_solve(fdm, wl, prec):
    """FP64: D, E, Tr and [H, D] to 1e-10 of the exact Fermi-Dirac matrix
    (tol = 1e-10 is the trace target).  Mixed: |dE| <= 1e-6 Ha and
    |Tr D - n_occ| <= 1e-8 (gates; tol = 1e-8); ||D - D_ref|| reported."""
    d_ref, e_ref, mu_ref, f = reference(wl)
    say("finite-T solve", prec, wl.name)
    D, e, st = fdm.solve(dev(wl.hp), wl.n_occ, wl.kT, 1e-10 if prec == "fp64" else 1e-8, prec)
    d = host(D)
    dd = np.linalg.norm(d - d_ref)
    de = abs(e - e_ref)
    tr = abs(np.trace(d) - wl.n_occ)
    comm = np.linalg.norm(wl.hp @ d - d @ wl.hp)
    print(f"[report] finite-T {prec} n={wl.n} evals={st.mu_evals} depth={st.depth} "
          f"mu={st.mu:.10f} (exact {mu_ref:.10f}) |dE|={de:.2e} ||dD||={dd:.2e} |dTr|={tr:.2e} "
          f"||[H,D]||={comm:.2e}", flush=True)
    assert st.status == 0
    assert np.array_equal(d, d.T)
    if prec == "fp64":
        assert dd <= 1e-10
        assert de <= 1e-10
        assert tr <= 1e-10
        assert comm <= 1e-10
    else:
        assert de <= 1e-6
        assert tr <= 1e-8
    return st


@pytest.mark.parametrize("n", [100, 257, 600])
def test_solve_fp64(fdm, n):
    check_solve(fdm, workloads.standard_workload("uniform", n=n), "fp64")


@pytest.mark.parametrize("prec", ["fp32", "fp16x3", "bf16x3"])
def test_solve_mixed_final_fp64(fdm, prec):
    """Low-precision mu search, one FP64 evaluation and the trace correction."""
    st = check_solve(fdm, workloads.standard_workload("uniform", n=400), prec)
    assert st.products[fdm.PRECISIONS[prec]] > 0 and st.products[0] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp16x3"])
def test_mu_guess_from_a_previous_solve(fdm, prec):
    """Started from the mu of an earlier solve of the same matrix (an SCF
    step), the search ends after one evaluation with the same result; the
    mixed form then goes straight to its FP64 evaluation."""
    wl = workloads.standard_workload("uniform", n=600)
    H = dev(wl.hp)
    D0, e0, st0 = fdm.solve(H, wl.n_occ, wl.kT, 1e-9, "fp64")
    D1, e1, st1 = fdm.solve(H, wl.n_occ, wl.kT, 1e-9, prec, mu_guess=st0.mu)
    print(f"[report] mu guess ({prec}): evals {st0.mu_evals} -> {st1.mu_evals}, "
          f"|dE|={abs(e1 - e0):.1e}", flush=True)
    assert st1.status == 0 and st1.mu_evals <= 2 < st0.mu_evals
    if prec != "fp64":
        assert st1.products[fdm.PRECISIONS[prec]] == 0 and st1.products[0] > 0
    assert abs(e1 - e0) <= 1e-9 and abs(st1.mu - st0.mu) <= 1e-9
    assert float((D1 - D0).abs().max()) <= 1e-9
