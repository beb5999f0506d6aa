"""The finite-temperature mu search hands its mu on to the FP64 evaluation
after a last Newton step of |beta dmu| <= 0.03 that it does not evaluate.
That is sound because a Newton step on the Fermi-Dirac trace
T(mu) = sum_i f_i leaves a second-order error of at most about
(beta dmu)^2 / 2 in beta mu (T'' = beta^2 sum f(1-f)(1-2f), so
|T''| <= beta T'): at 0.03 that is 4.5e-4, inside the FP64 evaluation's
acceptance of 1e-3 (Sec. II.A occupations; the exact traces come from the
eigenvalues).  Checked on gapless, banded and gapped spectra; where mu lies
in a gap the trace already meets the tolerance and the search ends on it."""
import numpy as np
import pytest

from oracle import density as den

KT = 0.0016
BETA = 1.0 / KT


def trace_and_slope(lam, mu):
    f = den.fermi_dirac(lam, mu, KT)
    return f.sum(), BETA * (f * (1.0 - f)).sum()


def spectra():
    rng = np.random.default_rng(11)
    yield "uniform", np.sort(rng.uniform(-1.0, 1.0, 3000))
    centres = np.linspace(-1.5, 1.5, 20)
    yield "bands", np.sort(np.concatenate([rng.normal(c, 0.01, 150) for c in centres]))
    from workloads.gen import paper_e1_matrix
    yield "paper-e1-600", np.linalg.eigvalsh(paper_e1_matrix(600))


@pytest.mark.parametrize("name,lam", list(spectra()))
def test_newton_handoff_error(name, lam):
    worst, checked = 0.0, 0
    for frac in (0.12, 0.33, 0.47, 0.71, 0.88):
        n_occ = frac * lam.size
        mu_star = den.chemical_potential(lam, n_occ, KT)
        for u in (-0.04, -0.02, -0.005, 0.005, 0.02, 0.04):   # beta (mu - mu*)
            mu = mu_star + u * KT
            t, slope = trace_and_slope(lam, mu)
            if abs(t - n_occ) <= 1e-9:
                continue   # the search ends on the trace itself (mu inside a gap)
            step = -(t - n_occ) / slope
            if abs(BETA * step) > 0.03:
                continue   # the search evaluates again instead
            after = BETA * abs(mu + step - mu_star)
            worst = max(worst, after)
            checked += 1
            assert after <= 0.55 * (BETA * step) ** 2 + 1e-9, (frac, u, after, BETA * step)
    assert checked >= 8 and worst <= 1e-3
