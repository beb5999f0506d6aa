"""CPU checks of the hidden-outlier inputs: the matrix has the stated
spectrum, the outlier's eigenvector is orthogonal to the Lanczos start
vector, and a numpy replay of the 16-step estimate misses the outlier."""
import numpy as np
import pytest

from spectral_probe import hidden_outlier_workload, lanczos_estimate, lanczos_start_vector


def test_start_vector_is_a_fixed_unit_vector():
    v = lanczos_start_vector(1000)
    assert abs(np.linalg.norm(v) - 1.0) < 1e-14
    # entry i depends on i alone: a prefix, renormalised, is the shorter vector
    assert np.allclose(v[:300] / np.linalg.norm(v[:300]), lanczos_start_vector(300),
                       rtol=1e-14, atol=1e-16)
    # spread like a uniform (-1/2, 1/2) sample
    raw = v * np.sqrt(1000 / 12.0)
    assert 0.9 < np.std(raw) * np.sqrt(12.0) < 1.1 and abs(np.mean(raw)) < 0.05


@pytest.mark.parametrize("lam_out", [1.06, 2.6])
def test_lanczos_replay_misses_the_hidden_outlier(lam_out):
    n, n_occ = 600, 150
    hp, vals, vecs = hidden_outlier_workload(n, n_occ, lam_out)
    assert np.abs((vecs * vals) @ vecs.T - hp).max() < 1e-13
    assert np.abs(vecs.T @ vecs - np.eye(n)).max() < 1e-13
    assert abs(vecs[:, -1] @ lanczos_start_vector(n)) < 1e-15
    w = np.linalg.eigvalsh(hp)
    assert abs(w[-1] - lam_out) < 1e-12 and w[-2] <= 1.0
    lo, hi = lanczos_estimate(hp)
    # the estimate covers the bulk it sees but not the outlier
    assert hi < lam_out and lo <= w[0] + 1e-9
    assert hi >= 0.95
