"""CPU oracle pinned to closed forms, invariants, brute force and a library
routine (never to itself).  See tests/oracle_pins.py for each pin."""
import numpy as np
import pytest

import oracle_pins as pins
from oracle import density as den
from oracle import fd, sp2


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_density_vs_construction_finite_t():
    pins.check_density_vs_construction(kT=0.0016)


def test_sp2_iteration_count_plausible():
    """Sec. IV reports about 50 SP2 products at its tolerance; a dense rotated
    band spectrum with Gershgorin bounds needs a similar count here."""
    import workloads
    wl = workloads.standard_workload("bands", n=400)
    x, info = sp2.sp2(wl.hp, wl.n_occ, tol=1e-8)
    assert info["converged"]
    assert 35 <= info["iterations"] <= 65, info["iterations"]


def test_reltr_definition():
    t = [10.0, 12.0, 11.5]
    assert np.allclose(sp2.rel_trace(t), [0.2, 0.5 / 12.0])


# --------------------------------------------------------------------------
# planted mistakes: each mutant of the oracle must fail at least one pin
# --------------------------------------------------------------------------

def _fails(fn, *a, **k):
    try:
        fn(*a, **k)
    except AssertionError:
        return True
    return False


def test_mutant_branch_rule_flipped(monkeypatch):
    monkeypatch.setattr(sp2, "choose_square",
                        lambda t, s, n: abs(s - n) > abs(2 * t - s - n))
    assert _fails(pins.check_sp2_matches_definition, sizes=(16,))


def test_mutant_dropped_term_in_update():
    def bad_sp2(h, n_occ, tol=1e-10, max_iter=100):
        lo, hi = sp2.gershgorin_bounds(h)
        x = sp2.initial_iterate(h, lo, hi)
        br = []
        for _ in range(max_iter):
            t, s = np.trace(x), np.sum(x * x)
            sq = sp2.choose_square(t, s, n_occ)
            p = x @ x
            if np.linalg.norm(p - x) <= tol:
                break
            br.append(1 if sq else 0)
            x = p if sq else x - p        # dropped "X +" term
        return x, dict(branches=br, converged=True)
    assert _fails(pins.check_sp2_diagonal, sp2fn=bad_sp2)


def test_mutant_transposed_eigenbasis():
    def bad_dm(h, n_occ, kT=0.0):
        d, e, mu, lam = den.density_matrix(h, n_occ, kT)
        w, v = np.linalg.eigh(h)
        f, _ = den.occupations(w, n_occ, kT)
        return (v.T * f) @ v, e, mu, lam       # Q^T f Q instead of Q f Q^T
    assert _fails(pins.check_density_vs_construction, density_matrix=bad_dm)


def test_mutant_gershgorin_radius_includes_diagonal():
    def bad_bounds(h):
        r = np.abs(h).sum(axis=1)
        return float((np.diag(h) - r).min()), float((np.diag(h) + r).max())
    assert _fails(pins.check_gershgorin, bounds=bad_bounds)


def test_mutant_fermi_missing_half():
    bad = lambda lam, mu, kT: 0.5 * (1.0 - np.tanh((np.asarray(lam) - mu) / kT))
    assert _fails(pins.check_fd_two_level, fermi=bad,
                  chem=lambda lam, n, kT: 0.0)


def test_mutant_doubling_wrong_start_scale():
    def bad(h, mu, beta, m):
        n = h.shape[0]
        eye = np.eye(n)
        y = beta * (h - mu * eye) / 2.0 ** (m + 1)   # wrong power of two
        for _ in range(m):
            y = np.linalg.solve(eye + 4.0 * y @ y, 2.0 * y)
        return 0.5 * eye - y
    assert _fails(pins.check_fd_recursion_closed_form, doubling=bad)


def test_mutant_jacobi_wrong_rotation_sign():
    def bad_eigh(h):
        w, v = np.linalg.eigh(h)
        return w, v[::-1]                              # rows permuted: wrong eigenvectors
    assert _fails(pins.check_jacobi_2x2, eigh=bad_eigh)


# --------------------------------------------------------------------------
# golden fixtures: the paper's own synthetic matrix (Sec. IV) at N = 8
# --------------------------------------------------------------------------

def _read_golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        out[k] = np.array([float(x) for x in v])
    return out


def test_golden_e1_zero_t():
    from workloads import paper_e1_matrix
    g = _read_golden("e1_n8_zero_t.txt")
    h = paper_e1_matrix(8)
    # independent check of the stored values with LAPACK
    w, v = np.linalg.eigh(h)
    assert np.allclose(g["eigenvalues"], w, atol=1e-13)
    d = v[:, :7] @ v[:, :7].T
    assert np.allclose(g["d_diag"], np.diag(d), atol=1e-13)
    assert np.allclose(g["d_row0"], d[0], atol=1e-13)
    assert abs(g["band_energy"][0] - w[:7].sum()) < 1e-13
    # and the oracle reproduces them
    d2, e2, _, _ = den.density_matrix(h, 7, 0.0)
    assert abs(e2 - g["band_energy"][0]) < 1e-13
    x, info = sp2.sp2(h, 7, tol=1e-12)
    assert np.abs(x - d).max() < 1e-11


def test_golden_e1_finite_t():
    from workloads import paper_e1_matrix
    g = _read_golden("e1_n8_finite_t.txt")
    h = paper_e1_matrix(8)
    w, v = np.linalg.eigh(h)
    kT = 0.0016
    mu = g["mu"][0]
    f = 1.0 / (np.exp((w - mu) / kT) + 1.0)
    assert abs(f.sum() - 6.8) < 1e-10
    d = (v * f) @ v.T
    assert np.allclose(g["d_diag"], np.diag(d), atol=1e-12)
    assert abs(g["band_energy"][0] - np.dot(f, w)) < 1e-12
    m = fd.depth(1.0 / kT, w.min(), w.max(), mu, extra=8)
    dm = fd.doubling(h, mu, 1.0 / kT, m)
    assert np.abs(dm - d).max() < 1e-11


def _az_step_variant(half=0.5, drop_linear=False, unshifted_bound=False, flip=False):
    """A copy of the accelerated step with one planted mistake."""
    def step(l, h):
        e_u, e_o = l, 1.0 - h
        if (e_u >= e_o) != flip:
            s = half * e_u
            k = 1.0 / (1.0 - s) ** 2
            coef = (k, 0.0 if drop_linear else -2.0 * k * s, k * s * s)
            h2 = k * h * h if unshifted_bound else k * (h - s) ** 2
            return coef, 1, s, k * max(s, e_u - s) ** 2, h2
        s = half * e_o
        k = 1.0 / (1.0 - s) ** 2
        u = 1.0 - s
        coef = (-k, 0.0 if drop_linear else 2.0 * k * u, 1.0 - k * u * u)
        return coef, 0, s, 1.0 - k * (u - l) ** 2, 1.0 - k * max(s, e_o - s) ** 2
    return step


def test_mutant_azrfoe_fold_point():
    assert _fails(pins.check_azrfoe_fold, step=_az_step_variant(half=1.0))


def test_mutant_azrfoe_dropped_linear_term():
    assert _fails(pins.check_azrfoe_fold, step=_az_step_variant(drop_linear=True))


def test_mutant_azrfoe_unshifted_bound(monkeypatch):
    from oracle import azrfoe as az
    monkeypatch.setattr(az, "step_polynomial", _az_step_variant(unshifted_bound=True))
    assert _fails(pins.check_azrfoe_diagonal, azfn=az.azrfoe)


def test_mutant_azrfoe_branch_flipped(monkeypatch):
    from oracle import azrfoe as az
    monkeypatch.setattr(az, "step_polynomial", _az_step_variant(flip=True))
    assert _fails(pins.check_azrfoe_matches_definition, azfn=az.azrfoe, sizes=(16,))


# --------------------------------------------------------------------------
# planted mistakes in the full-size references and the metrics
# --------------------------------------------------------------------------

def test_mutant_sp2_stop_on_idempotency_only():
    def bad_sp2(h, n_occ, tol=1e-10, max_iter=100, bounds=None):
        lo, hi = bounds
        x = sp2.initial_iterate(h, lo, hi)
        it = 0
        for it in range(max_iter):
            t, s = np.trace(x), np.sum(x * x)
            p = x @ x
            if np.linalg.norm(p - x) <= tol:        # trace condition dropped
                break
            x = p if sp2.choose_square(t, s, n_occ) else 2 * x - p
        return x, dict(iterations=it, converged=True)
    assert _fails(pins.check_sp2_stop_rule, sp2fn=bad_sp2)


def test_mutant_density_rows_without_occupations():
    def bad(q_rows, n, f, rows, chunk=4096):
        return den.density_rows(q_rows, n, np.ones_like(f), rows, chunk)
    assert _fails(pins.check_density_rows, rows_fn=bad)


def test_mutant_density_rows_chunk_offset():
    def bad(q_rows, n, f, rows, chunk=4096):
        qr = q_rows(np.asarray(rows)) * f[None, :]
        out = np.empty((len(rows), n))
        for c0 in range(0, n, chunk):
            idx = np.arange(c0, min(n, c0 + chunk))
            out[:, c0:c0 + idx.size] = qr @ q_rows(np.minimum(idx + 1, n - 1)).T
        return out
    assert _fails(pins.check_density_rows, rows_fn=bad)


def test_mutant_kron_wrong_axis_order(monkeypatch):
    import workloads.gen as gen

    def bad_hp(qa, qb, lam_grid):
        a, b = qa.shape[0], qb.shape[0]
        t = np.einsum('ik,ck,jk->cij', qb, lam_grid, qb, optimize=True)
        w = (qa[:, None, :] * qa[None, :, :]).reshape(a * a, a)
        h = (w @ t.reshape(a, b * b)).reshape(a, a, b, b)
        return np.ascontiguousarray(h).reshape(a * b, a * b)   # axes not interleaved
    monkeypatch.setattr(gen, "_hp_from_kron", bad_hp)
    assert _fails(pins.check_kron_workload, make=gen.make_workload)


def test_mutant_e1_band_wrong_row_index():
    def bad(n, bandwidth=80):
        bw = min(bandwidth, n - 1)
        ab = np.zeros((bw + 1, n))
        for d in range(bw + 1):
            j = np.arange(d, n)
            ab[bw - d, d:] = np.exp(-0.5 * d) * np.sin(j + 1.0)   # column index, not min
        return ab
    assert _fails(pins.check_paper_e1_band, band=bad)


def test_mutant_eps1_unnormalised():
    assert _fails(pins.check_eps_metrics, e1=lambda d, r: float(np.linalg.norm(d - r)))


def test_mutant_eps2_unsigned():
    assert _fails(pins.check_eps_metrics, e2=lambda e, r: abs((e - r) / r))


def test_mutant_reltr_absolute_change():
    def bad(h, n_occ, tol=1e-10, max_iter=100, bounds=None, reltr_stop=None):
        x = sp2.initial_iterate(h, *bounds)
        for it in range(1, max_iter):
            t, s = np.trace(x), np.sum(x * x)
            p = x @ x
            x = p if sp2.choose_square(t, s, n_occ) else 2 * x - p
            if abs(np.trace(x) - t) <= reltr_stop:          # not relative
                break
        return x, dict(iterations=it)
    assert _fails(pins.check_sp2_reltr_stop, sp2fn=bad)


def test_mutant_trfoe_wrong_map():
    from oracle import trfoe

    def bad(lam, n_occ, kT, e_min, e_max, m=None):
        m = trfoe.depth(kT, e_min, e_max) if m is None else m
        x = (e_max - np.asarray(lam)) / (e_max - e_min)
        for _ in range(m):
            t, s = x.sum(), (x * x).sum()
            x = x * x if sp2.choose_square(t, s, n_occ) else 2 * x + x * x   # sign
        return x, dict(branches=[], depth=m)
    assert _fails(pins.check_trfoe_properties, scal=bad)


def test_mutant_trfoe_depth_base_two(monkeypatch):
    from oracle import trfoe
    monkeypatch.setattr(trfoe, "GROWTH", 2.0)
    assert _fails(pins.check_trfoe_slope, scal=trfoe.scalar)


def test_mutant_trfoe_dense_transposed_start():
    from oracle import trfoe

    def bad(h, n_occ, kT, bounds=None, m=None):
        e_min, e_max = bounds
        return trfoe.dense(h - 0.05 * np.eye(h.shape[0]), n_occ, kT, bounds=(e_min, e_max), m=m)
    assert _fails(pins.check_trfoe_dense_vs_spectral, dense=bad)
