"""Step-level parity on the GPU: every kernel against the CPU oracle (or the
plain definition of the step) on seeded inputs, ragged sizes that span several
tiles, and every precision and epilogue."""
import numpy as np
import pytest

from gpu_util import dev, host, projector_like, say, sym_random

pytestmark = pytest.mark.gpu

RAGGED = [1, 7, 63, 64, 65, 127, 129, 257, 1000]


@pytest.fixture(scope="module")
def fdm():
    import paper_2301_04642_amd as m
    return m


@pytest.mark.parametrize("n", RAGGED)
def test_gershgorin_matches_oracle(fdm, n):
    from oracle import sp2
    rng = np.random.default_rng(100 + n)
    h = sym_random(n, rng)
    say("gershgorin", n)
    lo, hi, tr, f2, bad = fdm.fdm_gershgorin(dev(h))
    rlo, rhi = sp2.gershgorin_bounds(h)
    scale = np.abs(h).sum(axis=1).max()
    assert abs(lo - rlo) <= 1e-13 * scale and abs(hi - rhi) <= 1e-13 * scale
    assert abs(tr - np.trace(h)) <= 1e-12 * (1 + np.abs(np.diag(h)).sum())
    assert abs(f2 - (h * h).sum()) <= 1e-12 * (h * h).sum()
    assert bad == 0


def test_gershgorin_flags_nonfinite(fdm):
    h = np.eye(70)
    h[3, 5] = np.nan
    h[9, 9] = np.inf
    say("gershgorin nonfinite")
    *_, bad = fdm.fdm_gershgorin(dev(h))
    assert bad == 2


def test_gershgorin_leading_dimension(fdm):
    import torch
    rng = np.random.default_rng(7)
    h = sym_random(50, rng)
    big = torch.zeros((50, 64), dtype=torch.float64, device="cuda")
    big[:, :50] = dev(h)
    big[:, 50:] = 1e6   # outside the matrix: must be ignored
    from oracle import sp2
    say("gershgorin ld")
    lo, hi, *_ = fdm.fdm_gershgorin(big[:, :50])
    rlo, rhi = sp2.gershgorin_bounds(h)
    assert abs(lo - rlo) < 1e-12 and abs(hi - rhi) < 1e-12


# (unit roundoff of the stored operands, of the accumulation)
PREC_U = {"fp64": (1.2e-16, 1.2e-16), "fp32": (6.0e-8, 6.0e-8), "fp16x3": (5e-7, 6.0e-8),
          "bf16x3": (3.1e-5, 6.0e-8), "bf16": (4.0e-3, 6.0e-8), "fp16": (5.0e-4, 6.0e-8)}


def product_tol(prec, a, b):
    """Entrywise bound of a length-n dot product with rounded operands and
    accumulation: 4 (2 u_in + sqrt(n) u_acc) max_ij (|A||B|)_ij (+ the FP32
    rounding of the stored FP32 result for the low-precision forms)."""
    u_in, u_acc = PREC_U[prec]
    n = a.shape[0]
    m = (np.abs(a) @ np.abs(b)).max()
    t = 4.0 * (2 * u_in + np.sqrt(n) * u_acc) * m
    if prec != "fp64":
        t += 6e-8 * np.abs(a @ b).max() + 4 * 6e-8 * (np.abs(a).max() + np.abs(b).max())
    return t


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("n", [1, 63, 65, 257, 1000])
@pytest.mark.parametrize("tile", [32, 64, 128])
def test_square_sp2_epilogues(fdm, prec, n, tile):
    """X^2 and 2X - X^2 with the partial sums, against the FP64 definition."""
    import torch
    rng = np.random.default_rng(n)
    x = projector_like(n, rng)
    X = dev(x)
    C = torch.empty_like(X)
    p = x @ x
    tol = product_tol(prec, x, x)
    for alpha, beta, ref in ((1.0, 0.0, p), (-1.0, 2.0, 2 * x - p)):
        say("sym_product", prec, n, tile, alpha, beta)
        tr, f2, d2 = fdm.fdm_sym_product(prec, X, X, X, C, alpha, beta, 0.0, tile=tile)
        c = host(C)
        assert np.array_equal(c, c.T), "result must be exactly symmetric"
        err = np.abs(c - ref).max()
        assert err <= tol + (2e-7 * np.abs(ref).max() if prec != "fp64" else 0), (err, tol)
        assert abs(tr - np.trace(c)) <= 1e-12 * (1 + abs(tr))
        assert abs(f2 - (c * c).sum()) <= 1e-11 * (1 + f2)
        assert abs(np.sqrt(d2) - np.linalg.norm(p - x)) <= 10 * n * tol + 1e-12


@pytest.mark.parametrize("n", [65, 300])
def test_product_orientation_noncommuting(fdm, n):
    """For symmetric but non-commuting A, B the upper triangle is A @ B
    (not B @ A), which fixes operand order and the output lane layout."""
    import torch
    rng = np.random.default_rng(3 * n)
    a = sym_random(n, rng)
    b = sym_random(n, rng)
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    say("orientation", n)
    fdm.fdm_sym_product("fp64", dev(a), dev(b), None, C, tile=64)
    c = host(C)
    iu = np.triu_indices(n)
    ab = a @ b
    assert np.abs(c[iu] - ab[iu]).max() < 1e-12 * np.abs(a).sum(1).max() * np.abs(b).max() * n
    assert np.abs(c[iu] - (b @ a)[iu]).max() > 1e-3


@pytest.mark.parametrize("n", [64, 200])
def test_identity_term_and_general_epilogue(fdm, n):
    """C = alpha A B + beta E + gamma I (McWeeny output 3T - 2TX and the
    Newton-Schulz steps use this form)."""
    import torch
    rng = np.random.default_rng(11 * n)
    x = projector_like(n, rng)
    t = x @ x
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    say("epilogue", n)
    fdm.fdm_sym_product("fp64", dev(t), dev(x), dev(t), C, -2.0, 3.0, 0.25)
    ref = -2.0 * (t @ x) + 3.0 * t + 0.25 * np.eye(n)
    assert np.abs(host(C) - ref).max() < 1e-13 * n


def test_products_bitwise_reproducible(fdm):
    import torch
    rng = np.random.default_rng(5)
    x = projector_like(700, rng)
    X = dev(x)
    outs = []
    for prec in ("fp64", "fp16x3"):
        res = []
        for rep in range(3):
            C = torch.empty_like(X)
            say("repro", prec, rep)
            s = fdm.fdm_sym_product(prec, X, X, X, C, 1.0, 0.0, 0.0)
            res.append((host(C), s))
        for c, s in res[1:]:
            assert np.array_equal(c, res[0][0]) and s == res[0][1]


@pytest.mark.parametrize("n", [1, 65, 1000])
def test_band_energy(fdm, n):
    rng = np.random.default_rng(n + 1)
    h = sym_random(n, rng)
    d = projector_like(n, rng)
    say("band energy", n)
    e, tr = fdm.fdm_band_energy(dev(h), dev(d))
    assert abs(e - (h * d).sum()) <= 1e-12 * np.abs(h * d).sum()
    assert abs(tr - np.trace(d)) <= 1e-12 * n


@pytest.mark.parametrize("n", [4000, 3900])
def test_edge_block_products(fdm, n):
    """128-wide split products whose K extent ends 64 columns into the last
    tile column (round_up(n, 64) = 128 T - 64: T = 32 at n = 4000, the odd
    T = 31 at n = 3900): that column runs as 256 x 64 edge blocks.  Every
    entry against the FP64 product of the same operands, exact symmetry, the
    trace partial sum, and the same result as 64-wide tiles to rounding."""
    import torch
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal((n, n)) / np.sqrt(n)
    x = 0.5 * (x + x.T)
    ref = x @ x
    X = dev(x)
    C, C64 = torch.empty_like(X), torch.empty_like(X)
    for prec in ("fp16x3", "bf16x3"):
        say("edge-block product", prec, n)
        tr, f2, _ = fdm.fdm_sym_product(prec, X, X, None, C, 1.0, 0.0, 0.0, tile=128)
        fdm.fdm_sym_product(prec, X, X, None, C64, 1.0, 0.0, 0.0, tile=64)
        c, c64 = host(C), host(C64)
        assert np.array_equal(c, c.T), "result must be exactly symmetric"
        err = np.abs(c - ref).max()
        tol = product_tol(prec, x, x)
        print(f"[report] edge blocks n={n} {prec}: max err {err:.2e} (tol {tol:.2e}), "
              f"vs 64-wide tiles {np.abs(c - c64).max():.2e}", flush=True)
        assert err <= tol
        assert np.abs(c - c64).max() <= tol
        assert abs(tr - np.trace(c)) <= 1e-9 * (1 + abs(np.trace(c)))
    del X, C, C64


@pytest.mark.parametrize("n", [18000, 18500])
def test_large_tile128_products_sampled(fdm, n):
    """128-wide products at full size, either side of the padded leading
    dimension (18048 | 18560) where the split forms switch from direct-to-LDS
    to register staging: 64 sampled entries of X^2 and their mirrors against
    FP64 dot products of the same operands."""
    import torch
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n), dtype=np.float32).astype(np.float64)
    x += x.T
    x *= 0.5 / np.sqrt(n)
    X = dev(x)
    C = torch.empty_like(X)
    ii = rng.integers(0, n, 64)
    jj = rng.integers(0, n, 64)
    ref = np.einsum("ij,ij->i", x[ii], x[jj])
    mag = np.einsum("ij,ij->i", np.abs(x[ii]), np.abs(x[jj]))
    ti, tj = torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()
    for prec in ("fp64", "fp32", "fp16x3", "bf16x3"):
        say("large tile-128 product", prec, n)
        fdm.fdm_sym_product(prec, X, X, None, C, 1.0, 0.0, 0.0, tile=128)
        got = host(C[ti, tj])
        assert np.array_equal(got, host(C[tj, ti])), "result must be exactly symmetric"
        u_in, u_acc = PREC_U[prec]
        tol = 4.0 * (2 * u_in + np.sqrt(n) * u_acc) * mag
        if prec != "fp64":
            tol += 6e-8 * np.abs(ref) + 8 * 6e-8 * np.abs(x).max()
        err = np.abs(got - ref)
        assert (err <= tol).all(), (prec, float(err.max()), float(tol[np.argmax(err - tol)]))
    del X, C
