"""fdm_sym_product_noalloc (the product on the library's fixed device array)
against fdm_sym_product: the same kernels on the same inputs give the same
bits, on two calls in a row (the second smaller, so the array holds the first
call's larger contents), and both stay within the product's entrywise bound
of the FP64 definition.  Sizes above the array's limit are rejected."""
import numpy as np
import pytest

from gpu_util import dev, host, projector_like, say, sym_random
from test_gpu_kernels import product_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdm():
    import paper_2301_04642_amd as m
    return m


def _pair(fdm, prec, n, seed, tile):
    import torch
    rng = np.random.default_rng(seed)
    x = projector_like(n, rng)
    e = sym_random(n, rng, 0.1)
    X, E = dev(x), dev(e)
    C0 = torch.full_like(X, np.nan)
    C1 = torch.full_like(X, np.nan)
    say("noalloc", prec, n, tile)
    s0 = fdm.fdm_sym_product(prec, X, X, E, C0, -1.0, 2.0, 0.5, tile=tile)
    s1 = fdm.fdm_sym_product_noalloc(prec, X, X, E, C1, -1.0, 2.0, 0.5, tile=tile)
    c0, c1 = host(C0), host(C1)
    assert np.array_equal(c0, c1), "no-allocation product differs from fdm_sym_product"
    assert s0 == s1
    ref = -(x @ x) + 2.0 * e + 0.5 * np.eye(n)
    tol = product_tol(prec, x, x) + (2e-7 * np.abs(ref).max() if prec != "fp64" else 0)
    assert np.abs(c1 - ref).max() <= tol
    assert np.array_equal(c1, c1.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3", "bf16x3"])
@pytest.mark.parametrize("tile", [0, 32, 128])
def test_noalloc_matches_product_twice(fdm, prec, tile):
    _pair(fdm, prec, 1408, 11, tile)   # the largest size the array holds
    _pair(fdm, prec, 333, 12, tile)    # then a smaller, ragged one


def test_noalloc_rejects_above_limit(fdm):
    import torch
    n = 1409
    X = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    C = torch.zeros_like(X)
    say("noalloc reject", n)
    with pytest.raises(fdm.FdmError) as ei:
        fdm.fdm_sym_product_noalloc("fp64", X, X, None, C)
    assert ei.value.code == fdm.FDM_EINVAL and "1408" in str(ei.value)
