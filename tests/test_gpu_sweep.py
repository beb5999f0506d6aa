"""A seeded sweep over sizes, precisions, spectral-bound modes and
temperatures and tile edges (half the cases pick the edge from N, the others
force 32-, 64- or 128-wide tiles): every solve against the definition of the
density matrix, at the FP64 or mixed-precision gates."""
import numpy as np
import pytest

import workloads
from gpu_util import dev, host, reference, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdm():
    import paper_2301_04642_amd as m
    return m


def cases(count=36, seed=20261203):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(2), np.log(2100))))
        kind = ["gapped", "bands", "uniform"][i % 3]
        prec = ["fp64", "fp32", "fp16x3", "bf16x3"][int(rng.integers(4))]
        bounds = int(rng.integers(2))
        tile = [0, 128, 0, 64, 0, 32][i % 6]
        out.append((i, n, kind, prec, bounds, tile))
    return out


@pytest.mark.parametrize("i,n,kind,prec,bounds,tile", cases())
def test_sweep(fdm, i, n, kind, prec, bounds, tile):
    if kind == "bands" and n < 40:
        n = 40                       # twenty bands need a few states each
    wl = workloads.standard_workload(kind, n=n, seed_base=7000 + i)
    if wl.n_occ <= 0:
        pytest.skip("no occupied state")
    d_ref, e_ref, _, _ = reference(wl)
    fp64 = prec == "fp64"
    tol = 1e-10 if fp64 else 1e-8
    say("sweep", i, n, kind, prec, bounds, tile)
    D, e, st = fdm.solve(dev(wl.hp), wl.n_occ, wl.kT, tol, prec, bounds=bounds, tile=tile)
    d = host(D)
    de = abs(e - e_ref)
    dtr = abs(np.trace(d) - wl.n_occ)
    print(f"[report] sweep {i}: n={n} {kind} {prec} bounds={bounds} tile={st.tile} |dE|={de:.1e} "
          f"|dTr|={dtr:.1e} ||dD||={np.linalg.norm(d - d_ref):.1e}", flush=True)
    assert st.status == 0
    assert np.array_equal(d, d.T)
    # energies above 1000 Ha are gated relatively (the FP64 floor summed over states)
    assert de <= (max(1e-10, 1e-13 * abs(e_ref)) if fp64 else 1e-6)
    assert dtr <= tol
    if fp64:
        assert np.linalg.norm(d - d_ref) <= 1e-9
    if wl.kT == 0.0:
        assert np.linalg.norm(d @ d - d) <= (1e-10 if fp64 else 1e-8)
