"""Helpers for the GPU tests: device tensors from numpy, the oracle's
reference quantities, and printed case names (flushed before each GPU step)."""
import sys

import numpy as np


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def dev(a):
    torch = need_gpu()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def reference(wl):
    """(D_ref, E_ref, mu) of a workload from its known eigenbasis (oracle)."""
    from oracle import density as den
    f, mu = den.occupations(wl.lam, wl.n_occ, wl.kT)
    d, e = den.density_from_eig(wl.q_full(), wl.lam, f)
    return d, e, mu, f


def sym_random(n, rng, scale=1.0):
    g = rng.standard_normal((n, n))
    return scale * 0.5 * (g + g.T)


def projector_like(n, rng, k=None):
    """Symmetric X with spectrum in [0, 1] (a dense commuting pair X, X^2)."""
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = rng.uniform(0.0, 1.0, n)
    return (q * s) @ q.T
