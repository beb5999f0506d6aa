"""Python binding of libfermidm (MI355X / gfx950 density-matrix library).

Argument marshalling only: every step runs in the HIP library built from
``csrc/`` (``python paper_2301_04642_amd/build.py``).  PyTorch provides device
memory and the current stream.  Importing this module fails loudly when the
library has not been built; there is no CPU fallback.

The functions mirror the C ABI in ``include/fermidm.h`` (same names), plus
``solve`` which allocates D with torch.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfermidm.so")

FDM_OK, FDM_EINVAL, FDM_ENOMEM, FDM_ENOCONV, FDM_EHIP, FDM_ENONFINITE = 0, -1, -2, -3, -4, -5
FDM_FP64, FDM_FP32, FDM_FP16X3, FDM_BF16X3, FDM_BF16, FDM_FP16 = range(6)
FDM_NPREC = 6
PRECISIONS = {"fp64": FDM_FP64, "fp32": FDM_FP32, "fp16x3": FDM_FP16X3,
              "bf16x3": FDM_BF16X3, "bf16": FDM_BF16, "fp16": FDM_FP16}
PREC_NAMES = {v: k for k, v in PRECISIONS.items()}

# the public entry points declared in include/fermidm.h
EXPORTS = ("fdm_options_default", "fdm_workspace_bytes", "fermi_dm_solve", "fdm_strerror",
           "fdm_last_error", "fdm_gershgorin", "fdm_sym_product", "fdm_band_energy",
           "fdm_fermi_operator", "fdm_server_create", "fdm_submit", "fdm_poll", "fdm_result",
           "fdm_server_memory", "fdm_server_destroy", "fdm_sym_product_noalloc")


class fdm_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("k64", ctypes.c_int32), ("tau", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("mcweeny_max", ctypes.c_int32),
                ("max_mu_evals", ctypes.c_int32), ("fd_extra_depth", ctypes.c_int32),
                ("fd_final_fp64", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("bounds", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("estimate_gap", ctypes.c_int32), ("homo", ctypes.c_double),
                ("lumo", ctypes.c_double), ("mu_guess", ctypes.c_double),
                ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("reltr_schedule", ctypes.c_int32),
                ("trfoe", ctypes.c_int32), ("reltr_switch", ctypes.c_double),
                ("reltr_stop", ctypes.c_double), ("trfoe_depth", ctypes.c_int32),
                ("reserved0", ctypes.c_int32)]


class fdm_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters_fp64_first", ctypes.c_int32),
                ("iters_low", ctypes.c_int32), ("iters_fp64", ctypes.c_int32),
                ("mcweeny_steps", ctypes.c_int32), ("mu_evals", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("products", ctypes.c_int32 * FDM_NPREC), ("branch_bits", ctypes.c_uint64 * 4),
                ("e_min", ctypes.c_double), ("e_max", ctypes.c_double), ("mu", ctypes.c_double),
                ("idempotency", ctypes.c_double), ("trace", ctypes.c_double),
                ("band_energy", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("prod_ms", ctypes.c_double * FDM_NPREC), ("flops", ctypes.c_double * FDM_NPREC),
                ("gersh_min", ctypes.c_double), ("gersh_max", ctypes.c_double),
                ("lanczos_steps", ctypes.c_int32), ("accelerated", ctypes.c_int32),
                ("mcweeny_idem", ctypes.c_double * 4), ("mcweeny_trace_err", ctypes.c_double * 4),
                ("mu_hist", ctypes.c_double * 16), ("mu_trace_err", ctypes.c_double * 16),
                ("fallback_fp64", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("homo_ub", ctypes.c_double), ("lumo_lb", ctypes.c_double),
                ("rel_trace", ctypes.c_double), ("idem_tail", ctypes.c_double * 8),
                ("idem_tail_len", ctypes.c_int32), ("bounds_certified", ctypes.c_int32),
                ("lanczos_min", ctypes.c_double), ("lanczos_max", ctypes.c_double),
                ("cert_radius", ctypes.c_double), ("phase_ms", ctypes.c_double * 4),
                ("trfoe_depth", ctypes.c_int32), ("reltr_schedule", ctypes.c_int32),
                ("tick_steps", ctypes.c_int32), ("tick_shared", ctypes.c_int32)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if isinstance(v, ctypes.Array):
                v = list(v)
            d[name] = v
        d["branches"] = branch_list(self)
        return d


class fdm_server_options(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("independent", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class FdmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2301_04642_amd/build.py`")
    # PyTorch bundles its own HIP runtime with the same soname as the system
    # one.  Load torch's first so that libfermidm binds to it: one HIP runtime
    # (and one HSA runtime) per process, shared device memory and streams.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I32, I64, VP = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                          ctypes.c_void_p)
    sig = {
        "fdm_options_default": (ctypes.c_int, [ctypes.POINTER(fdm_options)]),
        "fdm_workspace_bytes": (ctypes.c_size_t, [I64, D, I32]),
        "fermi_dm_solve": (ctypes.c_int, [P, I64, I64, D, D, D, P, I64, ctypes.POINTER(D),
                                          ctypes.POINTER(fdm_options), ctypes.POINTER(fdm_stats),
                                          VP]),
        "fdm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "fdm_last_error": (ctypes.c_char_p, []),
        "fdm_gershgorin": (ctypes.c_int, [P, I64, I64, ctypes.POINTER(D), ctypes.POINTER(I32),
                                          VP]),
        "fdm_sym_product": (ctypes.c_int, [I32, P, P, P, P, I64, I64, D, D, D, ctypes.POINTER(D),
                                           I32, VP]),
        "fdm_sym_product_noalloc": (ctypes.c_int, [I32, P, P, P, P, I64, I64, D, D, D,
                                                   ctypes.POINTER(D), I32, VP]),
        "fdm_band_energy": (ctypes.c_int, [P, I64, P, I64, I64, ctypes.POINTER(D), VP]),
        "fdm_fermi_operator": (ctypes.c_int, [P, I64, I64, D, D, I32, I32, P, I64,
                                              ctypes.POINTER(D), VP]),
        "fdm_server_create": (ctypes.c_void_p, [ctypes.POINTER(fdm_server_options)]),
        "fdm_submit": (ctypes.c_int, [VP, P, I32, I64, D, D, D, I32,
                                      ctypes.POINTER(ctypes.c_uint64)]),
        "fdm_poll": (ctypes.c_int, [VP, ctypes.c_uint64]),
        "fdm_result": (ctypes.c_int, [VP, ctypes.c_uint64, P, I32, I64, ctypes.POINTER(D),
                                      ctypes.POINTER(fdm_stats), ctypes.POINTER(D)]),
        "fdm_server_memory": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_size_t),
                                             ctypes.POINTER(ctypes.c_size_t),
                                             ctypes.POINTER(ctypes.c_size_t)]),
        "fdm_server_destroy": (None, [VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def library():
    return _lib


def _check(rc, what):
    if rc != FDM_OK:
        msg = _lib.fdm_last_error().decode() or _lib.fdm_strerror(rc).decode()
        raise FdmError(rc, f"{what}: {msg}")
    return rc


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_matrix(t, n=None, name="matrix"):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
        raise ValueError(f"{name} must be a CUDA float64 row-major matrix")
    if n is not None and (t.shape[0] != n or t.shape[1] != n):
        raise ValueError(f"{name} must be {n} x {n}")
    return t.stride(0)


def branch_list(stats):
    """SP2 branches of the solve (1 = X^2), from stats.branch_bits."""
    n = stats.iters_fp64 + stats.iters_fp64_first + stats.iters_low
    bits = list(stats.branch_bits)
    return [(bits[k >> 6] >> (k & 63)) & 1 for k in range(min(n, 256))]


def fdm_options_default():
    o = fdm_options()
    _check(_lib.fdm_options_default(ctypes.byref(o)), "fdm_options_default")
    return o


def fdm_workspace_bytes(n, kT=0.0, precision=FDM_FP64):
    return int(_lib.fdm_workspace_bytes(int(n), float(kT), int(precision)))


def fdm_strerror(code):
    return _lib.fdm_strerror(int(code)).decode()


def fdm_last_error():
    return _lib.fdm_last_error().decode()


def fermi_dm_solve(H, n_occ, kT, tol, D, options=None, stream=None, raise_on_error=True):
    """Calls fermi_dm_solve on torch tensors H (input) and D (output).
    Returns (status, E_band, stats)."""
    n = H.shape[0]
    ldh = _check_matrix(H, n, "Hp")
    ldd = _check_matrix(D, n, "D")
    e = ctypes.c_double(0.0)
    st = fdm_stats()
    opt = options if options is not None else fdm_options_default()
    rc = _lib.fermi_dm_solve(_ptr(H), n, ldh, float(n_occ), float(kT), float(tol), _ptr(D), ldd,
                             ctypes.byref(e), ctypes.byref(opt), ctypes.byref(st), _stream(stream))
    if raise_on_error and rc not in (FDM_OK,):
        _check(rc, "fermi_dm_solve")
    return rc, e.value, st


def solve(H, n_occ, kT=0.0, tol=1e-8, precision="fp64", stream=None, raise_on_error=True,
          **opts):
    """D, E_band, stats for the torch CUDA float64 matrix H."""
    import torch
    opt = fdm_options_default()
    opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for k, v in opts.items():
        setattr(opt, k, v)
    D = torch.empty_like(H)
    rc, e, st = fermi_dm_solve(H, n_occ, kT, tol, D, opt, stream, raise_on_error)
    return D, e, st


def fdm_gershgorin(H, stream=None):
    """(e_min, e_max, Tr H, ||H||_F^2, nonfinite_rows)."""
    n = H.shape[0]
    ld = _check_matrix(H, n, "H")
    out = (ctypes.c_double * 4)()
    bad = ctypes.c_int32(0)
    _check(_lib.fdm_gershgorin(_ptr(H), n, ld, out, ctypes.byref(bad), _stream(stream)),
           "fdm_gershgorin")
    return out[0], out[1], out[2], out[3], bad.value


def fdm_sym_product(precision, A, B, E, C, alpha=1.0, beta=0.0, gamma=0.0, tile=0, stream=None):
    """C = alpha A B + beta E + gamma I on the upper tiles, mirrored.
    Returns (Tr C, ||C||_F^2, ||AB - E||_F^2)."""
    n = A.shape[0]
    ld = _check_matrix(A, n, "A")
    for t, nm in ((B, "B"), (C, "C")) + (((E, "E"),) if E is not None else ()):
        if _check_matrix(t, n, nm) != ld:
            raise ValueError("A, B, E and C must share one leading dimension")
    sums = (ctypes.c_double * 3)()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.fdm_sym_product(prec, _ptr(A), _ptr(B), _ptr(E), _ptr(C), n, ld, float(alpha),
                                float(beta), float(gamma), sums, int(tile), _stream(stream)),
           "fdm_sym_product")
    return sums[0], sums[1], sums[2]


def fdm_sym_product_noalloc(precision, A, B, E, C, alpha=1.0, beta=0.0, gamma=0.0, tile=0,
                            stream=None):
    """fdm_sym_product on the library's fixed device workspace (no allocation;
    N <= 1408).  Returns (Tr C, ||C||_F^2, ||AB - E||_F^2)."""
    n = A.shape[0]
    ld = _check_matrix(A, n, "A")
    for t, nm in ((B, "B"), (C, "C")) + (((E, "E"),) if E is not None else ()):
        if _check_matrix(t, n, nm) != ld:
            raise ValueError("A, B, E and C must share one leading dimension")
    sums = (ctypes.c_double * 3)()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.fdm_sym_product_noalloc(prec, _ptr(A), _ptr(B), _ptr(E), _ptr(C), n, ld,
                                        float(alpha), float(beta), float(gamma), sums, int(tile),
                                        _stream(stream)), "fdm_sym_product_noalloc")
    return sums[0], sums[1], sums[2]


def fdm_band_energy(H, D, stream=None):
    """(Tr(H D), Tr D)."""
    n = H.shape[0]
    ldh = _check_matrix(H, n, "H")
    ldd = _check_matrix(D, n, "D")
    out = (ctypes.c_double * 2)()
    _check(_lib.fdm_band_energy(_ptr(H), ldh, _ptr(D), ldd, n, out, _stream(stream)),
           "fdm_band_energy")
    return out[0], out[1]


def fdm_fermi_operator(H, mu, kT, D, depth=0, precision=FDM_FP64, stream=None):
    """One evaluation of the finite-temperature recursion at mu into D.
    Returns (Tr D, Tr(D - D^2), depth)."""
    n = H.shape[0]
    ldh = _check_matrix(H, n, "H")
    ldd = _check_matrix(D, n, "D")
    out = (ctypes.c_double * 3)()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.fdm_fermi_operator(_ptr(H), n, ldh, float(mu), float(kT), int(depth), prec,
                                   _ptr(D), ldd, out, _stream(stream)), "fdm_fermi_operator")
    return out[0], out[1], int(out[2])


class Server:
    """Continuous-batching server (fdm_server_* of the C ABI)."""

    def __init__(self, budget_bytes, max_active=4, precision="fp32", grouped=True):
        o = fdm_server_options(int(budget_bytes), int(max_active),
                               PRECISIONS[precision] if isinstance(precision, str) else precision,
                               0 if grouped else 1, 0)
        self._s = _lib.fdm_server_create(ctypes.byref(o))
        if not self._s:
            raise FdmError(FDM_EINVAL, "fdm_server_create: " + fdm_last_error())

    def submit(self, hp, n_occ, kT=0.0, tol=1e-8, precision=-1):
        """hp: numpy float64 (host) or torch CUDA float64 (device) N x N, contiguous."""
        import numpy as np
        t = ctypes.c_uint64(0)
        if isinstance(hp, np.ndarray):
            hp = np.ascontiguousarray(hp, dtype=np.float64)
            ptr, on_host, n = ctypes.c_void_p(hp.ctypes.data), 1, hp.shape[0]
        else:
            if not hp.is_contiguous():
                raise ValueError("device Hp must be contiguous")
            ptr, on_host, n = _ptr(hp), 0, hp.shape[0]
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(_lib.fdm_submit(self._s, ptr, on_host, n, float(n_occ), float(kT), float(tol),
                               prec, ctypes.byref(t)), "fdm_submit")
        return t.value

    def poll(self, ticket):
        return _lib.fdm_poll(self._s, ticket)

    def result(self, ticket, n, out=None):
        """Returns (status, D (numpy), E_band, stats, times[4])."""
        import numpy as np
        d = np.empty((n, n)) if out is None else out
        e = ctypes.c_double(0.0)
        st = fdm_stats()
        times = (ctypes.c_double * 4)()
        rc = _lib.fdm_result(self._s, ticket, ctypes.c_void_p(d.ctypes.data), 1, n,
                             ctypes.byref(e), ctypes.byref(st), times)
        return rc, d, e.value, st, list(times)

    def memory(self):
        """(held, reserved, pooled) device bytes."""
        h, r, p = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(_lib.fdm_server_memory(self._s, ctypes.byref(h), ctypes.byref(r), ctypes.byref(p)),
               "fdm_server_memory")
        return h.value, r.value, p.value

    def close(self):
        if self._s:
            _lib.fdm_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
