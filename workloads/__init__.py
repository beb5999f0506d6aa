"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds Hamiltonians Hp = Q diag(lam) Q^T with a known spectrum and a
known orthogonal eigenbasis.  It holds none of the density-matrix method's
arithmetic: no spectral bounds, no purification, no Fermi-Dirac evaluation.
Both the CPU oracle and the GPU library receive the same arrays from here.
"""
from .gen import (  # noqa: F401
    Workload,
    haar_orthogonal,
    spectrum_gapped_uniform,
    spectrum_bands,
    spectrum_bands_outliers,
    spectrum_uniform,
    make_workload,
    standard_workload,
    serving_requests,
    paper_e1_band,
    paper_e1_matrix,
    paper_e1_rows,
    serving_workload,
    WORKLOADS,
)
