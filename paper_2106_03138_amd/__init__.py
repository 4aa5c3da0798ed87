"""QRDM on AMD Instinct MI355X: rank-revealing QR with Deviation Maximization
pivoting (Dessole & Marcuzzi, arXiv 2106.03138) and the classical column
pivoting baseline, as hand-written HIP kernels for gfx950 behind the C ABI of
include/qrdm.h.

Python-side API (torch tensors are used for device memory and streams only):

    from paper_2106_03138_amd import qrdm_factor, qrp_factor, device_matrix
    A = device_matrix(numpy_array)          # float64, column-major, on cuda
    out = qrdm_factor(A, tau=0.15, delta=0.9, kmax=64)
    out.rank, out.perm, out.tau_house       # A now holds R and the reflectors
"""
from __future__ import annotations

from ._lib import (PREC_FP64, PREC_MIXED, STOP_MAXNORM, STOP_NONE, STOP_PAPER, QrdmError, load)
from .api import (Batch, BatchPlan, BatchRHS, Factorization, batch_params, batch_size_class, colnorms, device_matrix, dm_step,
                  host_matrix, lstsq, truncate_rank, mlp_adam, mlp_forward, mlp_gradient, mlp_to_params, qrdm_factor,
                  qrp_factor)

__all__ = [
    "PREC_FP64", "PREC_MIXED", "STOP_MAXNORM", "STOP_NONE", "STOP_PAPER", "QrdmError", "load",
    "Factorization", "colnorms", "lstsq", "truncate_rank", "BatchRHS", "device_matrix", "dm_step", "host_matrix", "qrdm_factor", "qrp_factor",
    "Batch", "BatchPlan", "batch_params", "batch_size_class", "mlp_adam", "mlp_forward", "mlp_gradient",
    "mlp_to_params",
]
