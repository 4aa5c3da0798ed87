"""Oracle for least squares on top of a pivoted QR (TEST INFRASTRUCTURE ONLY).

With A P = Q R from QRDM (or QRP) and rank r (the stopping criterion of
Section 3.4), column pivoting singles out the basic solution of min ||A x - b||,
the one with r nonzeros (Section 1):
    y = Q_r^T b,  R11 x1 = y[:r],  x = P [x1; 0],
with Q_r the product of the first r reflectors and R11 the leading r x r block
of R.  Written out with explicit loops: the reflectors are applied one at a
time, then row-oriented back substitution.
"""
from __future__ import annotations

import numpy as np


def apply_qt(qr: np.ndarray, tau: np.ndarray, b: np.ndarray, nref: int) -> np.ndarray:
    """Q^T b with Q = H_0 ... H_{nref-1}, H_i = I - tau_i v_i v_i^T, v_i[i] = 1 and
    v_i[i+1:] stored below the diagonal of column i (LAPACK layout)."""
    m = qr.shape[0]
    y = np.array(b, dtype=np.float64, copy=True)
    if y.ndim == 1:
        y = y[:, None]
    for i in range(nref):
        v = np.zeros(m)
        v[i] = 1.0
        v[i + 1:] = qr[i + 1:, i]
        w = tau[i] * (v[i:] @ y[i:, :])
        y[i:, :] -= np.outer(v[i:], w)
    return y


def back_substitute(r: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Solve the upper-triangular system r x = y (k x k, several right-hand sides)."""
    k = r.shape[0]
    x = np.array(y, dtype=np.float64, copy=True)
    for i in range(k - 1, -1, -1):
        s = x[i, :] - r[i, i + 1:k] @ x[i + 1:k, :]
        x[i, :] = s / r[i, i]
    return x


def basic_solution(qr: np.ndarray, tau: np.ndarray, perm: np.ndarray, rank: int, b: np.ndarray) -> np.ndarray:
    """x (n x nrhs) with x[perm[:r]] = R11^{-1} (Q^T b)[:r] and zeros elsewhere."""
    m, n = qr.shape
    bb = np.asarray(b, dtype=np.float64)
    if bb.ndim == 1:
        bb = bb[:, None]
    nrhs = bb.shape[1]
    x = np.zeros((n, nrhs))
    if rank == 0:
        return x
    y = apply_qt(qr, tau, bb, rank)
    x1 = back_substitute(np.triu(qr[:rank, :rank]), y[:rank, :])
    x[np.asarray(perm[:rank], dtype=np.int64), :] = x1
    return x
