"""Host-side quality metrics for a pivoted QR (test infrastructure only).

All quantities are the ones the paper evaluates (Section 5):
  sigma_i of A from LAPACK xgejsv (JOBA='A'); the numerical rank n_r = #{sigma_i > eps*n*sigma_1};
  d_i = i-th largest |r_ii| among the first n_r; the ratios d_i/sigma_i and sigma_i(R11)/sigma_i;
plus the backward error ||A P - Q R||_F / ||A||_F and the orthogonality of Q.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import lapack

EPS = np.finfo(np.float64).eps


def r_factor(qr: np.ndarray, nref: int) -> np.ndarray:
    """R with the reflector parts (below the diagonal of the first nref columns) removed.
    Columns >= nref keep all rows >= nref (the untriangularised trailing block)."""
    r = np.array(qr, copy=True)
    m, n = r.shape
    for j in range(min(nref, n)):
        r[j + 1:, j] = 0.0
    return r


def apply_qt(qr: np.ndarray, tau: np.ndarray, x: np.ndarray, nref: int) -> np.ndarray:
    """Q^T x with Q = H_0 ... H_{nref-1}, H_i = I - tau_i v_i v_i^T, v_i from below the diagonal."""
    y = np.array(x, dtype=np.float64, copy=True)
    m = qr.shape[0]
    for i in range(nref):
        v = np.empty(m - i)
        v[0] = 1.0
        v[1:] = qr[i + 1:, i]
        w = tau[i] * (v @ y[i:])
        y[i:] -= np.outer(v, w) if y.ndim == 2 else v * w
    return y


def apply_qt_blocked(qr: np.ndarray, tau: np.ndarray, x: np.ndarray, nref: int) -> np.ndarray:
    """Q^T x (x 2-D) by LAPACK dormqr: the blocked application of the same
    reflectors, for large sizes; apply_qt is the plain definition."""
    y = np.asfortranarray(x, dtype=np.float64)
    if nref <= 0:
        return np.array(y, copy=True)
    v = np.asfortranarray(qr[:, :nref])
    t = np.ascontiguousarray(tau[:nref], dtype=np.float64)
    out, _, info = lapack.dormqr("L", "T", v, t, y, max(1, 64 * y.shape[1]))
    assert info == 0
    return out


def apply_q(qr: np.ndarray, tau: np.ndarray, x: np.ndarray, nref: int) -> np.ndarray:
    """Q x."""
    y = np.array(x, dtype=np.float64, copy=True)
    m = qr.shape[0]
    for i in reversed(range(nref)):
        v = np.empty(m - i)
        v[0] = 1.0
        v[1:] = qr[i + 1:, i]
        w = tau[i] * (v @ y[i:])
        y[i:] -= np.outer(v, w) if y.ndim == 2 else v * w
    return y


def residual(a: np.ndarray, qr: np.ndarray, tau: np.ndarray, perm: np.ndarray, nref: int) -> float:
    """||A P - Q R||_F / ||A||_F (computed as ||Q^T A P - R||_F / ||A||_F)."""
    ap = a[:, perm]
    qtap = apply_qt(qr, tau, ap, nref)
    na = np.linalg.norm(a)
    return float(np.linalg.norm(qtap - r_factor(qr, nref)) / (na if na > 0 else 1.0))


def sampled_residual(a: np.ndarray, qr: np.ndarray, tau: np.ndarray, perm: np.ndarray, nref: int,
                     cols) -> float:
    """Estimate of ||A P - Q R||_F / ||A||_F from the columns `cols` of A P alone:
    sqrt(n / |cols| * sum_j ||Q^T A P e_j - R e_j||^2) / ||A||_F.  Equal to residual()
    when cols lists every column once."""
    cols = np.asarray(cols, dtype=np.int64)
    n = a.shape[1]
    qtap = apply_qt_blocked(qr, tau, a[:, np.asarray(perm)[cols]], nref)
    r = np.array(qr[:, cols], copy=True)
    for c, j in enumerate(cols):
        if j < nref:
            r[j + 1:, c] = 0.0
    na = np.linalg.norm(a)
    est = np.sqrt(n / len(cols) * np.sum((qtap - r) ** 2))
    return float(est / (na if na > 0 else 1.0))


def orthogonality(qr: np.ndarray, tau: np.ndarray, nref: int) -> float:
    """max |Q^T Q - I| over the full m x m Q."""
    m = qr.shape[0]
    q = apply_q(qr, tau, np.eye(m), nref)
    return float(np.max(np.abs(q.T @ q - np.eye(m))))


def singular_values(a: np.ndarray) -> np.ndarray:
    """sigma_i from LAPACK dgejsv with JOBA='A' (Section 5); falls back to dgesdd if the
    Jacobi driver reports a failure."""
    a = np.asfortranarray(a, dtype=np.float64)
    m, n = a.shape
    if m < n:
        a = np.asfortranarray(a.T)
        m, n = n, m
    try:
        out = lapack.dgejsv(a, joba=1, jobu=3, jobv=3)  # joba=1 -> 'A'; no vectors
        sva, work, info = out[0], out[-2], out[-1]
        if info == 0:
            scale = work[0] / work[1] if work[1] != 0 else 1.0
            return np.sort(np.asarray(sva) * scale)[::-1]
    except Exception:  # pragma: no cover - scipy build without dgejsv
        pass
    return np.linalg.svd(a, compute_uv=False)


def numerical_rank(sigma: np.ndarray, n: int) -> int:
    """n_r = #{sigma_i > eps * n * sigma_1} (Section 5)."""
    if len(sigma) == 0 or sigma[0] == 0:
        return 0
    return int(np.sum(sigma > EPS * n * sigma[0]))


def diag_ratios(r: np.ndarray, sigma: np.ndarray, nr: int) -> np.ndarray:
    """d_i / sigma_i, d_i = i-th largest |r_ii| among the first n_r diagonal entries."""
    d = np.sort(np.abs(np.diag(r)[:nr]))[::-1]
    return d / sigma[:nr]


def r11_ratios(r: np.ndarray, sigma: np.ndarray, nr: int) -> np.ndarray:
    """sigma_i(R11) / sigma_i with R11 = R[:n_r, :n_r]."""
    s11 = np.linalg.svd(r[:nr, :nr], compute_uv=False)
    return s11 / sigma[:nr]


def sigma_min_r11(r: np.ndarray, k: int) -> float:
    """sigma_min(R11), R11 = the leading k x k upper triangle of r (LAPACK dgesdd,
    values only)."""
    if k <= 0:
        return 0.0
    from scipy.linalg import svdvals
    return float(svdvals(np.triu(r[:k, :k]), check_finite=False)[-1])


def flops(m: int, n: int, r: int) -> float:
    """Algorithmic flop count of r Householder steps: sum_{s<r} 4 (m-s)(n-s)."""
    s = np.arange(r, dtype=np.float64)
    return float(np.sum(4.0 * (m - s) * (n - s)))
