"""Properties of a finished QRDM factorization that hold at any size, read from
the factors alone (shared by the GPU tests; test infrastructure only).

Orthogonal transformations keep the norms and inner products of the parts of
two columns below a given row.  So for a block of Algorithm 4 that starts at
row/column ns, the partial norm of any column q >= ns when the block was chosen
is ||R[ns:, q]||, and the cosine of two of its columns is the cosine of
R[ns:, p] and R[ns:, q]; both come from the final R, with no replay.  From them:

- Algorithm 1, candidate set: every column of a DM block has partial norm
  >= tau * (largest partial norm), and the block holds a column of largest norm;
- Algorithm 1, greedy pick: the columns of a DM block are pairwise |cos| < delta;
- Algorithm 2 / a single-column step: the pivot has the largest partial norm;
- the practical stopping criterion (Section 4): the recorded rank is the first
  block start where sqrt(n - ns) * max partial norm <= eps_1 * max column norm
  of A, eps_1 = n * eps;
- each reflector H_i = I - tau_i v_i v_i^T (v_i = [1; below the diagonal]) is
  orthogonal: tau_i * ||v_i||^2 = 2, or tau_i = 0 with v_i = e_1.

The decisions were taken on downdated partial norms, which the downdate and
recompute rule keeps within about sqrt(eps) relative of the exact ones, so the
norm comparisons carry a relative slack RTOL and the cosines an absolute CTOL.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps
RTOL = 1e-6
CTOL = 1e-6


def suffix_norms2(qr: np.ndarray) -> np.ndarray:
    """C[i, q] = ||R[i:, q]||^2 over the upper triangle R of qr (rows < min(m, n))."""
    p = min(qr.shape)
    t = np.triu(qr[:p, :]) ** 2
    return np.cumsum(t[::-1, :], axis=0)[::-1, :]


def check_reflectors(qr: np.ndarray, tau: np.ndarray, nref: int, tol: float = 1e-11) -> None:
    low = np.tril(qr[:, :nref], -1)
    s = 1.0 + np.sum(low ** 2, axis=0)
    t = np.asarray(tau[:nref], dtype=np.float64)
    zero = t == 0.0
    assert np.all(np.sum(low[:, zero] ** 2, axis=0) == 0.0), "tau = 0 with a nonzero reflector"
    dev = np.abs(t[~zero] * s[~zero] / 2.0 - 1.0)
    assert dev.size == 0 or np.max(dev) <= tol, f"reflector not orthogonal: {np.max(dev)}"


def check_blocks(qr: np.ndarray, blocks, tau: float, delta: float, nref: int, tail_single: bool = True):
    """blocks: (ns, nL, ks, l, ...) per step of the factorization.  Returns the list
    of block starts checked (in order)."""
    m, n = qr.shape
    c2 = suffix_norms2(qr)
    rr = np.triu(qr[: min(m, n), :])
    starts = []
    end = 0
    for b in blocks:
        ns, l = int(b[0]), int(b[3])
        if l <= 0 or ns >= nref:
            continue
        starts.append((ns, l))
        end = max(end, ns + l)
    if tail_single:
        starts += [(j, 1) for j in range(end, nref)]
    for ns, l in starts:
        pn = np.sqrt(c2[ns, ns:])
        umax = pn.max()
        blk = pn[:l]
        if umax == 0.0:
            continue
        assert blk.max() >= umax * (1 - RTOL), f"block at {ns}: no column of largest norm"
        if l == 1:
            continue
        assert blk.min() >= tau * umax * (1 - RTOL), f"block at {ns}: a column below tau * max"
        b = rr[ns:, ns:ns + l]
        g = b.T @ b
        d = np.sqrt(np.diag(g))
        cos = g / np.outer(d, d)
        np.fill_diagonal(cos, 0.0)
        assert np.max(np.abs(cos)) < delta + CTOL, f"block at {ns}: |cos| = {np.max(np.abs(cos))}"
    return [s for s, _ in starts]


def paper_rule_rank(qr: np.ndarray, a_colnorm_max: float, starts) -> tuple[int, float]:
    """Rank by the practical stopping criterion evaluated at the block starts, and
    the smallest relative margin |lhs / rhs - 1| met at or before it."""
    m, n = qr.shape
    c2 = suffix_norms2(qr)
    rhs = n * EPS * a_colnorm_max
    margin = np.inf
    for ns in sorted(starts):
        lhs = np.sqrt(n - ns) * np.sqrt(c2[ns, ns:].max())
        if rhs > 0:
            margin = min(margin, abs(lhs / rhs - 1.0))
        if lhs <= rhs:
            return ns, margin
    return min(m, n), margin
