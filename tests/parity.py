"""Comparison of a GPU factorization with the oracle's (shared by the GPU tests).

Decisions (arg-max, candidate order, tau threshold, |theta| < delta, the panel
break, the stopping test) must agree exactly up to the first block where the
oracle records a decision margin below ETA (relative); beyond it two correct
FP64 implementations may differ.  Floating-point results are compared
normwise: two Householder QRs with different summation orders differ by
O(eps ||A||).
"""
import numpy as np

from oracle import metrics as M

EPS = np.finfo(np.float64).eps
ETA = 1e-10


def compare(a, ref, qr, tau, perm, rank, blocks, tol_scale=10.0, check_blocks=True, full=False, residual_cols=None,
            norm2=None):
    """full: the factorization ran to min(m, n) reflectors (stop rule NONE).
    residual_cols: estimate the backward error from these columns of AP only (for
    sizes where applying Q^T to all of AP is too slow on the host).
    norm2: ||A||_2 when known by construction (an SVD of a large A is slow)."""
    m, n = a.shape
    k = ref.first_low_margin_block(ETA)
    ns_cut = ref.blocks[k].ns if k < len(ref.blocks) else min(m, n)
    # the oracle also logs the stopping step (l = 0) and takes the scalar-pivoting
    # steps of eq. (column_norm_bound_DM) in its own loop; the GPU's log holds the
    # DM loop's blocks and, at the switch, one hand-over record (fallback, l = 0)
    real = [b for b in ref.blocks[:k] if b.l > 0 and not b.fallback]
    if check_blocks:
        dm = [g for g in blocks if g[3] > 0]
        for i, rb in enumerate(real):
            assert i < len(dm), f"GPU log shorter than oracle at block {i}"
            g = dm[i]
            assert (g[0], g[1], g[2], g[3]) == (rb.ns, rb.nL, rb.ks, rb.l), f"block {i}: gpu {g} oracle {(rb.ns, rb.nL, rb.ks, rb.l)}"
        fb_ref = next((b.ns for b in ref.blocks[:k] if b.fallback), None)
        if fb_ref is not None:
            hand = [g[0] for g in blocks if len(g) > 4 and g[4]]
            assert hand == [fb_ref], f"switch to scalar pivoting: gpu {hand} oracle {fb_ref}"
    assert np.array_equal(perm[:ns_cut], ref.perm[:ns_cut])
    if k == len(ref.blocks):
        assert np.array_equal(perm, ref.perm)
        assert rank == ref.rank
    nref = min(m, n) if (full or rank >= min(m, n)) else rank
    # backward error of the GPU factorization itself
    if residual_cols is None:
        assert M.residual(a, qr, tau, perm, nref) <= 1e-13
    else:
        assert M.sampled_residual(a, qr, tau, perm, nref, residual_cols) <= 1e-13
    # R agrees normwise with the oracle's on the common prefix
    na = np.linalg.norm(a, 2) if norm2 is None else norm2
    p = min(ns_cut, nref)
    if p == 0:
        return
    # rows of R for the common prefix, columns aligned by original column index
    rg = np.triu(qr[:p, :])[:, np.argsort(perm)]
    ro = np.triu(ref.qr[:p, :])[:, np.argsort(ref.perm)]
    dr = np.abs(rg - ro)
    assert np.max(dr) <= tol_scale * n * EPS * na, np.max(dr)
    # R diagonal: relative where large, absolute where small
    d_g, d_o = np.abs(np.diag(qr)[:p]), np.abs(np.diag(ref.qr)[:p])
    big = d_o >= 1e-3 * na
    if np.any(big):
        assert np.max(np.abs(d_g[big] - d_o[big]) / d_o[big]) <= 1e-12
    assert np.max(np.abs(d_g - d_o)) <= tol_scale * n * EPS * na
