"""Comparison of a GPU factorization with the oracle's (shared by the GPU tests).

Decisions (arg-max, candidate order, tau threshold, |theta| < delta, the panel
break, the stopping test) must agree exactly up to the first block where the
oracle records a decision margin below ETA (relative); beyond it two correct
FP64 implementations may differ.  Floating-point results are compared
normwise: two Householder QRs with different summation orders differ by
O(eps ||A||); the R diagonal also entrywise (relative 1e-12 where it is at
least 1e-3 ||A||_2, above a floor of DIAG_FLOOR eps ||A||_2).

The rank (the practical stopping criterion of Section 4) is compared exactly
when the oracle took no low-margin decision.  Otherwise the GPU's rank must lie
in the oracle's noise band of the stopping test (invariants.stop_band): not
before the first column where the test can hold within the rounding noise NU
of the oracle's exact partial norms, and not after the first column where it
surely holds, plus one block when the band lies in the DM part of the
factorization (the GPU tests the rule at its own block starts, which differ
from the oracle's past the first low-margin decision).
"""
import numpy as np

import invariants as V
from oracle import metrics as M

EPS = np.finfo(np.float64).eps
ETA = 1e-10
NU_SCALE = 4.0  # noise of partial norms: NU_SCALE * eps * ||A||_F (the oracle's margin floor)
# Two FP64 Householder QRs of one matrix with one column order differ on the R
# diagonal by a few eps ||A||_2 (LAPACK's dgeqrf against a blocked Householder
# QR, on the 8192^2 Gaussian matrix: 5 eps ||A||_2, 4.4e-13 relative on its
# smallest entries), so the relative check of large diagonal entries has this
# floor, in units of eps ||A||_2; the normwise bound is 10 n eps ||A||_2.
DIAG_FLOOR = 32.0
STOP_PAPER, STOP_MAXNORM, STOP_NONE = 0, 1, 2


def compare(a, ref, qr, tau, perm, rank, blocks, tol_scale=10.0, check_blocks=True, full=False, residual_cols=None,
            norm2=None, stop_rule=STOP_PAPER, eps1=None, kmax=128, sigma=None):
    """full: the factorization ran to min(m, n) reflectors (stop rule NONE).
    residual_cols: estimate the backward error from these columns of AP only (for
    sizes where applying Q^T to all of AP is too slow on the host).
    norm2: ||A||_2 when known by construction (an SVD of a large A is slow).
    stop_rule, eps1 (default n eps), kmax: the run's stopping rule and block size.
    sigma: singular values of A (by construction) to compare sigma_min(R11) at the
    numerical rank n_r = #{sigma_i > eps n sigma_1}.
    Returns what was compared: ns_cut (the exact-prefix length), the rank band, and
    sigma_min(R11) / sigma_{n_r} of both factorizations when sigma is given."""
    m, n = a.shape
    p = min(m, n)
    out = {}
    k = ref.first_low_margin_block(ETA)
    ns_cut = ref.blocks[k].ns if k < len(ref.blocks) else p
    out["ns_cut"] = ns_cut
    if k < len(ref.blocks):  # which decision ended the exact prefix
        b = ref.blocks[k]
        names = ["m_order", "m_thr", "m_cos", "m_break", "m_stop", "m_fb", "m_recomp"]
        out["cut_by"] = min(names, key=lambda f: getattr(b, f))
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
    # ---- rank
    amax = float(np.linalg.norm(a, axis=0).max()) if p > 0 else 0.0
    nu = NU_SCALE * EPS * float(np.linalg.norm(a))
    e1 = n * EPS if eps1 is None else eps1
    if k == len(ref.blocks):
        assert np.array_equal(perm, ref.perm)
        assert rank == ref.rank, (rank, ref.rank)
        out["rank_band"] = (ref.rank, ref.rank)
    else:
        upto = p if (full or stop_rule == STOP_NONE) else ref.rank
        lo, hi = V.stop_band(ref.qr, amax, e1, nu, upto, maxnorm=(stop_rule == STOP_MAXNORM),
                             nref=None if upto == p else ref.rank)
        switch = next((b.ns for b in ref.blocks if b.fallback), None)
        slack = 0 if (switch is not None and lo >= switch) else max(kmax - 1, 0)
        out["rank_band"] = (lo, None if hi is None else hi + slack)
        assert lo <= rank, f"rank {rank} before the oracle's noise band [{lo}, {hi}] (oracle rank {ref.rank})"
        if hi is not None:
            assert rank <= hi + slack, \
                f"rank {rank} after the oracle's noise band [{lo}, {hi} + {slack}] (oracle rank {ref.rank})"
    nref = p if (full or rank >= p) else rank
    # backward error of the GPU factorization itself
    if residual_cols is None:
        assert M.residual(a, qr, tau, perm, nref) <= 1e-13
    else:
        assert M.sampled_residual(a, qr, tau, perm, nref, residual_cols) <= 1e-13
    # R agrees normwise with the oracle's on the common prefix
    na = np.linalg.norm(a, 2) if norm2 is None else norm2
    pc = min(ns_cut, nref)
    if pc > 0:
        # rows of R for the common prefix, columns aligned by original column index
        rg = np.triu(qr[:pc, :])[:, np.argsort(perm)]
        ro = np.triu(ref.qr[:pc, :])[:, np.argsort(ref.perm)]
        dr = np.abs(rg - ro)
        assert np.max(dr) <= tol_scale * n * EPS * na, np.max(dr)
        # R diagonal: relative 1e-12 where large, with a floor of DIAG_FLOOR eps ||A||_2
        d_g, d_o = np.abs(np.diag(qr)[:pc]), np.abs(np.diag(ref.qr)[:pc])
        big = d_o >= 1e-3 * na
        if np.any(big):
            dev = np.abs(d_g[big] - d_o[big])
            tol = np.maximum(1e-12 * d_o[big], DIAG_FLOOR * EPS * na)
            out["diag_rel"] = float(np.max(dev / d_o[big]))
            out["diag_eps"] = float(np.max(dev) / (EPS * na))  # in units of eps ||A||_2
            q = int(np.argmax(dev / tol))
            w = int(np.flatnonzero(big)[q])
            assert dev[q] <= tol[q], f"R diagonal {w}: {d_g[w]!r} vs {d_o[w]!r} ({dev[q] / (EPS * na):.1f} eps ||A||)"
        assert np.max(np.abs(d_g - d_o)) <= tol_scale * n * EPS * na
    # ---- sigma_min(R11) / sigma_r(A) at the numerical rank
    if sigma is not None:
        nr = M.numerical_rank(np.asarray(sigma), n)
        r_o = p if (full or ref.rank >= p) else ref.rank
        if 0 < nr <= min(nref, r_o):
            s_g = M.sigma_min_r11(qr, nr)
            s_o = M.sigma_min_r11(ref.qr, nr)
            out["n_r"] = nr
            out["smin_ratio"] = (s_g / sigma[nr - 1], s_o / sigma[nr - 1])
            if ns_cut >= nr:  # the same columns in both R11
                tol = 1e-12 * s_o if s_o >= 1e-3 * na else tol_scale * n * EPS * na
                assert abs(s_g - s_o) <= tol, (s_g, s_o, tol)
    return out
