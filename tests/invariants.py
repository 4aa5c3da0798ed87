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


def stop_band(qr: np.ndarray, amax: float, eps1: float, nu: float, upto: int, maxnorm: bool = False,
              rtol: float = RTOL, nref: int | None = None) -> tuple[int, int | None]:
    """Where the practical stopping criterion (Section 4) first holds on a
    factorization's exact partial norms, with the rounding noise of two correct
    implementations taken into account.

    For every column j < upto (the rows of R above `upto` must be final), lhs_j =
    sqrt(n - j) * max_{q >= j} ||R[j:, q]|| (MAXNORM: without sqrt(n - j)) against
    rhs = eps1 * amax; slack_j = sqrt(n - j) * nu + rtol * lhs_j (MAXNORM: nu +
    rtol * lhs_j).  Returns (lo, hi): lo = the first j with lhs_j <= rhs + slack_j
    (the test may hold there on another implementation's data), hi = the first j
    with lhs_j < rhs - slack_j (it surely holds), None when no j < upto is that
    clear.  lo = upto when the test cannot hold before upto.
    nref: the number of reflectors of a factorization that stopped early (its
    columns >= nref hold the trailing block in all rows >= nref); None = full."""
    m, n = qr.shape
    upto = min(upto, min(m, n))
    if upto <= 0:
        return upto, None
    if nref is None:
        c2 = suffix_norms2(qr)
    else:
        r = np.array(qr, copy=True)
        for j in range(min(nref, n)):
            r[j + 1:, j] = 0.0
        c2 = np.cumsum((r ** 2)[::-1, :], axis=0)[::-1, :]
    # row j of the suffix norms is zero left of column j (R is upper triangular)
    u = np.sqrt(np.maximum(c2[:upto].max(axis=1), 0.0))
    f = np.ones(upto) if maxnorm else np.sqrt(n - np.arange(upto, dtype=np.float64))
    lhs = f * u
    sl = f * nu + rtol * lhs
    rhs = eps1 * amax
    may, sure = lhs <= rhs + sl, lhs < rhs - sl
    lo = int(np.argmax(may)) if may.any() else upto
    hi = int(np.argmax(sure)) if sure.any() else None
    return lo, hi


def check_dm_replay(qr: np.ndarray, blocks, tau: float, delta: float, kmax: int, amax: float,
                    nu: float = 0.0, rtol: float = RTOL, ctol: float = CTOL) -> dict:
    """Algorithm 1 and the check step of Algorithm 4 replayed at every logged block
    start from the final R alone, for any size and past any low-margin decision.

    blocks: (ns, nL, ks, l, fallback, ...) per record of the DM loop; a record with
    fallback = 1 marks a step at or after the switch to scalar pivoting (the GPU
    logs one, with l = 0, at the switch column).  amax: max column norm of A.
    nu: absolute rounding-noise scale of partial norms (two correct FP64 runs may
    differ by it); rtol / ctol: slack of the norm comparisons (the selection
    compares downdated estimates) and of the cosines.

    For a block at ns with l kept columns K = ns..ns+l-1 (final positions; their
    order is the accepted order J), the candidates S = {q >= ns : u_q >= tau umax}
    with u_q = ||R[ns:, q]|| (orthogonal transformations keep the partial norms
    and cosines of the block's start), in norm order (Section 4) and cut to
    cap = min(k_DM, min(m, n) - ns) entries (eq. candidate_set_limited_by_kDM):
      - the logged |L| is the length of the cut list (up to columns at the
        threshold);
      - every kept column is in the cut list;
      - greedy maximality before K[l-1]: a listed candidate of clearly larger norm
        than K[l-1] that was not kept conflicts (|theta| >= delta) with a kept
        column ahead of it (J is in list order, so had it been accepted it would
        stand before K[l-1] and be kept);
      - without a break (k_s = l): every listed candidate after K[l-1] conflicts
        with a kept column (else the greedy test would have accepted it);
      - with a break (k_s > l): the first listed candidate after K[l-1] free of
        conflicts with K has partial norm below eps_s = tau umax after the l
        reflectors (eq. lenght_check); and every kept column i >= 1 had
        |r_ii| >= eps_s;
      - the switch to scalar pivoting (eq. column_norm_bound_DM, read as
        umax <= n eps amax): no DM block started at or below it, and every
        switch record is at or below it.
    Decisions within the slack are accepted either way.  Returns counts of the
    checks made."""
    m, n = qr.shape
    p = min(m, n)
    c2 = suffix_norms2(qr)
    rr = np.triu(qr[:p, :])
    fb_thr = n * EPS * amax
    out = dict(blocks=0, greedy_checked=0, breaks=0, maximal_no_break=0, switch=None)
    for b in blocks:
        ns, nL, ks, l = int(b[0]), int(b[1]), int(b[2]), int(b[3])
        fallback = len(b) > 4 and bool(b[4])
        if ns >= p:
            continue
        u = np.sqrt(np.maximum(c2[ns, ns:], 0.0))
        umax = u.max()
        if fallback:
            assert umax <= fb_thr * (1 + rtol) + nu, f"switch at {ns}: max partial norm {umax} above n eps amax {fb_thr}"
            if out["switch"] is None:
                out["switch"] = ns
            continue
        if l <= 0:
            continue
        assert umax > fb_thr * (1 - rtol) - nu, f"DM block at {ns}: max partial norm {umax} at the switch level {fb_thr}"
        if ks == 1 and nL == 1:
            continue  # a single-pivot step (k_DM = 1 or one column left): the arg-max is checked by check_blocks
        out["blocks"] += 1
        cap = min(kmax, p - ns)
        thr = tau * umax

        def slack(v):
            return rtol * v + nu

        lo = min(cap, int(np.sum(u >= thr + slack(thr))))
        hi = min(cap, int(np.sum(u >= thr - slack(thr))))
        assert lo <= nL <= hi, f"block at {ns}: |L| = {nL}, the list holds {lo}..{hi}"
        cand = np.nonzero(u >= thr - slack(thr))[0]
        cand = cand[np.argsort(-u[cand], kind="stable")]
        above = np.array([int(np.sum(u > u[c] + slack(u[c]))) for c in cand], dtype=np.int64)  # surely ahead
        ahead = np.array([int(np.sum(u >= u[c] - slack(u[c]))) - 1 for c in cand], dtype=np.int64)  # maybe ahead
        possible = cand[above < cap]                         # may be in the cut list
        sure = set(int(c) for c, a in zip(cand, ahead) if a < cap and u[c] >= thr + slack(thr))
        for i in range(l):
            assert int(np.sum(u > u[i] + slack(u[i]))) < cap, \
                f"block at {ns}: kept column {ns + i} is not among the {cap} largest candidates"
        cols = np.unique(np.concatenate([possible, np.arange(l)]))
        blk = rr[ns:, ns + cols]
        g = blk.T @ blk
        d = np.sqrt(np.diag(g))
        with np.errstate(invalid="ignore", divide="ignore"):
            cos = np.abs(g / np.outer(d, d))
        idx = {int(c): k for k, c in enumerate(cols)}
        ck = [idx[i] for i in range(l)]
        ulast = u[l - 1]
        for c in possible:
            c = int(c)
            if c < l or c not in sure or not u[c] > ulast + slack(ulast):
                continue
            prior = [idx[i] for i in range(l) if u[i] >= u[c] - slack(u[c])]
            assert prior and np.max(cos[idx[c], prior]) >= delta - ctol, \
                f"block at {ns}: candidate {ns + c} conflicts with no accepted column yet was not taken"
            out["greedy_checked"] += 1
        after = [int(c) for c in possible if int(c) >= l and u[int(c)] <= ulast + slack(ulast)]
        eps_s = thr
        for i in range(1, l):
            assert abs(rr[ns + i, ns + i]) >= eps_s * (1 - rtol) - nu, \
                f"block at {ns}: kept column {ns + i} has norm {abs(rr[ns + i, ns + i])} below eps_s {eps_s} (missed break)"
        if ks == l:
            for c in after:
                if c not in sure:
                    continue
                assert np.max(cos[idx[c], ck]) >= delta - ctol, \
                    f"block at {ns}: candidate {ns + c} conflicts with no kept column, yet the block stopped at {l} (not maximal)"
                out["maximal_no_break"] += 1
        else:
            # the break column: the first candidate after K[l-1] free of conflicts
            maybe = []
            for c in after:
                worst = np.max(cos[idx[c], ck])
                if worst >= delta + ctol:
                    continue
                maybe.append(c)
                if worst < delta - ctol and c in sure:
                    break
            assert maybe, f"block at {ns}: a break after {l} columns with no candidate left to break on"
            post = [np.sqrt(max(c2[ns + l, ns + c], 0.0)) if ns + l < p else 0.0 for c in maybe]
            assert min(post) < eps_s * (1 + rtol) + nu, \
                f"block at {ns}: break after {l} columns, but the next accepted column has norm {min(post)} >= eps_s {eps_s}"
            out["breaks"] += 1
    return out
