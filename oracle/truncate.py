"""Oracle for the post-hoc rank truncation (TEST INFRASTRUCTURE ONLY).

Section 5 observes that when the stopping criterion overestimates the numerical
rank, the diagonal of R still shows the gap of the singular values, so an
application can truncate R afterwards.  The rule written out here: with
eps_1 = scale * eps (scale = n unless given, eps = 2^-52, the threshold of eq.
(practical stopping criterion), choice (1)), the truncated rank is the first
index i < rank with |r_ii| <= eps_1 |r_00| (a NaN entry counts as small), or
rank if there is none; it keeps R11 a leading block, as the basic solution
needs.  |r_00| is the largest column norm of A, within a factor sqrt(n) of
sigma_1.
"""
from __future__ import annotations

import numpy as np

EPS = 2.0 ** -52


def truncated_rank(qr: np.ndarray, rank: int, eps1_scale: float = 0.0) -> int:
    m, n = qr.shape
    if rank < 0:
        return rank
    r = min(rank, m, n)
    if r == 0:
        return 0
    scale = eps1_scale if eps1_scale > 0 else float(n)
    thr = scale * EPS * abs(qr[0, 0])
    for i in range(r):
        if not abs(qr[i, i]) > thr:
            return i
    return r
