"""Pins of the certified DM mode and the Lemma 1 record of the oracle
(oracle/qrdm_oracle.c): eq. (delta_max) and Lemma 1, checked against library
SVDs of the selected columns and against closed forms."""
import numpy as np
import pytest

import oracle
from paper_2106_03138_amd import inputs as I


def _first_block_columns(a, ref):
    """C of the first block: the accepted columns of the input, in order."""
    ks = ref.blocks[0].ks
    return a[:, ref.perm[:ks]], ks


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("certified", [False, True])
def test_lemma1_bound_below_sigma_min(seed, certified):
    """The recorded bound never exceeds sigma_min(C) of the first block
    (library SVD), whether or not the lemma's hypotheses were enforced."""
    rng = np.random.default_rng(seed)
    m, n = 150, 90
    # columns of similar norms with moderate correlation: large DM blocks
    base = rng.standard_normal((m, 6))
    a = np.asfortranarray(rng.standard_normal((m, n)) + 0.3 * base @ rng.standard_normal((6, n)))
    ref = oracle.qrdm(a, tau=0.5, delta=0.9, kmax=32, certified=certified)
    c, ks = _first_block_columns(a, ref)
    smin = np.linalg.svd(c, compute_uv=False)[-1]
    b = ref.blocks[0]
    assert b.sigma_bound <= smin * (1 + 1e-12)
    if certified:
        assert b.sigma_bound > 0.0  # eq. (delta_max) makes Lemma 1 apply
        th = c.T @ c / np.outer(np.linalg.norm(c, axis=0), np.linalg.norm(c, axis=0))
        off = np.abs(th[~np.eye(ks, dtype=bool)])
        assert off.size == 0 or np.max(off) < 0.25 / (b.nL - 1) + 1e-15


def test_orthogonal_columns_closed_form():
    """Theta = I: gamma = 1 and the bound is min_J ||c_j|| = sigma_min(C)."""
    norms = np.geomspace(1.0, 0.2, 20)
    a, _ = I.orthogonal_columns(80, norms, 3)
    ref = oracle.qrdm(a, tau=0.15, delta=0.9, kmax=64, certified=True)
    b = ref.blocks[0]
    assert b.ks == 20
    assert abs(b.gamma - 1.0) < 1e-13
    assert b.sigma_bound == pytest.approx(0.2, rel=1e-13)


def test_single_column_blocks():
    """k_DM = 1 (QRP): every block is one column, gamma = 1 and the bound is
    the column's partial norm, which is |r_ii|."""
    a = I.gaussian(60, 40, 5)
    ref = oracle.qrdm(a, tau=1.0, delta=0.0, kmax=1)
    for i, b in enumerate(ref.blocks[:40]):
        if b.l == 0:
            continue
        assert b.gamma == 1.0
        assert b.sigma_bound == pytest.approx(abs(ref.qr[b.ns, b.ns]), rel=1e-12)


def test_certified_blocks_all_satisfy_the_lemma():
    """In certified mode every block of a full run meets gamma > 1 - tau_J^2
    (positive bound), and blocks are smaller than with the default delta."""
    a = I.half_rank_noise(256, 3)
    cert = oracle.qrdm(a, certified=True)
    dflt = oracle.qrdm(a)
    real = [b for b in cert.blocks if b.l > 0]
    assert all(b.sigma_bound > 0.0 for b in real)
    assert len(real) > len([b for b in dflt.blocks if b.l > 0])
