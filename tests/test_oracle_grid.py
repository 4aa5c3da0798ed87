"""Pins of the oracle at the corners of the (tau, delta) grid of Section 5."""
import numpy as np

import oracle
from paper_2106_03138_amd import inputs as I


def test_tau_zero_admits_every_column():
    """tau = 0: every column is a candidate; on orthogonal columns (Theta = I)
    the first block takes min(n, k_DM) of them, in norm order."""
    norms = np.geomspace(1.0, 1e-6, 30)
    a, _ = I.orthogonal_columns(90, norms, 4)
    ref = oracle.qrdm(a, tau=0.0, delta=0.5, kmax=64, stop_rule=oracle.STOP_NONE)
    assert ref.code == 0
    b = ref.blocks[0]
    assert (b.nL, b.ks, b.l) == (30, 30, 30)
    np.testing.assert_allclose(np.abs(np.diag(ref.qr)), norms, rtol=1e-10)
    ref = oracle.qrdm(a, tau=0.0, delta=0.5, kmax=8, stop_rule=oracle.STOP_NONE)
    assert ref.blocks[0].ks == 8


def test_delta_zero_is_column_pivoting():
    """delta = 0: no cosine is below 0, so every block is the arg-max column
    alone and the factorization equals QRP's (Algorithm 2)."""
    a = I.gaussian(70, 50, 6)
    dm = oracle.qrdm(a, tau=0.3, delta=0.0, stop_rule=oracle.STOP_NONE)
    qp = oracle.qrp(a, stop_rule=oracle.STOP_NONE)
    assert all(b.ks == 1 for b in dm.blocks if b.l > 0)
    assert np.array_equal(dm.perm, qp.perm)
    np.testing.assert_allclose(dm.qr, qp.qr, rtol=0, atol=1e-13)


def test_tau_negative_rejected():
    a = I.gaussian(10, 8, 1)
    assert oracle.qrdm(a, tau=-0.1).code == -5
