"""Pins of the post-hoc rank truncation oracle (oracle/truncate.py)."""
import numpy as np

import oracle
from oracle import learned as Lr
from oracle import truncate as Tr
from paper_2106_03138_amd import inputs as I


def test_diagonal_by_hand():
    d = np.diag([4.0, -2.0, 1e-3, 3e-15, 1.0, 0.0])
    # threshold 6 * 2^-52 * 4 = 5.3e-15: the first entry at or below it is index 3
    assert Tr.truncated_rank(d, 6) == 3
    assert Tr.truncated_rank(d, 2) == 2            # never above the given rank
    assert Tr.truncated_rank(d, 6, eps1_scale=1.0) == 5  # threshold 8.9e-16 keeps 3e-15
    assert Tr.truncated_rank(d, -1) == -1
    assert Tr.truncated_rank(np.zeros((3, 3)), 3) == 0
    nan = d.copy()
    nan[1, 1] = np.nan
    assert Tr.truncated_rank(nan, 6) == 1


def test_gap_below_the_threshold_gives_the_numerical_rank():
    """The 256 x 256 matrix with 64 singular values in [1e-3, 1] and the rest at
    1e-15: the stopping criterion (eps n) overestimates the rank, the truncated
    rank equals n_r = #{sigma_i > eps n sigma_1} = 64 of the prescribed spectrum."""
    a = I.small_rank64(1)
    sigma = np.concatenate([np.geomspace(1.0, 1e-3, 64), np.full(192, 1e-15)])
    nr = Lr.numerical_rank(sigma, 256)
    assert nr == 64
    ref = oracle.qrdm(a, tau=0.9, delta=0.9, kmax=32)
    assert ref.rank > nr
    assert Tr.truncated_rank(ref.qr, ref.rank) == nr
    full = oracle.qrdm(a, stop_rule=oracle.STOP_NONE)
    assert Tr.truncated_rank(full.qr, full.rank) == nr


def test_full_rank_keeps_everything():
    a = I.gaussian(80, 50, 2)
    ref = oracle.qrdm(a)
    assert ref.rank == 50 and Tr.truncated_rank(ref.qr, ref.rank) == 50


def test_gapped_spectra_match_the_numerical_rank():
    """sigma geometric from 1 to 1e-6 over r values, then 1e-18: a gap around
    the threshold eps n sigma_1 that the truncation must land in exactly, for
    the full factorization and for the early-stopped one."""
    for seed, (m, n, r) in enumerate([(160, 120, 70), (230, 200, 31), (90, 90, 89)]):
        sig = np.concatenate([np.geomspace(1.0, 1e-6, r), np.full(n - r, 1e-18)])
        assert Lr.numerical_rank(sig, n) == r
        a = I.from_spectrum(m, n, sig, seed + 5)
        full = oracle.qrdm(a, stop_rule=oracle.STOP_NONE)
        assert Tr.truncated_rank(full.qr, full.rank) == r
        early = oracle.qrdm(a)
        assert Tr.truncated_rank(early.qr, early.rank) == r
