"""Stop-rule and rank variants on the GPU against the oracle: the stopping
criterion with eps_1 = eps sqrt(n) (eq. practical stopping criterion, choice
2), column pivoting (QRP) with the same stopping criterion as QRDM, and the
post-hoc truncation of the rank on the diagonal of R (Section 5)."""
import numpy as np
import pytest

import oracle
from oracle import learned as Lr
from oracle import truncate as Tr
from paper_2106_03138_amd import inputs as I
from parity import EPS, compare

pytestmark = pytest.mark.gpu


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


@pytest.mark.parametrize("kind", ["rank64", "half_rank_512", "gapped"])
def test_eps_sqrt_n_stop_matches_oracle(kind):
    Q = _gpu()
    if kind == "rank64":
        a = I.small_rank64(3)
    elif kind == "half_rank_512":
        a = I.half_rank_noise(512, 1)
    else:
        a = I.from_spectrum(300, 240, np.concatenate([np.geomspace(1, 1e-6, 100), np.full(140, 1e-18)]), 2)
    n = a.shape[1]
    ref = oracle.qrdm(a, eps1_scale=np.sqrt(n))
    A = Q.device_matrix(a)
    out = Q.qrdm_factor(A, eps1_scale=float(np.sqrt(n)), log=True)
    compare(a, ref, Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out.blocks,
            eps1=float(np.sqrt(n)) * EPS, kmax=64)


@pytest.mark.parametrize("rule", [oracle.STOP_PAPER, oracle.STOP_MAXNORM])
def test_qrp_with_the_qrdm_stopping_criterion(rule):
    """Column pivoting stops by the same criterion as QRDM (the comparison the
    paper leaves for future work): same rank and pivots as the oracle."""
    Q = _gpu()
    for a in (I.small_rank64(5), I.half_rank_noise(384, 2)):
        ref = oracle.qrp(a, stop_rule=rule)
        A = Q.device_matrix(a)
        out = Q.qrp_factor(A, stop_rule=rule)
        compare(a, ref, Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, [],
                check_blocks=False, stop_rule=rule, kmax=1)


def test_truncation_recovers_the_numerical_rank_single():
    """The stopping criterion overestimates the rank of the 256 x 256 rank-64
    matrix; truncation on the GPU's R gives n_r = 64, as the oracle's does."""
    Q = _gpu()
    a = I.small_rank64(1)
    sigma = np.concatenate([np.geomspace(1.0, 1e-3, 64), np.full(192, 1e-15)])
    nr = Lr.numerical_rank(sigma, 256)
    for kw in (dict(tau=0.9, delta=0.9, kmax=32), dict(stop_rule=oracle.STOP_NONE)):
        A = Q.device_matrix(a)
        out = Q.qrdm_factor(A, **kw)
        assert out.rank >= nr
        assert Q.truncate_rank(A, out.rank) == nr
        ref = oracle.qrdm(a, **kw)
        assert Tr.truncated_rank(ref.qr, ref.rank) == nr


def test_truncation_edge_cases():
    import torch
    Q = _gpu()
    d = np.diag([4.0, -2.0, 1e-3, 3e-15, 1.0, 0.0])
    A = Q.device_matrix(d)
    for rank, scale in [(6, 0.0), (2, 0.0), (6, 1.0), (-1, 0.0), (0, 0.0), (99, 0.0)]:
        assert Q.truncate_rank(A, rank, scale) == Tr.truncated_rank(d, rank, scale), (rank, scale)
    d[1, 1] = np.nan
    assert Q.truncate_rank(Q.device_matrix(d), 6) == Tr.truncated_rank(d, 6) == 1
    z = Q.device_matrix(np.zeros((0, 4)))
    assert Q.truncate_rank(z, 3) == 0
    assert Q.truncate_rank(Q.device_matrix(np.zeros((5, 3))), 3) == 0
    torch.cuda.synchronize()


def test_truncation_batched():
    """Per matrix of an uneven batch: the truncated rank of the GPU's R equals
    the oracle's, except where the deciding diagonal entry lies within a factor
    100 of the threshold, where rounding of the factorization decides."""
    Q = _gpu()
    shapes = I.batch_shapes(48, seed=41, mmin=8, mmax=220, nmin=1)
    seqs = np.random.SeedSequence(41).spawn(len(shapes))
    mats = [I.batch_matrix(m, n, r, s) for (m, n, r), s in zip(shapes, seqs)]
    mats += [I.from_spectrum(200, 150, np.concatenate([np.geomspace(1, 1e-5, 60), np.full(90, 1e-19)]), 9),
             np.zeros((7, 3), order="F")]
    bt = Q.Batch([a.shape for a in mats])
    bt.load(mats)
    plan = Q.BatchPlan(bt)
    plan.factor()
    tr = plan.truncate_rank().cpu().numpy()
    rank = bt.rank.cpu().numpy()
    exact = 0
    for i, a in enumerate(mats):
        assert 0 <= tr[i] <= rank[i], i
        # the rule applied to the GPU's own R, written out here
        qr = bt.matrix(i)
        r = min(int(rank[i]), *qr.shape)
        d = np.abs(np.diag(qr)[:r])
        small = np.nonzero(~(d > a.shape[1] * Tr.EPS * (d[0] if r else 0.0)))[0]
        assert tr[i] == (small[0] if len(small) else r), i
        ref = oracle.qrdm(a)
        to = Tr.truncated_rank(ref.qr, ref.rank)
        if tr[i] == to:
            exact += 1
            continue
        thr = a.shape[1] * Tr.EPS * abs(ref.qr[0, 0])
        k = min(tr[i], to)
        assert abs(ref.qr[k, k]) <= 100 * thr and abs(ref.qr[k, k]) >= thr / 100, (i, tr[i], to)
    assert tr[-2] == 60 and tr[-1] == 0
    print(f"{exact} of {len(mats)} truncated ranks equal to the oracle's")
    plan.close()
