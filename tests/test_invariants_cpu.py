"""Pins of the size-independent factorization checks (tests/invariants.py) and of
the sampled backward error, on the oracle's own factorizations (CPU only).

The checks read Algorithm 1's candidate and greedy rules, the single-pivot rule
and the practical stopping criterion (Section 4) off the final R; they must hold
on the oracle's factorizations, and each must fail on a factorization with a
planted mistake."""
import numpy as np
import pytest

import invariants as V
import oracle
from oracle import metrics as M
from paper_2106_03138_amd import inputs as I


def _blocks(res):
    return [(b.ns, b.nL, b.ks, b.l) for b in res.blocks]


@pytest.fixture(scope="module")
def geo():
    n = 384
    a = I.from_spectrum(448, n, np.geomspace(1.0, 1e-16, n), 5)
    res = oracle.qrdm(a, tau=0.15, delta=0.9, kmax=32, stop_rule=oracle.STOP_NONE)
    return a, res


def test_invariants_hold_on_oracle(geo):
    a, res = geo
    n = a.shape[1]
    starts = V.check_blocks(res.qr, _blocks(res), 0.15, 0.9, n)
    assert any(b.l > 1 for b in res.blocks)
    V.check_reflectors(res.qr, res.tau, n)
    r, margin = V.paper_rule_rank(res.qr, np.linalg.norm(a, axis=0).max(), starts)
    assert margin > 1e-6
    assert r == res.rank


def test_sampled_residual_matches_full(geo):
    a, res = geo
    n = a.shape[1]
    full = M.residual(a, res.qr, res.tau, res.perm, n)
    # LAPACK's blocked Q^T against the reflector-by-reflector definition
    assert M.sampled_residual(a, res.qr, res.tau, res.perm, n, np.arange(n)) == pytest.approx(full, rel=1e-6)
    x = np.random.default_rng(4).standard_normal((a.shape[0], 7))
    d = M.apply_qt_blocked(res.qr, res.tau, x, n) - M.apply_qt(res.qr, res.tau, x, n)
    assert np.max(np.abs(d)) <= 1e-13 * np.linalg.norm(x)
    assert np.array_equal(M.apply_qt_blocked(res.qr, res.tau, x, 0), x)
    # a planted error x in one sampled column of R is seen at sqrt(n / |S|) x / ||A||_F
    qr = res.qr.copy()
    cols = np.array([3, 50, 200])
    qr[1, 50] += 1e-6
    est = M.sampled_residual(a, qr, res.tau, res.perm, n, cols)
    assert est == pytest.approx(np.sqrt(n / 3) * 1e-6 / np.linalg.norm(a), rel=1e-3)
    assert M.sampled_residual(a, qr, res.tau, res.perm, n, np.array([3, 200])) < 1e-13


def test_planted_column_swap_fails(geo):
    a, res = geo
    n = a.shape[1]
    b = next(b for b in res.blocks if b.l > 1)
    qr = res.qr.copy()
    # a block column that was not the largest, shrunk below tau * max
    c2 = V.suffix_norms2(qr)[b.ns, b.ns:b.ns + b.l]
    j = b.ns + int(np.argmin(c2))
    qr[:, j] *= 0.1
    with pytest.raises(AssertionError, match="tau"):
        V.check_blocks(qr, _blocks(res), 0.15, 0.9, n, tail_single=False)


def test_planted_single_pivot_fails(geo):
    a, res = geo
    n = a.shape[1]
    qr = res.qr.copy()
    j = n - 40  # a single-pivot step of the noise-level tail
    qr[:, [j, j + 1]] = qr[:, [j + 1, j]]
    qr[j + 1, j] = 0.0
    qr[j, j] *= 1e-3
    with pytest.raises(AssertionError, match="largest norm"):
        V.check_blocks(qr, _blocks(res), 0.15, 0.9, n)


def test_planted_parallel_pair_fails():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((60, 8))
    a[:, 0] *= 3.0
    a[:, 1] = a[:, 0] * 0.99 + 1e-3 * rng.standard_normal(60)
    # an unpivoted R of [a_0 a_1 ...]: a block that claims the parallel pair
    r = np.zeros((60, 8))
    r[:8] = np.linalg.qr(a, mode="r")
    with pytest.raises(AssertionError, match="cos"):
        V.check_blocks(r, [(0, 2, 2, 2)], 0.15, 0.9, 8, tail_single=False)


def test_planted_reflector_fails(geo):
    a, res = geo
    n = a.shape[1]
    tau = res.tau.copy()
    tau[7] *= 1 + 1e-8
    with pytest.raises(AssertionError, match="orthogonal"):
        V.check_reflectors(res.qr, tau, n)


# ------------------------------------------- Algorithm 1 replayed from R alone
def _log(res):
    return [(b.ns, b.nL, b.ks, b.l, b.fallback) for b in res.blocks]


def _case(name):
    if name == "geo":
        return I.from_spectrum(448, 384, np.geomspace(1.0, 1e-16, 384), 5), dict(tau=0.15, delta=0.9, kmax=32)
    if name == "gauss":
        return I.gaussian(300, 200, 3), dict(tau=0.15, delta=0.9, kmax=32)
    if name == "rank64":
        return I.small_rank64(1), dict(tau=0.9, delta=0.9, kmax=32)
    if name == "paired":
        return I.paired_columns(200, 40, 0.95, 4), dict(tau=0.15, delta=0.9, kmax=32)
    raise KeyError(name)


def _replay(a, res, kw):
    amax = np.linalg.norm(a, axis=0).max()
    nu = 4 * V.EPS * np.linalg.norm(a)
    return V.check_dm_replay(res.qr, _log(res), kw["tau"], kw["delta"], kw["kmax"], amax, nu)


@pytest.mark.parametrize("name", ["geo", "gauss", "rank64", "paired"])
def test_replay_holds_on_oracle(name):
    a, kw = _case(name)
    res = oracle.qrdm(a, stop_rule=oracle.STOP_NONE, **kw)
    out = _replay(a, res, kw)
    assert out["blocks"] > 0
    if name == "paired":  # candidates rejected by the cosine test
        assert out["greedy_checked"] + out["maximal_no_break"] > 0
    if name in ("geo", "rank64"):
        assert out["breaks"] > 0 and out["switch"] is not None


@pytest.mark.parametrize("plant,name,msg", [
    (oracle.PLANT_SINGLE, "gauss", "not maximal"),        # a run of single pivots
    (oracle.PLANT_TRUNC, "gauss", "break after"),          # blocks cut short without the break test
    (oracle.PLANT_ACCEPT, "paired", "cos"),                # a block with a conflicting pair
    (oracle.PLANT_REJECT, "gauss", "not maximal"),         # a conflict-free candidate dropped
    (oracle.PLANT_NOBREAK, "rank64", "missed break"),      # the length check of Algorithm 4 ignored
    (oracle.PLANT_FBSCALE, "geo", "switch level"),         # the scalar-pivoting switch at eps, not n eps
])
def test_replay_catches_planted_mistakes(plant, name, msg):
    a, kw = _case(name)
    res = oracle.qrdm(a, stop_rule=oracle.STOP_NONE, plant=plant, **kw)
    with pytest.raises(AssertionError, match=msg):
        V.check_blocks(res.qr, _log(res), kw["tau"], kw["delta"], a.shape[1], tail_single=False)
        _replay(a, res, kw)


# ------------------------------------------------ the rank's noise band, sigma_min(R11)
def _band(res, a, n, rule=oracle.STOP_PAPER, eps1=None, nref=None, upto=None):
    amax = np.linalg.norm(a, axis=0).max()
    nu = 4 * V.EPS * np.linalg.norm(a)
    e1 = n * V.EPS if eps1 is None else eps1
    p = min(a.shape)
    return V.stop_band(res.qr, amax, e1, nu, p if upto is None else upto, maxnorm=(rule == oracle.STOP_MAXNORM),
                       nref=nref)


def test_stop_band_holds_the_rank_of_the_oracle_and_of_a_perturbed_run(geo):
    """The oracle's rank lies in its own band, and so does the rank of a second
    run on A perturbed at the rounding level (a stand-in for another correct
    implementation); the band is a few columns wide on a geometric spectrum."""
    a, res = geo
    n = a.shape[1]
    lo, hi = _band(res, a, n)
    assert hi is not None and lo <= res.rank <= hi
    assert hi - lo <= 60
    pert = a * (1 + 2 * V.EPS * np.random.default_rng(7).standard_normal(a.shape))
    r2 = oracle.qrdm(pert, tau=0.15, delta=0.9, kmax=32, stop_rule=oracle.STOP_NONE)
    assert lo <= r2.rank <= hi, (lo, hi, r2.rank)


def test_stop_band_rejects_a_rank_from_the_wrong_rule(geo):
    """Planted mistake: the rank of the eps sqrt(n) variant (a rule the paper
    calls less accurate) falls outside the band of eps n."""
    a, res = geo
    n = a.shape[1]
    lo, hi = _band(res, a, n)
    wrong = oracle.qrdm(a, tau=0.15, delta=0.9, kmax=32, stop_rule=oracle.STOP_NONE, eps1_scale=np.sqrt(n))
    assert not (lo <= wrong.rank <= hi), (lo, hi, wrong.rank)


def test_stop_band_of_stopped_runs():
    """A run that stopped early keeps the trailing block in its columns >= rank:
    the band reads it (nref).  On the gapped 256^2 spectrum (sigma 1e-3 -> 1e-15
    at n_r = 64) the MAXNORM rule's band is the single column 64; the PAPER rule
    compares sqrt(n - j) max ||c|| with eps n max ||a_j||, and past the gap both
    sides are at the noise level, so its band starts after n_r (the rule never
    fires before the numerical rank) and has no clear end before the stop."""
    a = I.small_rank64(1)
    n = a.shape[1]
    res = oracle.qrdm(a, tau=0.9, delta=0.9, kmax=32, stop_rule=oracle.STOP_MAXNORM)
    lo, hi = _band(res, a, n, rule=oracle.STOP_MAXNORM, nref=res.rank, upto=res.rank + 1)
    assert res.rank == 64 and lo == 64 and hi == 64, (lo, hi, res.rank)
    res = oracle.qrdm(a, tau=0.9, delta=0.9, kmax=32, stop_rule=oracle.STOP_PAPER)
    lo, hi = _band(res, a, n, nref=res.rank, upto=res.rank + 1)
    assert 64 < lo <= res.rank and hi is None, (lo, hi, res.rank)
    # without nref the untriangularised block would be cut by triu: a smaller
    # partial norm, and a band that starts earlier than the true one
    res = oracle.qrdm(a, tau=0.9, delta=0.9, kmax=32, stop_rule=oracle.STOP_PAPER)
    lo_bad, _ = _band(res, a, n, upto=res.rank + 1)
    lo_ok, _ = _band(res, a, n, nref=res.rank, upto=res.rank + 1)
    assert lo_bad <= lo_ok


def test_sigma_min_r11_closed_forms():
    """sigma_min of the leading block: a diagonal R (orthogonal columns, so the
    singular values are the |r_ii|), and 1/||R11^{-1}||_2 by explicit inversion."""
    r = np.zeros((9, 7))
    d = np.array([5.0, -3.0, 2.0, 0.5, -0.25, 4.0, 1.0])
    r[np.arange(7), np.arange(7)] = d
    r[5:, 0] = 1.0  # reflector storage below the diagonal is ignored
    assert M.sigma_min_r11(r, 5) == pytest.approx(0.25, rel=1e-15)
    rng = np.random.default_rng(3)
    t = np.triu(rng.standard_normal((40, 40))) + 5 * np.eye(40)
    inv = np.linalg.inv(t[:30, :30])
    assert M.sigma_min_r11(t, 30) == pytest.approx(1.0 / np.linalg.norm(inv, 2), rel=1e-12)
    assert M.sigma_min_r11(t, 0) == 0.0
