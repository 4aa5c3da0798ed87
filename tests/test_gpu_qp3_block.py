"""The QP3 column loop (Algorithm 2 blocked like xgeqp3) runs one block of up
to nb pivots per launch; the per-step kernels remain selectable
(QRDM_QP3_STEPS=1).  Both carry out the same arithmetic in the same order, so
pivots and rank must agree exactly and R / tau to rounding of the contraction
(1e-13 relative); these comparisons switch the register-resident tail off
(QRDM_QP3_TAIL=0).  The block kernel holds its columns in LDS when they fit
(2048 rows at most) and reads them from memory otherwise: tall_2200x400
starts in the second mode and ends in the first.  The block path is also
checked against the oracle.

Once the trailing block fits in the registers of the grid (at most 2048 rows
and 8 columns per workgroup), the loop hands every remaining step to one
launch of the tail kernel (unblocked, one grid barrier per step): from the
start on matrices of at most 2048 rows and columns, after some block launches
on taller ones (the hand-over finishes the block's last reflector and its
flagged norms, or a stop inside the block); wide_150x3000 never fits and runs
on block launches throughout.  It is checked against the oracle on the same
cases."""
import numpy as np
import pytest

import oracle
from paper_2106_03138_amd import inputs as I
from parity import compare

pytestmark = pytest.mark.gpu


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


def _graded(m, n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    return a * 10.0 ** (-12.0 * ((np.arange(n) * 7) % n) / n)


CASES = {
    "tall_700x300": lambda: np.random.default_rng(11).standard_normal((700, 300)),
    "wide_200x500": lambda: np.random.default_rng(12).standard_normal((200, 500)),
    "wide_150x3000": lambda: np.random.default_rng(16).standard_normal((150, 3000)),
    "tall_2200x400": lambda: np.random.default_rng(17).standard_normal((2200, 400)),
    "half_rank_384": lambda: I.half_rank_noise(384, 2),
    "graded_600x200": lambda: _graded(600, 200, 13),
    "rank64_256": lambda: I.small_rank64(5),
    "one_column": lambda: np.random.default_rng(14).standard_normal((90, 1)),
    "one_row": lambda: np.random.default_rng(15).standard_normal((1, 70)),
    "zero_40x30": lambda: np.zeros((40, 30)),
}


def _run(Q, a, steps, monkeypatch, tail=False, **kw):
    if steps:
        monkeypatch.setenv("QRDM_QP3_STEPS", "1")
    else:
        monkeypatch.delenv("QRDM_QP3_STEPS", raising=False)
    if tail:
        monkeypatch.delenv("QRDM_QP3_TAIL", raising=False)
    else:
        monkeypatch.setenv("QRDM_QP3_TAIL", "0")
    A = Q.device_matrix(a)
    out = Q.qrp_factor(A, **kw)
    return Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out.stats


def _same(x, y, scale):
    assert np.array_equal(x[2], y[2]), "pivots differ"
    assert x[3] == y[3], "rank differs"
    tol = 1e-13 * max(scale, 1e-300)
    np.testing.assert_allclose(x[0], y[0], rtol=0, atol=tol)
    np.testing.assert_allclose(x[1], y[1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("nb,rule", [(32, oracle.STOP_PAPER), (64, oracle.STOP_NONE), (7, oracle.STOP_MAXNORM)])
def test_block_kernel_matches_per_step_kernels(name, nb, rule, monkeypatch):
    Q = _gpu()
    a = CASES[name]()
    print(f"case {name} nb {nb} rule {rule}", flush=True)
    x = _run(Q, a, True, monkeypatch, nb=nb, stop_rule=rule)
    y = _run(Q, a, False, monkeypatch, nb=nb, stop_rule=rule)
    _same(x, y, float(np.abs(a).max()) if a.size else 1.0)
    assert x[4]["nrecompute"] == y[4]["nrecompute"]


@pytest.mark.parametrize("name", ["tall_700x300", "half_rank_384", "graded_600x200"])
def test_block_kernel_matches_oracle(name, monkeypatch):
    Q = _gpu()
    a = CASES[name]()
    ref = oracle.qrp(a)
    R, tau, perm, rank, _ = _run(Q, a, False, monkeypatch)
    compare(a, ref, R, tau, perm, rank, [], check_blocks=False, kmax=1)


def test_qrdm_continuation_block_vs_steps(monkeypatch):
    """QRDM switches to the QP3 loop once the partial norms reach the noise
    level (geometric spectrum): the continuation agrees between the two paths."""
    Q = _gpu()
    n = 768
    a = I.from_spectrum(n, n, np.geomspace(1, 1e-16, n), 2)
    res = []
    monkeypatch.setenv("QRDM_QP3_TAIL", "0")
    for steps in (True, False):
        if steps:
            monkeypatch.setenv("QRDM_QP3_STEPS", "1")
        else:
            monkeypatch.delenv("QRDM_QP3_STEPS", raising=False)
        A = Q.device_matrix(a)
        out = Q.qrdm_factor(A)
        res.append((Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out.stats))
    assert res[0][4]["nfallback"] > 0
    _same(res[0], res[1], 1.0)


TAIL_CASES = dict(CASES)
TAIL_CASES["graded_2200x300"] = lambda: _graded(2200, 300, 19)  # blocks with flagged norms, then the tail


@pytest.mark.parametrize("name", sorted(TAIL_CASES))
@pytest.mark.parametrize("rule", [oracle.STOP_PAPER, oracle.STOP_NONE, oracle.STOP_MAXNORM])
def test_tail_kernel_matches_oracle(name, rule, monkeypatch):
    """QRP with the register-resident tail (the default path) against the oracle."""
    Q = _gpu()
    a = TAIL_CASES[name]()
    print(f"case {name} rule {rule}", flush=True)
    R, tau, perm, rank, st = _run(Q, a, False, monkeypatch, tail=True, stop_rule=rule)
    ref = oracle.qrp(a, stop_rule=rule)
    m, n = a.shape
    if min(m, n) == 0 or not np.any(a):
        assert rank == 0 and np.array_equal(perm, np.arange(n))
        return
    compare(a, ref, R, tau, perm, rank, [], check_blocks=False, full=(rule == oracle.STOP_NONE), stop_rule=rule,
            kmax=1)


def test_tail_after_a_stop_inside_a_block(monkeypatch):
    """A stop inside a block launch (column 60 of the block 32..63), and the tail
    launch right after it (no poll lag: the host sees 2040 rows left): the tail
    finishes the stopped block and ends the loop."""
    Q = _gpu()
    n = 300
    s = np.concatenate([np.geomspace(1.0, 1e-3, 60), np.full(n - 60, 1e-15)])
    a = I.from_spectrum(2100, n, s, 23)
    ref = oracle.qrp(a, stop_rule=oracle.STOP_MAXNORM)
    R, tau, perm, rank, _ = _run(Q, a, False, monkeypatch, tail=True, stop_rule=oracle.STOP_MAXNORM, poll_lag=0)
    assert rank == ref.rank == 60
    compare(a, ref, R, tau, perm, rank, [], check_blocks=False, stop_rule=oracle.STOP_MAXNORM, kmax=1)


def test_qrdm_continuation_with_the_tail(monkeypatch):
    """QRDM's scalar-pivoting continuation on the tail kernel agrees with the
    block kernel's to rounding on the decisions taken above the noise level,
    and both with the oracle."""
    Q = _gpu()
    n = 1300
    a = I.from_spectrum(1500, n, np.geomspace(1, 1e-16, n), 9)
    ref = oracle.qrdm(a, stop_rule=oracle.STOP_NONE)
    outs = []
    for tail in (True, False):
        if tail:
            monkeypatch.delenv("QRDM_QP3_TAIL", raising=False)
        else:
            monkeypatch.setenv("QRDM_QP3_TAIL", "0")
        A = Q.device_matrix(a)
        out = Q.qrdm_factor(A, stop_rule=oracle.STOP_NONE, log=True)
        outs.append(out)
        compare(a, ref, Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out.blocks,
                full=True, stop_rule=oracle.STOP_NONE, kmax=64)
    assert outs[0].stats["qp3_start"] == outs[1].stats["qp3_start"] > 0
