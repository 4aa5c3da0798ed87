"""The QP3 column loop (Algorithm 2 blocked like xgeqp3) runs one block of up
to nb pivots per cooperative launch; the per-step kernels remain selectable
(QRDM_QP3_STEPS=1).  Both carry out the same arithmetic in the same order, so
pivots and rank must agree exactly and R / tau to rounding of the contraction
(1e-13 relative).  The block kernel holds its columns in LDS when they fit
(2048 rows at most) and reads them from memory otherwise: tall_2200x400
starts in the second mode and ends in the first.  The block path is also
checked against the oracle."""
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


def _run(Q, a, steps, monkeypatch, **kw):
    if steps:
        monkeypatch.setenv("QRDM_QP3_STEPS", "1")
    else:
        monkeypatch.delenv("QRDM_QP3_STEPS", raising=False)
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
