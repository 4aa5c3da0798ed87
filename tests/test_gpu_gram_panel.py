"""The two panels of a QRDM block (Algorithm 4, the Householder panel with the
break of eq. lenght_check).  For blocks of at most 64 columns the panel is
formed from the Gram matrix of the block: CholeskyQR2 with the break on the
Cholesky diagonal and Householder reconstruction (k_cpanel.hip); otherwise,
or when that route declines the block (a Cholesky diagonal below 1e-4 of its
column's norm, max |Q1^T Q1 - I| > 1e-9), column by column (k_panel.hip).
QRDM_GRAM_PANEL=0 sends every block to the column-by-column panel.

Each case runs both ways; each run is compared with the oracle on the same
input (tests/parity.compare: exact decisions up to the first low-margin block,
R normwise and on its diagonal, the rank, the backward error), and
stats['ngram'] shows which route took the blocks.  Cases: a geometric
spectrum that switches to scalar pivoting, a rank-64 matrix whose panel
breaks, Gaussian blocks of 32 and 64 columns, a wide matrix whose last block
reaches the last row (a one-row column: tau = 0, the sign of its R entry kept),
the Kahan matrix, and mixed precision.
"""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from paper_2106_03138_amd import inputs as I
from parity import compare

pytestmark = pytest.mark.gpu


def _run(a, monkeypatch, gram, **kw):
    import paper_2106_03138_amd as Q
    Q.load()
    if gram:
        monkeypatch.delenv("QRDM_GRAM_PANEL", raising=False)
    else:
        monkeypatch.setenv("QRDM_GRAM_PANEL", "0")
    A = Q.device_matrix(a)
    out = Q.qrdm_factor(A, log=True, **kw)
    return Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out


def _say(msg):
    print(f"[gram panel] {msg}", flush=True)


def _geometric():
    return I.from_spectrum(1500, 1300, np.geomspace(1.0, 1e-16, 1300), 9)


def _wide():
    a = I.gaussian(96, 200, 4)
    return np.asfortranarray(a * np.exp(np.linspace(0, -3, 200))[None, :])


CASES = {
    "geometric 1500x1300 k64": (_geometric, dict(tau=0.15, delta=0.9, kmax=64), False),
    "rank64 256 k64": (lambda: I.small_rank64(1), dict(tau=0.9, delta=0.9, kmax=64), False),
    "gaussian 700x600 k32": (lambda: I.gaussian(700, 600, 3), dict(tau=0.15, delta=0.9, kmax=32), True),
    "gaussian 900x640 k64": (lambda: I.gaussian(900, 640, 8), dict(tau=0.5, delta=0.5, kmax=64), True),
    "wide 96x200 k32": (_wide, dict(tau=0.15, delta=0.9, kmax=32), True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_both_panels_against_oracle(case, monkeypatch):
    make, kw, full = CASES[case]
    a = make()
    rule = oracle.STOP_NONE if full else oracle.STOP_PAPER
    ref = oracle.qrdm(a, stop_rule=rule, **kw)
    for gram in (True, False):
        qr, tau, perm, rank, out = _run(a, monkeypatch, gram, stop_rule=rule, **kw)
        st = out.stats
        cmp = compare(a, ref, qr, tau, perm, rank, out.blocks, full=full, stop_rule=rule, kmax=kw["kmax"])
        _say(f"{case} gram={gram}: rank {rank} (oracle {ref.rank}), panels {st['npanel']}, from the Gram "
             f"matrix {st['ngram']}, breaks {st['nbreaks']}, ns_cut {cmp['ns_cut']}, diag {cmp.get('diag_eps')} "
             f"eps ||A||")
        if gram:
            assert st["ngram"] >= 1
        else:
            assert st["ngram"] == 0


@pytest.mark.parametrize("gram", [True, False])
def test_last_row_block(gram, monkeypatch):
    """96 rows, 200 columns, blocks of up to 32: the factorization ends on a block
    that reaches the last row; its last reflector has one row, which larfg leaves
    alone (tau = 0, the sign of the R entry kept), on either panel."""
    a = _wide()
    qr, tau, perm, rank, out = _run(a, monkeypatch, gram, stop_rule=oracle.STOP_NONE, tau=0.15, delta=0.9,
                                    kmax=32)
    last = max(b[0] + b[3] for b in out.blocks if b[3] > 0)
    assert last == 96
    ref = oracle.qrdm(a, stop_rule=oracle.STOP_NONE, tau=0.15, delta=0.9, kmax=32)
    assert ref.tau[95] == 0.0 and tau[95] == 0.0
    assert np.sign(qr[95, 95]) == np.sign(ref.qr[95, 95])
    assert (out.stats["ngram"] >= 1) == gram


def test_kahan(monkeypatch):
    """Kahan K_512(1.2), whose trailing columns are nearly dependent: the
    factorization with the Gram route on is backward stable and its rank at
    least the numerical rank."""
    a = I.kahan(512, 1.2)
    qr, tau, perm, rank, out = _run(a, monkeypatch, True)
    st = out.stats
    _say(f"Kahan 512: panels {st['npanel']}, from the Gram matrix {st['ngram']}, rank {rank}")
    assert 1 <= st["ngram"] <= st["npanel"]
    assert sorted(perm.tolist()) == list(range(512))
    assert M.residual(a, qr, tau, perm, rank) <= 1e-13
    sig = np.linalg.svd(a, compute_uv=False)
    assert rank >= M.numerical_rank(sig, 512)


def test_mixed_precision_both_panels(monkeypatch):
    """Mixed precision writes the FP32 copy of V from either panel: the two runs
    reach the same rank and an FP32-level backward error."""
    a = _geometric()
    ranks = {}
    for gram in (True, False):
        qr, tau, perm, rank, out = _run(a, monkeypatch, gram, precision=1)
        res = M.residual(a, qr, tau, perm, rank)
        _say(f"mixed gram={gram}: rank {rank}, residual {res:.2e}, Gram panels {out.stats['ngram']}")
        assert res <= 1e-5
        ranks[gram] = rank
    assert abs(ranks[True] - ranks[False]) <= 64
