"""Pins of the least-squares oracle against library solvers and the normal
equations of the basic solution."""
import numpy as np
import pytest

import oracle
from oracle import lstsq as Ls
from paper_2106_03138_amd import inputs as I


def _fac(a, **kw):
    r = oracle.qrdm(a, **kw)
    return r.qr, r.tau, r.perm, r.rank


@pytest.mark.parametrize("seed", range(3))
def test_square_full_rank_equals_solve(seed):
    rng = np.random.default_rng(seed)
    a = np.asfortranarray(rng.standard_normal((60, 60)) + 8 * np.eye(60))
    b = rng.standard_normal((60, 3))
    qr, tau, perm, rank = _fac(a, stop_rule=oracle.STOP_NONE)
    x = Ls.basic_solution(qr, tau, perm, 60, b)
    np.testing.assert_allclose(x, np.linalg.solve(a, b), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_tall_full_column_rank_equals_lstsq(seed):
    rng = np.random.default_rng(seed + 10)
    a = np.asfortranarray(rng.standard_normal((200, 40)))
    b = rng.standard_normal(200)
    qr, tau, perm, rank = _fac(a)
    assert rank == 40
    x = Ls.basic_solution(qr, tau, perm, rank, b)[:, 0]
    np.testing.assert_allclose(x, np.linalg.lstsq(a, b, rcond=None)[0], rtol=1e-10, atol=1e-12)


def test_rank_deficient_basic_solution():
    """Rank r < n: n - r zeros at perm[r:], the least-squares solution over the
    selected columns, and a residual orthogonal to them."""
    rng = np.random.default_rng(3)
    a = I.from_spectrum(150, 90, np.concatenate([np.geomspace(1, 1e-4, 30), np.zeros(60)]), 4)
    b = rng.standard_normal((150, 2))
    qr, tau, perm, rank = _fac(a, stop_rule=oracle.STOP_MAXNORM)
    assert rank == 30
    x = Ls.basic_solution(qr, tau, perm, rank, b)
    assert np.all(x[perm[rank:], :] == 0.0)
    sel = a[:, perm[:rank]]
    np.testing.assert_allclose(x[perm[:rank], :], np.linalg.lstsq(sel, b, rcond=None)[0], rtol=1e-8, atol=1e-8)
    res = b - a @ x
    assert np.max(np.abs(sel.T @ res)) <= 1e-10 * np.linalg.norm(sel) * np.linalg.norm(b)


def test_apply_qt_is_orthogonal():
    rng = np.random.default_rng(5)
    a = np.asfortranarray(rng.standard_normal((80, 50)))
    qr, tau, perm, rank = _fac(a, stop_rule=oracle.STOP_NONE)
    b = rng.standard_normal((80, 4))
    y = Ls.apply_qt(qr, tau, b, 50)
    np.testing.assert_allclose(np.linalg.norm(y, axis=0), np.linalg.norm(b, axis=0), rtol=1e-13)
    # Q^T A P = R
    r = Ls.apply_qt(qr, tau, a[:, perm], 50)
    np.testing.assert_allclose(np.tril(r, -1), 0.0, atol=1e-12 * np.linalg.norm(a))


def test_zero_rank():
    x = Ls.basic_solution(np.zeros((5, 4)), np.zeros(4), np.arange(4), 0, np.ones(5))
    assert np.all(x == 0.0)
