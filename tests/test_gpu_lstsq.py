"""Least-squares solve (qrdm_lstsq, qrdm_batch_lstsq) against the oracle
(oracle/lstsq.py).

Tolerances.  Applying r reflectors is backward stable: both sides compute
y = Q_r^T b to within a few units of eps * ||b|| per reflector block, so rows of
y agree to TOL_Y * ||b||.  Back substitution amplifies a relative perturbation
of y and R11 by at most cond(R11), so x agrees to TOL_X * cond(R11) * ||x||.
End to end (each side factors the matrix itself) the factors agree normwise
to rounding, and the solutions are compared through the residual norm and the
normal equations of the selected columns, which hold at any condition number.
"""
import numpy as np
import pytest

import oracle
from oracle import lstsq as Ls
from paper_2106_03138_amd import inputs as I
from parity import ETA

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
TOL_Y = 200 * EPS
TOL_X = 1000 * EPS


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


def _check_isolated(qr, tau, perm, r, b, B_out, X, resid, tag):
    m, n = qr.shape
    nrhs = b.shape[1]
    rr = max(0, min(r, m, n))
    y = Ls.apply_qt(qr, tau, b, rr) if m else b
    xo = Ls.basic_solution(qr, tau, perm, rr, b)
    # exact zeros on the columns that were not selected (index work)
    assert np.all(X[perm[rr:], :] == 0.0), tag
    nb = max(np.max(np.linalg.norm(b, axis=0)), 1e-300) if m else 1.0
    if m > rr:
        assert np.max(np.abs(B_out[rr:] - y[rr:])) <= TOL_Y * nb, tag
    np.testing.assert_allclose(resid, np.linalg.norm(y[rr:], axis=0) if m else np.zeros(nrhs), rtol=1e-12,
                               atol=TOL_Y * nb, err_msg=tag)
    if rr:
        cond = np.linalg.cond(np.triu(qr[:rr, :rr]))
        scale = max(np.max(np.abs(xo)), 1e-300)
        assert np.max(np.abs(X - xo)) <= TOL_X * cond * scale, (tag, np.max(np.abs(X - xo)) / scale, cond)
        assert np.max(np.abs(B_out[:rr] - xo[perm[:rr]])) <= TOL_X * cond * scale, tag


SHAPES = [(300, 200, 150), (40, 40, 40), (520, 30, 30), (17, 60, 17), (1, 5, 1), (9, 1, 1), (33, 20, 0),
          (270, 270, 263), (600, 300, 299), (64, 64, 8), (1100, 700, 650)]


@pytest.mark.parametrize("nrhs", [1, 3, 5])
def test_single_entry_matches_oracle_on_given_factors(nrhs):
    """qrdm_lstsq on synthetic factors (the same arrays on both sides)."""
    import torch
    Q = _gpu()
    rng = np.random.default_rng(nrhs)
    for i, (m, n, r) in enumerate(SHAPES):
        qr, tau, perm = I.lstsq_factors(m, n, r, 100 + i)
        b = rng.standard_normal((m, nrhs))
        A = Q.device_matrix(qr)
        fac = Q.Factorization(torch.as_tensor(tau).cuda(), torch.as_tensor(perm).cuda(), r)
        B = Q.device_matrix(b)
        X, resid = Q.lstsq(A, fac, B)
        torch.cuda.synchronize()
        _check_isolated(qr, tau, perm, r, b, Q.host_matrix(B), X.cpu().numpy(), resid.cpu().numpy(),
                        f"{m}x{n} r={r} nrhs={nrhs}")


def _batched_isolated(nrhs, shapes, seed):
    import torch
    Q = _gpu()
    rng = np.random.default_rng(seed)
    facs = [I.lstsq_factors(m, n, r, seed * 1000 + i) for i, (m, n, r) in enumerate(shapes)]
    bt = Q.Batch([(m, n) for m, n, _ in shapes])
    bt.load([f[0] for f in facs])
    bt.tau.copy_(torch.as_tensor(np.concatenate([f[1] for f in facs] + [np.zeros(1)])[: bt.tau.numel()]))
    bt.perm.copy_(torch.as_tensor(np.concatenate([f[2] for f in facs] + [np.zeros(1, np.int32)])[: bt.perm.numel()]))
    bt.rank.copy_(torch.as_tensor([r for _, _, r in shapes] or [0], dtype=torch.int64))
    plan = Q.BatchPlan(bt)
    rhs = Q.BatchRHS(bt, nrhs)
    bs = [rng.standard_normal((m, nrhs)) for m, _, _ in shapes]
    rhs.load(bs)
    plan.lstsq(rhs)
    torch.cuda.synchronize()
    for i, (m, n, r) in enumerate(shapes):
        qr, tau, perm = facs[i]
        _check_isolated(qr, tau, perm, r, bs[i], rhs.rhs(i), rhs.solution(i), rhs.residual(i),
                        f"batched matrix {i} {m}x{n} r={r} nrhs={nrhs}")
    plan.close()


@pytest.mark.parametrize("nrhs", [1, 4, 6])
def test_batched_entry_matches_oracle_on_given_factors(nrhs):
    shapes = [(m, n, r) for m, n, r in SHAPES if n <= 512]
    shapes += [(0, 3, 0), (512, 512, 512), (77, 77, 76)]
    _batched_isolated(nrhs, shapes, seed=7 + nrhs)


def test_rank_clamped_and_failed_factorization():
    """rank > min(m, n) is read as min(m, n); rank < 0 gives NaN solutions and
    leaves B as it was."""
    import torch
    Q = _gpu()
    qr, tau, perm = I.lstsq_factors(50, 30, 30, 5)
    b = np.random.default_rng(1).standard_normal((50, 2))
    A = Q.device_matrix(qr)
    fac = Q.Factorization(torch.as_tensor(tau).cuda(), torch.as_tensor(perm).cuda(), 99)
    B = Q.device_matrix(b)
    X, resid = Q.lstsq(A, fac, B)
    _check_isolated(qr, tau, perm, 30, b, Q.host_matrix(B), X.cpu().numpy(), resid.cpu().numpy(), "clamped")
    B = Q.device_matrix(b)
    X, resid = Q.lstsq(A, fac, B, rank=-1)
    torch.cuda.synchronize()
    assert np.all(np.isnan(X.cpu().numpy())) and np.all(np.isnan(resid.cpu().numpy()))
    assert np.array_equal(Q.host_matrix(B), b)


def _end_to_end_checks(a, b, x, resid, perm, rank, ref, tag):
    """x, resid, perm, rank from the GPU path; ref the oracle's factorization of
    the same matrix.  The pivot order must equal the oracle's wherever the
    oracle's decisions have a clear margin (the parity rule of the
    factorization tests); the solutions are then compared through residuals."""
    r = int(rank)
    same = r == ref.rank and np.array_equal(perm, ref.perm)
    if ref.first_low_margin_block(ETA) == len(ref.blocks):
        assert same, tag
    # exact zeros outside the selected columns (index work)
    assert np.all(x[perm[r:], :] == 0.0), tag
    res_g = b - a @ x
    nb = np.linalg.norm(b, axis=0)
    na = np.linalg.norm(a, 2)
    nx = np.linalg.norm(x, axis=0)
    # the reported residual is the true one
    assert np.all(np.abs(resid - np.linalg.norm(res_g, axis=0)) <= 1e-10 * (na * nx + nb)), tag
    # normal equations of the selected columns: A_S^T (b - A x) = 0
    sel = a[:, perm[:r]]
    ns = np.linalg.norm(sel, 2)
    assert np.all(np.linalg.norm(sel.T @ res_g, axis=0) <= 1e-10 * ns * (ns * nx + nb)), tag
    if same:
        xo = Ls.basic_solution(ref.qr, ref.tau, ref.perm, ref.rank, b)
        res_o = b - a @ xo
        assert np.all(np.abs(np.linalg.norm(res_g, axis=0) - np.linalg.norm(res_o, axis=0))
                      <= 1e-10 * (na * nx + nb)), tag
    return same


@pytest.mark.parametrize("kind", ["rank64", "gaussian_tall", "wide"])
def test_end_to_end_single(kind):
    import torch
    Q = _gpu()
    if kind == "rank64":
        a = I.small_rank64(2)
    elif kind == "gaussian_tall":
        a = I.gaussian(900, 400, 3)
    else:
        a = I.gaussian(120, 300, 4)
    b = np.random.default_rng(9).standard_normal((a.shape[0], 3))
    ref = oracle.qrdm(a)
    A = Q.device_matrix(a)
    fac = Q.qrdm_factor(A)
    B = Q.device_matrix(b)
    X, resid = Q.lstsq(A, fac, B)
    torch.cuda.synchronize()
    _end_to_end_checks(a, b, X.cpu().numpy(), resid.cpu().numpy(), fac.perm.cpu().numpy(), fac.rank, ref, kind)


def test_end_to_end_qrp():
    import torch
    Q = _gpu()
    a = I.small_rank64(4)
    b = np.random.default_rng(2).standard_normal((256, 1))
    ref = oracle.qrp(a)
    A = Q.device_matrix(a)
    fac = Q.qrp_factor(A)
    B = Q.device_matrix(b)
    X, resid = Q.lstsq(A, fac, B)
    torch.cuda.synchronize()
    _end_to_end_checks(a, b, X.cpu().numpy(), resid.cpu().numpy(), fac.perm.cpu().numpy(), fac.rank, ref, "qrp")


def test_end_to_end_batched_small():
    """A scaled-down uneven least-squares batch: GPU factor + solve against the
    oracle's factor + solve of every matrix."""
    import torch
    Q = _gpu()
    shapes = I.batch_shapes(40, seed=31, mmin=8, mmax=200, nmin=1)
    seqs = np.random.SeedSequence(31).spawn(len(shapes))
    mats = [I.batch_matrix(m, n, r, s) for (m, n, r), s in zip(shapes, seqs)]
    rng = np.random.default_rng(5)
    bs = [rng.standard_normal((a.shape[0], 2)) for a in mats]
    bt = Q.Batch([a.shape for a in mats])
    bt.load(mats)
    plan = Q.BatchPlan(bt)
    plan.factor()
    rhs = Q.BatchRHS(bt, 2)
    rhs.load(bs)
    plan.lstsq(rhs)
    torch.cuda.synchronize()
    rank = bt.rank.cpu().numpy()
    same = 0
    for i, a in enumerate(mats):
        ref = oracle.qrdm(a)
        same += _end_to_end_checks(a, bs[i], rhs.solution(i), rhs.residual(i), bt.permutation(i), rank[i], ref,
                                   f"batched {i} {a.shape}")
    print(f"{same} of {len(mats)} matrices with the oracle's pivot order and rank")
    plan.close()


def test_full_batch_sampled():
    """The full uneven batch (2048 matrices, m in [32, 512]) factored and solved
    in the configuration the benchmark times; sampled matrices checked against
    the oracle, and the normal equations checked on every matrix."""
    import torch
    Q = _gpu()
    mats, shapes = I.batch(2048, seed=0)
    rng = np.random.default_rng(0)
    bs = [rng.standard_normal(a.shape[0]) for a in mats]
    bt = Q.Batch([a.shape for a in mats])
    bt.load(mats)
    plan = Q.BatchPlan(bt)
    plan.factor(use_graph=True)
    rhs = Q.BatchRHS(bt, 1)
    rhs.load(bs)
    plan.lstsq(rhs)
    torch.cuda.synchronize()
    rank = bt.rank.cpu().numpy()
    xs = rhs.x.cpu().numpy()
    for i, a in enumerate(mats):
        n = a.shape[1]
        x = xs[rhs.xoff[i]: rhs.xoff[i] + n]
        perm = bt.permutation(i)
        r = int(rank[i])
        assert np.all(x[perm[r:]] == 0.0), i
        res = bs[i] - a @ x
        sel = a[:, perm[:r]]
        ns = np.linalg.norm(sel)  # Frobenius: an upper bound of the 2-norm
        assert np.linalg.norm(sel.T @ res) <= 1e-10 * ns * (ns * np.linalg.norm(x) + np.linalg.norm(bs[i])), i
    for i in rng.choice(len(mats), 6, replace=False):
        ref = oracle.qrdm(mats[i])
        _end_to_end_checks(mats[i], bs[i][:, None], rhs.solution(i), rhs.residual(i), bt.permutation(i), rank[i],
                           ref, f"full batch {i}")
    plan.close()
