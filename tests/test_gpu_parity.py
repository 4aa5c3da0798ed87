"""GPU parity: libqrdm.so (HIP, gfx950) against the FP64 CPU oracle.

Both sides run on the same seeded inputs.  Decisions (arg-max, candidate
order, tau threshold, |theta| < delta, the panel break, the stopping test) are
compared exactly up to the first block where the oracle records a decision
margin below ETA (relative), beyond which two correct FP64 implementations
may legitimately differ.  Floating-point results are compared normwise: two
Householder QRs with different summation orders differ by O(eps ||A||).
"""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from paper_2106_03138_amd import inputs as I
from parity import EPS, ETA, compare as _compare

pytestmark = pytest.mark.gpu


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


def _run_gpu(a, **kw):
    Q = _gpu()
    A = Q.device_matrix(a)
    out = Q.qrdm_factor(A, log=True, **kw)
    return Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out


def test_colnorms():
    Q = _gpu()
    a = I.gaussian(1000, 77, 1)
    v = Q.colnorms(Q.device_matrix(a)).cpu().numpy()
    np.testing.assert_allclose(v, np.linalg.norm(a, axis=0), rtol=1e-14)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("tau,delta,kmax", [(0.15, 0.9, 64), (0.5, 0.5, 32), (0.05, 0.95, 128)])
def test_dm_step(seed, tau, delta, kmax):
    Q = _gpu()
    rng = np.random.default_rng(seed)
    m, n = 300, 200
    a = rng.standard_normal((m, n)) @ (np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n))
    a = np.asfortranarray(a * np.exp(rng.uniform(-1, 1, n))[None, :])
    ns = 7
    u = np.linalg.norm(a[ns:, :], axis=0)
    L0, th0, J0 = oracle.dm_step(a, u, ns, tau, delta, kmax)
    A = Q.device_matrix(a)
    import torch
    vn1 = torch.from_numpy(u).cuda()
    L1, th1, J1 = Q.dm_step(A, ns, vn1, tau, delta, kmax)
    assert np.array_equal(L1, L0)
    assert np.max(np.abs(th1 - th0)) <= 1e-13
    assert np.array_equal(J1, J0)
    assert np.array_equal(Q.host_matrix(A), a)  # A untouched


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("rule", [oracle.STOP_PAPER, oracle.STOP_MAXNORM, oracle.STOP_NONE])
def test_rank64_256(seed, rule):
    """256^2, sigma_1..64 geometric 1 -> 1e-3, the rest 1e-15; tau = delta = 0.9, k = 32."""
    a = I.small_rank64(seed)
    ref = oracle.qrdm(a, tau=0.9, delta=0.9, kmax=32, stop_rule=rule)
    qr, tau, perm, rank, out = _run_gpu(a, tau=0.9, delta=0.9, kmax=32, stop_rule=rule)
    _compare(a, ref, qr, tau, perm, rank, out.blocks, full=(rule == oracle.STOP_NONE), stop_rule=rule, kmax=32)
    if rule == oracle.STOP_MAXNORM:
        assert rank == 64


@pytest.mark.parametrize("shape,params", [
    ((300, 200), dict(tau=0.15, delta=0.9, kmax=64)),
    ((333, 257), dict(tau=0.15, delta=0.9, kmax=64)),
    ((333, 257), dict(tau=0.3, delta=0.6, kmax=128)),
    ((520, 390), dict(tau=0.05, delta=0.95, kmax=48)),
    ((200, 300), dict(tau=0.15, delta=0.9, kmax=64)),
    ((129, 129), dict(tau=0.15, delta=0.9, kmax=1)),
    ((17, 5), dict(tau=0.5, delta=0.5, kmax=8)),
])
def test_gaussian_shapes(shape, params):
    """Ragged sizes across several panel slabs, GEMM tiles and split-K chunks."""
    a = I.gaussian(*shape, seed=shape[0] + shape[1])
    a = np.asfortranarray(a * np.exp(np.linspace(0, -5, shape[1]))[None, :])
    ref = oracle.qrdm(a, stop_rule=oracle.STOP_NONE, **params)
    qr, tau, perm, rank, out = _run_gpu(a, stop_rule=oracle.STOP_NONE, **params)
    _compare(a, ref, qr, tau, perm, rank, out.blocks, full=True)


def test_tall_1500():
    """Tall panel: 12 slabs of the cooperative panel, two GEMM1 row splits."""
    a = I.from_spectrum(1500, 300, np.geomspace(1, 1e-10, 300), seed=5)
    ref = oracle.qrdm(a, stop_rule=oracle.STOP_PAPER)
    qr, tau, perm, rank, out = _run_gpu(a, stop_rule=oracle.STOP_PAPER)
    _compare(a, ref, qr, tau, perm, rank, out.blocks)


def test_three_directions_break():
    a = I.three_directions(16, 0)
    ref = oracle.qrdm(a, tau=0.5, delta=0.9, kmax=8)
    qr, tau, perm, rank, out = _run_gpu(a, tau=0.5, delta=0.9, kmax=8)
    assert rank == 2 and ref.rank == 2
    assert out.blocks[0][1:4] == (3, 3, 2)
    _compare(a, ref, qr, tau, perm, rank, out.blocks)


def test_qrp_parity():
    Q = _gpu()
    a = I.gaussian(240, 180, 9)
    a = np.asfortranarray(a * np.exp(np.linspace(0, -8, 180))[None, :])
    ref = oracle.qrp(a, stop_rule=oracle.STOP_NONE)
    A = Q.device_matrix(a)
    out = Q.qrp_factor(A, stop_rule=oracle.STOP_NONE)
    qr = Q.host_matrix(A)
    _compare(a, ref, qr, out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, [], check_blocks=False,
             full=True)


def test_degenerate():
    Q = _gpu()
    z = np.zeros((40, 30), order="F")
    A = Q.device_matrix(z)
    out = Q.qrdm_factor(A)
    assert out.rank == 0
    assert np.array_equal(out.perm.cpu().numpy(), np.arange(30))
    bad = I.gaussian(50, 20, 0)
    bad[3, 4] = np.inf
    A = Q.device_matrix(bad)
    with pytest.raises(Q.QrdmError) as ei:
        Q.qrdm_factor(A)
    assert ei.value.code == 1
    got = Q.host_matrix(A)
    assert np.array_equal(got[np.isfinite(bad)], bad[np.isfinite(bad)])
    r1 = Q.device_matrix(I.rank1(64, 20, 1))
    assert Q.qrdm_factor(r1).rank == 1
    with pytest.raises(Q.QrdmError) as ei:
        Q.qrdm_factor(Q.device_matrix(I.gaussian(8, 8, 0)), tau=-0.1)
    assert ei.value.code == -5


def test_mixed_precision_rank64():
    """Mixed mode (FP32 MFMA trailing update, FP64 panel/norms/rank test with eps_w = 2^-23):
    rank equals the FP64 oracle's where the spectrum gap (1e-3 -> 1e-15) lies far above
    FP32 rounding.  Pivots may differ once FP32 noise breaks near-ties, so quality is
    judged as in Section 5: d_i / sigma_i within the factor-10 band, and the backward
    error is of FP32 size."""
    a = I.small_rank64(0)
    ref = oracle.qrdm(a, tau=0.9, delta=0.9, kmax=32, stop_rule=oracle.STOP_MAXNORM)
    qr, tau, perm, rank, out = _run_gpu(a, tau=0.9, delta=0.9, kmax=32, stop_rule=oracle.STOP_MAXNORM, precision=1)
    assert rank == ref.rank == 64
    res = M.residual(a, qr, tau, perm, rank)
    assert res <= 1e-6, res
    sig = M.singular_values(a)
    rg = M.diag_ratios(M.r_factor(qr, rank), sig, 64)
    ro = M.diag_ratios(M.r_factor(ref.qr, ref.rank), sig, 64)
    assert rg.min() >= 0.1 and rg.max() <= 10.0
    assert ro.min() >= 0.1 and ro.max() <= 10.0
    # leading diagonal (before FP32 noise can matter) agrees to FP32 accuracy
    np.testing.assert_allclose(np.abs(np.diag(qr)[:3]), np.abs(np.diag(ref.qr)[:3]), rtol=1e-5)


def test_deterministic():
    Q = _gpu()
    a = I.gaussian(700, 500, 3)
    outs = []
    for _ in range(2):
        A = Q.device_matrix(a)
        o = Q.qrdm_factor(A, stop_rule=oracle.STOP_NONE)
        outs.append((Q.host_matrix(A), o.perm.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("precision", [0, 1])
def test_bits_independent_of_poll_lag(precision):
    """The host polls the device's progress `poll_lag` steps behind and sizes the
    launches from that bound; the kernels take every split from the actual sizes,
    so the factorization comes out the same to the bit for any lag, with or
    without the block log (which polls every step).  The switch to scalar
    pivoting is decided on the device, which idles the DM loop from that step on,
    so the column-pivoting kernels start at the same column whatever the lag: the
    comparison covers all n columns."""
    Q = _gpu()
    a = I.from_spectrum(1500, 1300, np.geomspace(1.0, 1e-16, 1300), 9)
    outs = []
    fb = None
    starts = set()
    for lag, log in [(4, True), (0, False), (1, False), (4, False), (9, False)]:
        A = Q.device_matrix(a)
        o = Q.qrdm_factor(A, stop_rule=oracle.STOP_NONE, precision=precision, poll_lag=lag, log=log)
        if log:
            hand = [x for x in o.blocks if x[4]]
            assert len(hand) <= 1 and all(x[3] == 0 for x in hand)
            fb = hand[0][0] if hand else -1
        starts.add(o.stats["qp3_start"])
        outs.append((Q.host_matrix(A), o.tau_house.cpu().numpy(), o.perm.cpu().numpy(), o.rank))
    assert starts == {fb}
    if precision == 0:
        assert fb > 100  # FP64: the geometric spectrum reaches n eps max||a_j|| before column n
    else:
        assert fb == -1  # FP32 rounding noise stays above the FP64 switch: DM blocks to the end
    for qr, tau, perm, rank in outs[1:]:
        assert np.array_equal(qr, outs[0][0]) and np.array_equal(tau, outs[0][1])
        assert np.array_equal(perm, outs[0][2]) and rank == outs[0][3]


def test_workspace_entry_two_streams():
    """qrdm_factor_ws in caller-owned workspaces: two factorizations launched from
    two host threads on two streams at once give the same bits and ranks as the
    same calls run one after the other, and as qrdm_factor_ex."""
    import threading

    import torch
    Q = _gpu()
    mats = [I.from_spectrum(1100, 900, np.geomspace(1.0, 1e-9, 900), 21),
            I.gaussian(1300, 700, 22)]
    kw = dict(tau=0.15, delta=0.9, kmax=64, stop_rule=oracle.STOP_PAPER)
    ref = []
    for a in mats:
        A = Q.device_matrix(a)
        o = Q.qrdm_factor(A, **kw)
        ref.append((Q.host_matrix(A), o.tau_house.cpu().numpy(), o.perm.cpu().numpy(), o.rank))
    dev = torch.device("cuda")
    wss = [torch.empty(Q.api.workspace_size(*a.shape, 64), dtype=torch.uint8, device=dev) for a in mats]
    ranks = [torch.full((1,), -7, dtype=torch.int64, device=dev) for _ in mats]

    def run(i, stream, out):
        with torch.cuda.stream(stream):
            A = Q.device_matrix(mats[i])
            stream.synchronize()
            o = Q.api.qrdm_factor_ws(A, wss[i], ranks[i], stream=stream, **kw)
            stream.synchronize()
            out[i] = (Q.host_matrix(A), o.tau_house.cpu().numpy(), o.perm.cpu().numpy(), int(ranks[i].item()))

    for concurrent in (False, True):
        out = [None, None]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        if concurrent:
            th = [threading.Thread(target=run, args=(i, streams[i], out)) for i in range(2)]
            for t in th:
                t.start()
            for t in th:
                t.join()
        else:
            for i in range(2):
                run(i, streams[i], out)
        for i in range(2):
            assert out[i] is not None, f"thread {i} failed"
            qr, tau, perm, rank = out[i]
            assert rank == ref[i][3]
            assert np.array_equal(qr, ref[i][0]) and np.array_equal(tau, ref[i][1]) and np.array_equal(perm, ref[i][2])
