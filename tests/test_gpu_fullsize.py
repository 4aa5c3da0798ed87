"""Parity at the benchmark's full size and launch configuration: 8192 x 8192,
tau = 0.15, delta = 0.9, k_DM = 64, stopping criterion off (full factorization),
FP64, the library's default stream, preallocated tau and perm as the benchmark
passes them, on the three spectra of the 8192^2 workload: geometric from 1 to
1e-16 (the benchmark's matrix), the devil's stairs (steps of 512 columns, each
10x lower) and Gaussian N(0, 1) entries.

Checks, per spectrum:
- the oracle on the same matrix: permutation identical up to the first block with
  a decision margin below 1e-10 (that prefix length, ns_cut, is printed and must
  reach the first column with sigma_j < 1e-6 sigma_1; all of it on the Gaussian
  matrix), R normwise and its diagonal relatively on that prefix, the rank
  (exact, or inside the oracle's noise band of the stopping test), and the
  backward error estimated from 64 sampled columns of AP (applying Q^T to all of
  AP is too slow on the host);
- sigma_min(R11) / sigma_r(A) at the numerical rank (geometric spectrum);
- Algorithm 1 and the check step of Algorithm 4 replayed from the GPU's R at every
  logged block start to column n (invariants.check_dm_replay): candidate list,
  greedy maximality, the break, the switch to scalar pivoting;
- the properties that hold at any size (tests/invariants.py): the candidate and
  greedy rules for every logged block, the single-pivot rule on the
  scalar-pivoting tail, the practical stopping criterion's rank, and the
  orthogonality of every reflector;
- both runs, the benchmark's and one with the block log.  The log makes the host
  wait on every step (no poll lag), so the launch bounds differ; the kernels take
  their splits from the actual sizes, so the two runs agree to the bit in every
  column.  Each run is also compared with the oracle on its own.
"""
import time

import numpy as np
import pytest

import invariants as V
import oracle
from parity import EPS, NU_SCALE, compare
from paper_2106_03138_amd import inputs as I

N = 8192
TAU, DELTA, KMAX = 0.15, 0.9, 64
SPECTRA = ["geometric", "stairs", "gaussian"]

pytestmark = pytest.mark.gpu


def _say(spec, msg):
    print(f"[fullsize {N}x{N} {spec} seed 0] {msg}", flush=True)


def _sigma(spec):
    """Singular values fixed by construction (None for the Gaussian matrix)."""
    if spec == "geometric":
        return np.geomspace(1.0, 1e-16, N)
    if spec == "stairs":
        return 10.0 ** (-np.floor(np.arange(N) / 512))
    return None


def _norm2(a, spec):
    """||A||_2: sigma_1 = 1 by construction, else 40 power iterations (from below,
    raised by 1% for the tolerance scale)."""
    if spec != "gaussian":
        return 1.0
    x = np.random.default_rng(5).standard_normal(a.shape[1])
    s = 0.0
    for _ in range(40):
        y = a.T @ (a @ x)
        s = np.sqrt(np.linalg.norm(y))
        x = y / np.linalg.norm(y)
    return 1.01 * s


@pytest.fixture(scope="module", params=SPECTRA)
def run(request):
    import torch

    import paper_2106_03138_amd as Q
    spec = request.param
    Q.load()
    torch.cuda.set_device(0)
    _say(spec, "generating the input on the GPU")
    a0 = I.device_matrix(N, spec, 0, torch)
    torch.cuda.synchronize()
    a = Q.host_matrix(a0)
    A = torch.empty_like(a0.t().contiguous()).t()
    tau_h = torch.empty(N, dtype=torch.float64, device="cuda")
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    kw = dict(tau=TAU, delta=DELTA, kmax=KMAX, stop_rule=Q.STOP_NONE, precision=Q.PREC_FP64,
              tau_house=tau_h, perm=perm)
    _say(spec, "qrdm_factor as the benchmark calls it")
    A.copy_(a0)
    out = Q.qrdm_factor(A, **kw)
    torch.cuda.synchronize()
    bench = dict(qr=Q.host_matrix(A), tau=tau_h.cpu().numpy(), perm=perm.cpu().numpy(), rank=out.rank)
    _say(spec, f"rank {out.rank}; qrdm_factor with the block log")
    A.copy_(a0)
    out2 = Q.qrdm_factor(A, log=True, **kw)
    torch.cuda.synchronize()
    logged = dict(qr=Q.host_matrix(A), tau=tau_h.cpu().numpy(), perm=perm.cpu().numpy(), rank=out2.rank,
                  blocks=out2.blocks)
    _say(spec, "qrdm_factor in mixed precision")
    A.copy_(a0)
    kw["precision"] = Q.PREC_MIXED
    out3 = Q.qrdm_factor(A, **kw)
    torch.cuda.synchronize()
    mixed = dict(qr=Q.host_matrix(A), tau=tau_h.cpu().numpy(), perm=perm.cpu().numpy(), rank=out3.rank)
    del A, a0
    torch.cuda.empty_cache()
    t0 = time.time()
    _say(spec, "oracle")
    ref = oracle.qrdm(a, tau=TAU, delta=DELTA, kmax=KMAX, stop_rule=oracle.STOP_NONE)
    _say(spec, f"oracle done in {time.time() - t0:.1f} s; rank {ref.rank}")
    return dict(spec=spec, a=a, bench=bench, logged=logged, mixed=mixed, ref=ref)


def test_log_run_same_bits(run):
    g, b = run["logged"], run["bench"]
    hand = [x[0] for x in g["blocks"] if x[4]]  # the hand-over to column pivoting
    if run["spec"] == "gaussian":
        assert hand == []  # full rank: the partial norms never reach the noise level
    else:
        assert len(hand) == 1 and hand[0] > N // 2
        _say(run["spec"], f"switch to scalar pivoting at column {hand[0]}")
    assert np.array_equal(g["perm"], b["perm"]) and np.array_equal(g["tau"], b["tau"])
    assert np.array_equal(g["qr"], b["qr"]) and g["rank"] == b["rank"]


def test_invariants_at_full_size(run):
    spec = run["spec"]
    _say(spec, "invariants")
    g = run["logged"]
    qr, blocks = g["qr"], g["blocks"]
    V.check_reflectors(qr, g["tau"], N)
    V.check_reflectors(run["bench"]["qr"], run["bench"]["tau"], N)
    for out in (g, run["bench"]):
        assert sorted(out["perm"].tolist()) == list(range(N))
    starts = V.check_blocks(qr, blocks, TAU, DELTA, N)
    assert sum(1 for b in blocks if b[3] > 1) >= 50  # the DM blocks of the well-conditioned part
    r, margin = V.paper_rule_rank(qr, np.linalg.norm(run["a"], axis=0).max(), starts)
    _say(spec, f"rank {g['rank']} from the GPU's own R {r} (margin {margin:.2e})")
    if margin > 1e-6:
        assert g["rank"] == r


def test_dm_replay_to_column_n(run):
    """Algorithm 1 replayed at every block start of the GPU's factorization, past
    the first low-margin decision, to the last column."""
    spec = run["spec"]
    g = run["logged"]
    a = run["a"]
    amax = float(np.linalg.norm(a, axis=0).max())
    nu = NU_SCALE * EPS * float(np.linalg.norm(a))
    t0 = time.time()
    res = V.check_dm_replay(g["qr"], g["blocks"], TAU, DELTA, KMAX, amax, nu)
    _say(spec, f"replay in {time.time() - t0:.1f} s: {res}")
    assert res["blocks"] >= 50
    last = max(b[0] + b[3] for b in g["blocks"] if b[3] > 0)
    switch = res["switch"]
    if spec == "gaussian":
        assert switch is None and last == N  # DM blocks to the last column
    else:
        assert switch is not None and last == switch  # DM blocks up to the switch, single pivots after


@pytest.mark.parametrize("which", ["bench", "logged"])
def test_oracle_parity_at_full_size(run, which):
    spec = run["spec"]
    g, ref = run[which], run["ref"]
    _say(spec, f"comparing the {which} run with the oracle")
    cols = np.random.default_rng(1).choice(N, 64, replace=False)
    blocks = [b[:5] for b in g.get("blocks", [])]
    sig = _sigma(spec) if (spec == "geometric" and which == "bench") else None
    out = compare(run["a"], ref, g["qr"], g["tau"], g["perm"], g["rank"], blocks, full=True,
                  residual_cols=cols, check_blocks=which == "logged", norm2=_norm2(run["a"], spec),
                  stop_rule=oracle.STOP_NONE, kmax=KMAX, sigma=sig)
    cut = out["ns_cut"]
    _say(spec, f"R diagonal against the oracle's (entries >= 1e-3 ||A||): relative {out.get('diag_rel')}, "
               f"{out.get('diag_eps')} eps ||A||_2")
    _say(spec, f"exact prefix ns_cut = {cut} (ended by {out.get('cut_by')}); rank gpu {g['rank']} oracle "
               f"{ref.rank} band {out['rank_band']}; sigma_min(R11)/sigma_r {out.get('smin_ratio')} at n_r = "
               f"{out.get('n_r')}")
    if spec == "gaussian":
        assert cut == N  # every decision of the factorization is clear of the rounding noise
    else:
        # Householder QR is normwise stable: the trailing entries of two correct
        # runs differ by about eps ||A||, so decisions among partial norms far
        # above that agree.  The exact prefix reaches at least the first column
        # whose singular value is below 1e-6 sigma_1.
        floor = int(np.argmax(_sigma(spec) < 1e-6))
        assert cut >= floor, (cut, floor)
    if sig is not None:
        ro, rg = out["smin_ratio"][1], out["smin_ratio"][0]
        assert 0.1 <= rg <= 10.0 and 0.1 <= ro <= 10.0, out["smin_ratio"]


def test_mixed_precision_error_at_full_size(run):
    """Mixed precision (FP32 MFMA trailing updates) against the FP64 oracle on the
    same matrix: the backward error is at the FP32 level, the sorted R diagonal
    (d_i, Section 5) differs from the oracle's by FP32 rounding of the updates
    relative to ||A||, and below the FP32 noise floor the diagonal is noise of
    that size; the error is reported."""
    spec = run["spec"]
    g, ref, a = run["mixed"], run["ref"], run["a"]
    na = _norm2(a, spec)
    cols = np.random.default_rng(1).choice(N, 64, replace=False)
    from oracle import metrics as M
    res = M.sampled_residual(a, g["qr"], g["tau"], g["perm"], N, cols)
    dg = np.sort(np.abs(np.diag(g["qr"])))[::-1]
    do = np.sort(np.abs(np.diag(ref.qr)))[::-1]
    gap = float(np.max(np.abs(dg - do)) / na)
    sig = _sigma(spec)
    msg = f"mixed: rank {g['rank']}, residual {res:.2e}, max |d_i - d_i(oracle)| / ||A|| = {gap:.2e}"
    if sig is not None:
        nr32 = int(np.sum(sig > N * 2.0 ** -23 * sig[0]))
        d = dg[:nr32] / sig[:nr32]
        msg += f"; d_i/sigma_i over the {nr32} values above n 2^-23 sigma_1: [{d.min():.4g}, {d.max():.4g}]"
    _say(spec, msg)
    assert sorted(g["perm"].tolist()) == list(range(N))
    assert res <= 1e-5
    assert gap <= 1e-4
