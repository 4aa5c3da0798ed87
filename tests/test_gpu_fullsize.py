"""Parity at the benchmark's full size and launch configuration: 8192 x 8192,
singular values geometric from 1 to 1e-16 (the Section 5 test family at its
largest size), tau = 0.15, delta = 0.9, k_DM = 64, stopping criterion off (full
factorization), FP64, the library's default stream, preallocated tau and perm as
the benchmark passes them.

Checks:
- the oracle on the same matrix: permutation identical up to the first block with
  a decision margin below 1e-10, R normwise and its diagonal relatively on that
  prefix, the rank, and the backward error estimated from 64 sampled columns of AP
  (applying Q^T to all of AP is too slow on the host);
- the properties that hold at any size, read off the GPU's R (tests/invariants.py):
  Algorithm 1's candidate and greedy rules for every logged block, the single-pivot
  rule on the scalar-pivoting tail, the practical stopping criterion's rank, and the
  orthogonality of every reflector;
- both runs, the benchmark's and one with the block log.  The log makes the host
  wait on every step (no poll lag), so the launch bounds differ; the kernels take
  their splits from the actual sizes, so the two runs agree to the bit in every
  column: the switch to scalar pivoting is taken on the device, so the
  column-pivoting kernels start at the same column in both runs.  Each run is
  also compared with the oracle on its own.
"""
import time

import numpy as np
import pytest

import invariants as V
import oracle
from parity import compare
from paper_2106_03138_amd import inputs as I

N = 8192
TAU, DELTA, KMAX = 0.15, 0.9, 64

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[fullsize {N}x{N} geometric seed 0] {msg}", flush=True)


@pytest.fixture(scope="module")
def run():
    import torch

    import paper_2106_03138_amd as Q
    Q.load()
    torch.cuda.set_device(0)
    _say("generating the input on the GPU")
    a0 = I.device_matrix(N, "geometric", 0, torch)
    torch.cuda.synchronize()
    a = Q.host_matrix(a0)
    A = torch.empty_like(a0.t().contiguous()).t()
    tau_h = torch.empty(N, dtype=torch.float64, device="cuda")
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    kw = dict(tau=TAU, delta=DELTA, kmax=KMAX, stop_rule=Q.STOP_NONE, precision=Q.PREC_FP64,
              tau_house=tau_h, perm=perm)
    _say("qrdm_factor as the benchmark calls it")
    A.copy_(a0)
    out = Q.qrdm_factor(A, **kw)
    torch.cuda.synchronize()
    bench = dict(qr=Q.host_matrix(A), tau=tau_h.cpu().numpy(), perm=perm.cpu().numpy(), rank=out.rank)
    _say(f"rank {out.rank}; qrdm_factor with the block log")
    A.copy_(a0)
    out2 = Q.qrdm_factor(A, log=True, **kw)
    torch.cuda.synchronize()
    logged = dict(qr=Q.host_matrix(A), tau=tau_h.cpu().numpy(), perm=perm.cpu().numpy(), rank=out2.rank,
                  blocks=out2.blocks)
    del A, a0
    torch.cuda.empty_cache()
    return dict(a=a, bench=bench, logged=logged)


@pytest.fixture(scope="module")
def ref(run):
    t0 = time.time()
    _say("oracle")
    r = oracle.qrdm(run["a"], tau=TAU, delta=DELTA, kmax=KMAX, stop_rule=oracle.STOP_NONE)
    _say(f"oracle done in {time.time() - t0:.1f} s; rank {r.rank}")
    return r


def test_log_run_same_bits(run):
    g, b = run["logged"], run["bench"]
    fb = next(x[0] for x in g["blocks"] if x[4])  # the hand-over to column pivoting
    assert fb > N // 2
    _say(f"switch to scalar pivoting at column {fb}")
    assert np.array_equal(g["perm"], b["perm"]) and np.array_equal(g["tau"], b["tau"])
    assert np.array_equal(g["qr"], b["qr"]) and g["rank"] == b["rank"]


def test_invariants_at_full_size(run):
    _say("invariants")
    g = run["logged"]
    qr, blocks = g["qr"], g["blocks"]
    V.check_reflectors(qr, g["tau"], N)
    V.check_reflectors(run["bench"]["qr"], run["bench"]["tau"], N)
    for out in (g, run["bench"]):
        assert sorted(out["perm"].tolist()) == list(range(N))
    starts = V.check_blocks(qr, blocks, TAU, DELTA, N)
    assert sum(1 for b in blocks if b[3] > 1) >= 50  # the DM blocks of the well-conditioned part
    r, margin = V.paper_rule_rank(qr, np.linalg.norm(run["a"], axis=0).max(), starts)
    if margin > 1e-6:
        assert g["rank"] == r


@pytest.mark.parametrize("which", ["bench", "logged"])
def test_oracle_parity_at_full_size(run, ref, which):
    g = run[which]
    _say(f"comparing the {which} run with the oracle")
    cols = np.random.default_rng(1).choice(N, 64, replace=False)
    blocks = [b[:4] for b in g.get("blocks", [])]
    compare(run["a"], ref, g["qr"], g["tau"], g["perm"], g["rank"], blocks, full=True,
            residual_cols=cols, check_blocks=which == "logged", norm2=1.0)  # sigma_1 = 1 by construction
    _say("compared")
