"""The (tau, delta) grid study (paper_2106_03138_amd/grid.py) on a small grid,
with the corners tau = 0 and delta in {0, 1}: every grid point's batched
factorization against the oracle's, and the tabulated ratio against the
ratio recomputed from the GPU's own R."""
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


def test_small_grid_matches_oracle():
    import torch
    Q = _gpu()
    from paper_2106_03138_amd import grid as G
    mats, shapes, sigmas, kinds = I.training_batch(8, seed=3, mmin=16, mmax=120, nmin=4)
    taus, deltas = [0.0, 0.15, 0.5], [0.0, 0.9, 1.0]
    rep = G.run_grid(mats, sigmas, taus=taus, deltas=deltas, verbose=False)
    ratio = np.array(rep["ratio"])
    assert ratio.shape == (3, 3) and np.all(np.array(rep["ms"]) > 0)
    for jt, t in enumerate(taus):
        for idl, d in enumerate(deltas):
            b = Q.Batch([a.shape for a in mats])
            b.load(mats)
            plan = Q.BatchPlan(b, tau=t, delta=d, stop_rule=oracle.STOP_NONE)
            plan.factor()
            torch.cuda.synchronize()
            rk = b.rank.cpu().numpy()
            got = []
            for i, a in enumerate(mats):
                ref = oracle.qrdm(a, tau=t, delta=d, stop_rule=oracle.STOP_NONE)
                compare(a, ref, b.matrix(i), b.tau_house(i), b.permutation(i), int(rk[i]), [],
                        check_blocks=False, full=True, stop_rule=oracle.STOP_NONE, kmax=64)
                got.append(G.min_ratio(np.diag(b.matrix(i)), sigmas[i], a.shape[1]))
            assert ratio[jt, idl] == min(got), (t, d)
            plan.close()


def test_tau_zero_single_matches_oracle():
    Q = _gpu()
    a = I.orthogonal_columns(300, np.geomspace(1.0, 1e-6, 150), 8)[0]
    for d in (0.0, 0.5, 1.0):
        ref = oracle.qrdm(a, tau=0.0, delta=d, stop_rule=oracle.STOP_NONE)
        A = Q.device_matrix(a)
        out = Q.qrdm_factor(A, tau=0.0, delta=d, stop_rule=oracle.STOP_NONE, log=True, poll_lag=0)
        compare(a, ref, Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank,
                out.blocks, full=True, stop_rule=oracle.STOP_NONE, kmax=64)
