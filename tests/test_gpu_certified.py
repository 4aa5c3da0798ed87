"""Certified DM mode (eq. delta_max) and the Lemma 1 record per block on the
GPU against the oracle, and the lemma itself checked on the GPU's blocks."""
import numpy as np
import pytest

import oracle
from paper_2106_03138_amd import inputs as I
from parity import ETA, compare

pytestmark = pytest.mark.gpu


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


def _matrices():
    rng = np.random.default_rng(12)
    base = rng.standard_normal((400, 8))
    corr = np.asfortranarray(rng.standard_normal((400, 300)) + 0.3 * base @ rng.standard_normal((8, 300)))
    return {"rank64": I.small_rank64(6), "correlated": corr, "half_rank": I.half_rank_noise(512, 4),
            "orthogonal": I.orthogonal_columns(200, np.geomspace(1, 1e-3, 120), 7)[0]}


@pytest.mark.parametrize("certified", [True, False])
@pytest.mark.parametrize("name", ["rank64", "correlated", "half_rank", "orthogonal"])
def test_block_records_match_oracle(name, certified):
    """Pivots, blocks and rank as the oracle's; gamma and sigma_bound of every
    block before the first low-margin decision agree to rounding (both come
    from Gram matrices summed in different orders)."""
    Q = _gpu()
    a = _matrices()[name]
    kw = dict(tau=0.5, delta=0.9, kmax=64) if name == "correlated" else {}
    ref = oracle.qrdm(a, certified=certified, **kw)
    A = Q.device_matrix(a)
    out = Q.qrdm_factor(A, certified=certified, log=True, poll_lag=0, **kw)
    compare(a, ref, Q.host_matrix(A), out.tau_house.cpu().numpy(), out.perm.cpu().numpy(), out.rank, out.blocks,
            kmax=kw.get("kmax", 64))
    k = ref.first_low_margin_block(ETA)
    real = [b for b in ref.blocks if b.l > 0]
    tau = kw.get("tau", 0.15)
    # the two implementations update the trailing columns in different orders,
    # so those columns differ by nu ~ eps ||A|| (absolute); a cosine of columns
    # of norm >= tau * umax then differs by about nu / (tau umax), gamma by k_s
    # such terms, and bound^2 = slack * max||c_j||^2 by a few of them
    nu = 100 * np.finfo(float).eps * np.linalg.norm(a, 2)
    for i in range(min(k, len(real), len(out.blocks))):
        g, r = out.blocks[i], real[i]
        if r.fallback or r.umax == 0.0:
            continue
        rel = nu / (tau * r.umax)
        tol_g = 1e-12 + r.ks * rel
        assert abs(g[5] - r.gamma) <= tol_g, (i, g[5], r.gamma, tol_g)
        tol_b2 = (4 * tol_g + 4 * rel) * (1.1 * r.umax) ** 2
        assert abs(g[6] ** 2 - r.sigma_bound ** 2) <= tol_b2, (i, g[6], r.sigma_bound)
        if certified:
            assert g[6] > 0.0, i


@pytest.mark.parametrize("seed", range(3))
def test_first_block_bound_holds_on_gpu_output(seed):
    """Lemma 1 on the GPU's first block: sigma_min of the accepted input
    columns (library SVD) is at least the recorded bound."""
    Q = _gpu()
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((300, 5))
    a = np.asfortranarray(rng.standard_normal((300, 200)) + 0.4 * base @ rng.standard_normal((5, 200)))
    A = Q.device_matrix(a)
    out = Q.qrdm_factor(A, tau=0.4, certified=True, log=True, poll_lag=0)
    ks, gamma, bound = out.blocks[0][2], out.blocks[0][5], out.blocks[0][6]
    perm = out.perm.cpu().numpy()
    c = a[:, perm[:ks]]
    smin = np.linalg.svd(c, compute_uv=False)[-1]
    assert 0.0 < bound <= smin * (1 + 1e-12)
    th = c.T @ c / np.outer(np.linalg.norm(c, axis=0), np.linalg.norm(c, axis=0))
    if ks > 1:
        assert np.max(np.abs(th[~np.eye(ks, dtype=bool)])) < 0.16 / (out.blocks[0][1] - 1) + 1e-15
        assert gamma > 1 - 0.16


def test_batched_certified_matches_oracle():
    import torch
    Q = _gpu()
    shapes = I.batch_shapes(24, seed=17, mmin=8, mmax=200, nmin=1)
    seqs = np.random.SeedSequence(17).spawn(len(shapes))
    mats = [I.batch_matrix(m, n, r, s) for (m, n, r), s in zip(shapes, seqs)]
    mats.append(_matrices()["rank64"])
    b = Q.Batch([a.shape for a in mats])
    b.load(mats)
    plan = Q.BatchPlan(b, certified=True)
    plan.factor()
    torch.cuda.synchronize()
    rank = b.rank.cpu().numpy()
    for i, a in enumerate(mats):
        ref = oracle.qrdm(a, certified=True)
        compare(a, ref, b.matrix(i), b.tau_house(i), b.permutation(i), int(rank[i]), [], check_blocks=False)
    plan.close()
