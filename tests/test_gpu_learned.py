"""Learned-parameter predictor on the GPU against its oracle (oracle/learned.py)."""
import numpy as np
import pytest

import oracle
from oracle import learned as Lr
from paper_2106_03138_amd import inputs as I
from parity import compare

pytestmark = pytest.mark.gpu


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


def _mats(seed=21, count=20):
    shapes = I.batch_shapes(count, seed=seed, mmin=8, mmax=300, nmin=1)
    seqs = np.random.SeedSequence(seed).spawn(len(shapes))
    mats = [I.batch_matrix(m, n, r, s) for (m, n, r), s in zip(shapes, seqs)]
    rng = np.random.default_rng(seed)
    mats += [np.zeros((9, 5), order="F"), I.rank1(30, 20, 2), np.asfortranarray(rng.standard_normal((1, 6))),
             np.asfortranarray(rng.standard_normal((12, 1))), np.asfortranarray(rng.standard_normal((20, 60))),
             I.orthogonal_columns(100, np.geomspace(1, 1e-5, 70), 1)[0],
             np.asfortranarray(rng.standard_normal((512, 512)))]
    return mats


def _plan(mats, **kw):
    Q = _gpu()
    b = Q.Batch([a.shape for a in mats])
    b.load(mats)
    return b, Q.BatchPlan(b, **kw)


def test_features_match_oracle():
    import torch
    mats = _mats()
    b, plan = _plan(mats)
    f = plan.features().cpu().numpy()
    for i, a in enumerate(mats):
        ref = Lr.features(a)
        # order statistics and shape features: the same values; cosine statistics:
        # Gram sums in another order, so the values agree to rounding
        np.testing.assert_allclose(f[i, :12], ref[:12], rtol=1e-13, atol=1e-13, err_msg=f"matrix {i} {a.shape}")
        np.testing.assert_allclose(f[i, 12:], ref[12:], rtol=1e-12, atol=1e-12, err_msg=f"matrix {i} {a.shape}")


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def test_mlp_forward_gradient_adam_match_oracle():
    import torch
    Q = _gpu()
    rng = np.random.default_rng(4)
    theta = _f32(rng.standard_normal(Lr.NPARAM) * 0.2)
    feats = rng.standard_normal((37, 16)) * 3.0
    norm = _f32(np.concatenate([rng.standard_normal(16), np.exp(rng.uniform(-1, 1, 16))]))
    target = _f32(rng.standard_normal((37, 3)))
    x = (_f32(feats) - norm[:16]) * norm[16:]
    P = torch.as_tensor(theta.astype(np.float32)).cuda()
    N = torch.as_tensor(norm.astype(np.float32)).cuda()
    F = torch.as_tensor(feats).cuda()
    T = torch.as_tensor(target.astype(np.float32)).cuda()
    y = Q.mlp_forward(P, F, N).cpu().numpy()
    yref, _ = Lr.mlp_forward(theta, x)
    np.testing.assert_allclose(y, yref, rtol=2e-5, atol=2e-5)
    g, _, sq = Q.mlp_gradient(P, F, T, N)
    gref = Lr.mlp_grad(theta, x, target)
    g = g.cpu().numpy()
    assert np.max(np.abs(g - gref)) <= 1e-4 * max(1.0, np.max(np.abs(gref)))
    np.testing.assert_allclose(sq.cpu().numpy(), np.sum((yref - target) ** 2, axis=1), rtol=1e-4, atol=1e-5)
    # one Adam step at t = 3 from given moments
    m0 = _f32(rng.standard_normal(Lr.NPARAM) * 0.01)
    v0 = _f32(np.abs(rng.standard_normal(Lr.NPARAM)) * 1e-4)
    G = torch.as_tensor(_f32(gref).astype(np.float32)).cuda()
    M = torch.as_tensor(m0.astype(np.float32)).cuda()
    V = torch.as_tensor(v0.astype(np.float32)).cuda()
    Q.mlp_adam(P, G, M, V, 3, lr=1e-3)
    # the kernel holds the hyperparameters in FP32 (1 - 0.999 differs from 1e-3
    # by 1.3e-5 relative there), so the oracle takes the same rounded values
    tref, mref, vref = Lr.adam_step(theta, _f32(gref), m0, v0, 3, lr=float(_f32(1e-3)), b1=float(_f32(0.9)),
                                    b2=float(_f32(0.999)), eps=float(_f32(1e-8)))
    # FP32 arithmetic: absolute errors of a few units of 2^-24 times the
    # operands (|m| + 0.1 |g| <= 0.1, |v| + 0.001 g^2 <= 1e-3, |theta| <= 1)
    np.testing.assert_allclose(P.cpu().numpy(), tref, rtol=1e-6, atol=2e-7)
    np.testing.assert_allclose(M.cpu().numpy(), mref, rtol=1e-6, atol=3e-8)
    np.testing.assert_allclose(V.cpu().numpy(), vref, rtol=1e-6, atol=3e-10)


def test_mlp_to_params_nearest_grid_point():
    import torch
    Q = _gpu()
    ys = np.array([[0.0, 0.0, 0.0], [0.1, 0.6, 0.49], [0.23, 0.81, 0.5], [0.61, 0.93, 2.0], [5.0, 5.0, -1.0],
                   [0.4, 0.92, 0.51], [0.26, 0.79, 0.7]], dtype=np.float32)
    out = Q.mlp_to_params(torch.as_tensor(ys).cuda()).cpu().numpy()
    rec = out.view(np.dtype([("tau", "<f8"), ("delta", "<f8"), ("kmax", "<i4"), ("pad", "<i4")]))
    taus, deltas = np.array([0.05, 0.15, 0.3, 0.5, 0.7, 0.9]), np.array([0.5, 0.7, 0.9, 0.95])
    for i, y in enumerate(ys.astype(np.float64)):
        # nearest value by definition; ties go to the smaller grid value
        assert rec["tau"][i] == taus[np.argmin(np.abs(taus - y[0]))]
        assert rec["delta"][i] == deltas[np.argmin(np.abs(deltas - y[1]))]
        assert rec["kmax"][i] == (64 if y[2] >= 0.5 else 32)


def test_condition_check_matches_oracle():
    mats = _mats(seed=23, count=16)
    b, plan = _plan(mats)
    plan.factor()
    ok, est = plan.check(0.1)
    ok, est = ok.cpu().numpy(), est.cpu().numpy()
    rank = b.rank.cpu().numpy()
    for i, a in enumerate(mats):
        r = int(rank[i])
        if r == 0:
            assert ok[i] == 1
            continue
        R = np.triu(b.matrix(i)[:r, :r])
        ref = Lr.ice_sigma_min(R)
        # the dot products sum in another order; the estimate is a sequence of
        # such steps, so it agrees to rounding relative to the largest |r_jj|
        scale = np.max(np.abs(np.diag(R)))
        assert abs(est[i] - ref) <= 1e-12 * scale + 1e-8 * ref, (i, est[i], ref)
        thr = 0.1 * np.min(np.abs(np.diag(R)))
        if abs(ref - thr) > 1e-8 * max(ref, thr) + 1e-12 * scale:
            assert ok[i] == int(ref >= thr), i


def test_predict_factor_fallback_equals_default():
    """With a band no estimate can meet, every matrix is factored again with the
    defaults: the result equals a plain default factorization bit for bit."""
    import torch
    Q = _gpu()
    from paper_2106_03138_amd import learned as Ld
    mats = _mats(seed=25, count=12)
    b, plan = _plan(mats)
    pristine = b.data.clone()
    model = Ld.Model(I.mlp_init(3), np.concatenate([np.zeros(16), np.ones(16)]))
    _, nfb = Ld.predict_factor(b, plan, model, pristine, band=1e300)
    torch.cuda.synchronize()
    got = (b.data.clone(), b.rank.clone(), b.perm.clone())
    b2, plan2 = _plan(mats)
    plan2.factor()
    torch.cuda.synchronize()
    nz = sum(1 for a in mats if min(a.shape) > 0 and np.any(a))
    assert nfb >= nz
    assert torch.equal(got[0], b2.data) and torch.equal(got[1], b2.rank) and torch.equal(got[2], b2.perm)


def test_checked_factor_matches_separate_launches():
    """The checked launch (factorization with the predicted parameters, the
    online check, and the re-run of the failures with the plan's parameters, all
    in one launch) equals the same steps as separate launches: factor with the
    predictions, qrdm_batch_check, then the failures restored and factored again
    with per-matrix parameters that leave every other matrix as it is (k_DM = 0).
    Bit for bit, and the same failures."""
    import torch
    Q = _gpu()
    from paper_2106_03138_amd import learned as Ld
    mats = _mats(seed=29, count=24)
    mats += [I.batch_matrix(200, 150, 140, np.random.SeedSequence(5)),
             I.from_spectrum(300, 280, np.geomspace(1.0, 1e-15, 280), 6)]
    model = Ld.Model(I.mlp_init(7) * 3.0, np.concatenate([np.zeros(16), np.ones(16)]))
    for band in (0.1, 0.5):
        b, plan = _plan(mats)
        pristine = b.data.clone()
        pm = Ld.predict_params(plan, model)
        ok = plan.factor_checked(pm, b.pointers(pristine), band)
        torch.cuda.synchronize()
        got = (b.data.clone(), b.rank.clone(), b.perm.clone(), b.tau.clone(), ok.clone())
        # the same steps as separate launches
        b2, plan2 = _plan(mats)
        plan2.factor(params=pm)
        ok2, _ = plan2.check(band)
        bad = torch.nonzero(ok2 == 0).flatten()
        if len(bad):
            for i in bad.cpu().numpy():
                s0, s1 = int(b2.off[i]), int(b2.off[i + 1])
                b2.data[s0:s1].copy_(pristine[s0:s1])
            pm2 = torch.zeros_like(pm)
            f64, i32 = pm2.view(torch.float64).view(-1, 3), pm2.view(torch.int32).view(-1, 6)
            t, d, k = Ld.DEFAULT
            f64[bad, 0] = t
            f64[bad, 1] = d
            i32[bad, 4] = k
            plan2.factor(params=pm2)
        torch.cuda.synchronize()
        print(f"[checked] band {band}: {len(bad)} of {len(mats)} factored again", flush=True)
        assert torch.equal(got[4], ok2)
        assert torch.equal(got[0], b2.data) and torch.equal(got[1], b2.rank)
        assert torch.equal(got[2], b2.perm) and torch.equal(got[3], b2.tau)


def test_predicted_parameters_match_oracle_factorization():
    """Each matrix factored with its predicted (tau, delta, k_DM) equals the
    oracle's factorization with those parameters."""
    import torch
    Q = _gpu()
    from paper_2106_03138_amd import learned as Ld
    mats = _mats(seed=27, count=12)
    b, plan = _plan(mats)
    model = Ld.Model(I.mlp_init(5) * 3.0, np.concatenate([np.zeros(16), np.ones(16)]))
    pm = Ld.predict_params(plan, model)
    plan.factor(params=pm)
    torch.cuda.synchronize()
    rec = pm.cpu().numpy().view(np.dtype([("tau", "<f8"), ("delta", "<f8"), ("kmax", "<i4"), ("pad", "<i4")]))
    rank = b.rank.cpu().numpy()
    for i, a in enumerate(mats):
        if min(a.shape) == 0 or not np.any(a):
            continue
        ref = oracle.qrdm(a, tau=float(rec["tau"][i]), delta=float(rec["delta"][i]), kmax=int(rec["kmax"][i]))
        compare(a, ref, b.matrix(i), b.tau_house(i), b.permutation(i), int(rank[i]), [], check_blocks=False,
                kmax=int(rec["kmax"][i]))


def test_training_steps_follow_the_oracle():
    """Five Adam steps with the GPU kernels track the FP64 oracle from the same
    initial parameters and minibatches (eps = 1e-3, so that rounding noise in
    gradients near zero is not normalized up to a full step)."""
    import torch
    Q = _gpu()
    mats = _mats(seed=29, count=40)
    b, plan = _plan(mats)
    F = plan.features()
    fh = F.cpu().numpy()
    rng = np.random.default_rng(2)
    y = _f32(rng.uniform(0, 1, (len(mats), 3)))
    mu, sd = fh.mean(axis=0), fh.std(axis=0)
    norm = _f32(np.concatenate([mu, np.where(sd > 1e-12, 1 / np.maximum(sd, 1e-12), 0.0)]))
    theta = _f32(I.mlp_init(1))
    P = torch.as_tensor(theta.astype(np.float32)).cuda()
    N = torch.as_tensor(norm.astype(np.float32)).cuda()
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    T = torch.as_tensor(y.astype(np.float32)).cuda()
    th, mo, ve = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    x = (_f32(fh) - norm[:16]) * norm[16:]
    for t in range(1, 6):
        sel = np.arange((t - 1) * 8, t * 8) % len(mats)
        g, _, _ = Q.mlp_gradient(P, F[torch.as_tensor(sel).cuda()], T[torch.as_tensor(sel).cuda()], N)
        Q.mlp_adam(P, g, M, V, t, lr=1e-2, eps=1e-3)
        th, mo, ve = Lr.adam_step(th, Lr.mlp_grad(th, x[sel], y[sel]), mo, ve, t, lr=float(_f32(1e-2)),
                                  b1=float(_f32(0.9)), b2=float(_f32(0.999)), eps=float(_f32(1e-3)))
    np.testing.assert_allclose(P.cpu().numpy(), th, rtol=1e-4, atol=2e-5)
