"""Learned (tau, delta, k_DM) per matrix for the batched path.

The paper selects (tau, delta) by a grid study and judges the result with the
factor-10 rule d_i / sigma_i >= 0.1 (Section 5).  This module turns that study
into a per-matrix predictor:

  label sweep   every matrix of a training set is factored with each point of
                the grid tau x delta x k_DM (6 x 4 x 2); its label is the point
                with the fewest GPU clock ticks among those that meet the
                factor-10 rule (sigma known by construction), else the default.
  training      the 16 -> 64 -> 64 -> 3 MLP (library kernels: forward,
                gradient, Adam) regresses the label (tau, delta, [k_DM = 64]).
  inference     features -> MLP -> nearest grid point per matrix -> batched
                factorization -> online condition check; a matrix that fails
                the check is factored again with the defaults.

    python -m paper_2106_03138_amd.learned train [--count 4096] [--out FILE]

Every numerical step runs in the library's kernels; this module moves data
between them and keeps the bookkeeping of the sweep.
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import _lib
from . import inputs as I
from .api import Batch, BatchPlan, mlp_adam, mlp_forward, mlp_gradient, mlp_to_params

TAU_GRID = (0.05, 0.15, 0.3, 0.5, 0.7, 0.9)
DELTA_GRID = (0.5, 0.7, 0.9, 0.95)
K_GRID = (32, 64)
DEFAULT = (0.15, 0.9, 64)
HERE = os.path.dirname(os.path.abspath(__file__))


def model_path(device_name: str = "gfx950") -> str:
    return os.environ.get("QRDM_MLP_WEIGHTS", os.path.join(HERE, "tuned", f"mlp_{device_name}.npz"))


class Model:
    """Trained weights (float32 device tensors) and the feature normalization."""

    def __init__(self, params, norm):
        import torch
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).cuda()
        self.norm = torch.as_tensor(np.asarray(norm, dtype=np.float32)).cuda()

    @staticmethod
    def load(path: str | None = None):
        path = path or model_path()
        if not os.path.exists(path):
            return None
        d = np.load(path, allow_pickle=False)
        return Model(d["params"], d["norm"])


# ------------------------------------------------------------------ labels
def factor10_ok(rdiag: np.ndarray, sigma: np.ndarray, n: int, band: float = 0.1) -> bool:
    """Section 5's rule on the first n_r = #{sigma_i > eps n sigma_1} values."""
    if len(sigma) == 0 or sigma[0] == 0:
        return True
    nr = int(np.sum(sigma > np.finfo(np.float64).eps * n * sigma[0]))
    if nr == 0:
        return True
    d = np.sort(np.abs(rdiag[:nr]))[::-1]
    return bool(np.min(d / sigma[:nr]) >= band)


def _diag_index(batch: Batch):
    idx = []
    for i, (m, n) in enumerate(batch.shapes):
        p = min(m, n)
        off, ld = int(batch.off[i]), batch.lda[i]
        idx.append(off + np.arange(p) * (ld + 1))
    return idx


def sweep(mats, shapes, sigmas, verbose: bool = True):
    """Ticks and factor-10 verdict of every matrix at every grid point.
    Returns (configs [G, 3], ticks [G, B], ok [G, B])."""
    import torch
    b = Batch([(m, n) for m, n, _ in shapes])
    b.load(mats)
    pristine = b.data.clone()
    info = torch.zeros(4 * len(mats), dtype=torch.int64, device="cuda")
    didx = _diag_index(b)
    flat = torch.as_tensor(np.concatenate(didx)).cuda()
    cuts = np.cumsum([0] + [len(x) for x in didx])
    configs = [(t, d, k) for t in TAU_GRID for d in DELTA_GRID for k in K_GRID]
    ticks = np.zeros((len(configs), len(mats)), dtype=np.int64)
    ok = np.zeros((len(configs), len(mats)), dtype=bool)
    for g, (t, d, k) in enumerate(configs):
        b.data.copy_(pristine)
        plan = BatchPlan(b, tau=t, delta=d, kmax=k)
        plan.factor(info=info)
        torch.cuda.synchronize()
        ticks[g] = info.view(-1, 4)[:, 3].cpu().numpy()
        diag = b.data[flat].cpu().numpy()
        for i, (m, n, _) in enumerate(shapes):
            ok[g, i] = factor10_ok(diag[cuts[i]: cuts[i + 1]], sigmas[i], n)
        plan.close()
        if verbose:
            print(f"sweep {g + 1}/{len(configs)} tau {t} delta {d} k {k}: ticks {ticks[g].sum() / 1e5:.1f} ms-WG, "
                  f"factor-10 ok {ok[g].mean():.3f}", flush=True)
    return np.array(configs, dtype=np.float64), ticks, ok


def labels_from_sweep(configs, ticks, ok):
    """Per matrix: the fastest configuration that meets the rule (default if none)."""
    big = np.where(ok, ticks, np.iinfo(np.int64).max)
    best = np.argmin(big, axis=0)
    none = ~ok.any(axis=0)
    lab = configs[best].copy()
    lab[none] = DEFAULT
    return lab


def targets(lab):
    """Regression targets: (tau, delta, 1 if k_DM = 64 else 0)."""
    return np.stack([lab[:, 0], lab[:, 1], (lab[:, 2] >= 64).astype(np.float64)], axis=1)


# ---------------------------------------------------------------- training
def train(features, y, epochs: int = 300, batch: int = 256, lr: float = 3e-3, seed: int = 0, verbose: bool = True):
    """Adam on the squared loss with the library's kernels.  features [N, 16]
    float64 device tensor, y [N, 3] host array.  Returns (params, norm, losses)."""
    import torch
    fh = features.cpu().numpy()
    mu = fh.mean(axis=0)
    sd = fh.std(axis=0)
    inv = np.where(sd > 1e-12, 1.0 / np.maximum(sd, 1e-12), 0.0)
    norm = torch.as_tensor(np.concatenate([mu, inv]).astype(np.float32)).cuda()
    params = torch.as_tensor(I.mlp_init(seed).astype(np.float32)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    yt = torch.as_tensor(y.astype(np.float32)).cuda()
    n = fh.shape[0]
    rng = np.random.default_rng(seed)
    t = 0
    losses = []
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(n)).cuda()
        tot = 0.0
        for s0 in range(0, n, batch):
            sel = order[s0: s0 + batch]
            g, _, sq = mlp_gradient(params, features[sel], yt[sel], norm)
            t += 1
            mlp_adam(params, g, m, v, t, lr=lr)
            tot += float(sq.sum())
        losses.append(0.5 * tot / n)
        if verbose and (ep % 50 == 0 or ep == epochs - 1):
            print(f"epoch {ep}: loss {losses[-1]:.5f}", flush=True)
    return params.cpu().numpy(), norm.cpu().numpy(), losses


# ---------------------------------------------------------------- inference
def predict_params(plan: BatchPlan, model: Model):
    """Per-matrix parameters (device qrdm_batch_params array) for the plan's batch."""
    feats = plan.features()
    y = mlp_forward(model.params, feats, model.norm)
    return mlp_to_params(y)


def predict_factor(batch: Batch, plan: BatchPlan, model: Model, pristine, band: float = 0.1,
                   use_graph: bool = False, breakdown: dict = None, pristine_ptrs=None):
    """Predicted parameters, then the factorization with the online check in the
    same launch: a matrix that fails the check is factored again with the
    defaults (the plan's parameters) by its own workgroup.
    pristine: a copy of batch.data before the call (the factorization is in
    place); pristine_ptrs: batch.pointers(pristine), made here when not given.
    use_graph is accepted for the caller's convenience; the checked launch is
    not captured.
    breakdown: when a dict, the device is synchronized after each stage and the
    stage times (ms) are stored in it, with the factorization's per-matrix
    clock ticks ("ticks": int64 device tensor).
    Returns (params, number of matrices factored again)."""
    import torch
    clock = [time.perf_counter()]

    def stage(name):
        if breakdown is not None:
            torch.cuda.synchronize()
            now = time.perf_counter()
            breakdown[name] = 1e3 * (now - clock[0])
            clock[0] = now

    if breakdown is not None:
        torch.cuda.synchronize()
        clock[0] = time.perf_counter()
    pm = predict_params(plan, model)
    stage("features_mlp_snap_ms")
    info = torch.zeros(4 * max(len(batch), 1), dtype=torch.int64, device="cuda") if breakdown is not None else None
    ptrs = pristine_ptrs if pristine_ptrs is not None else batch.pointers(pristine)
    ok = plan.factor_checked(pm, ptrs, band, info=info)
    stage("factor_check_rerun_ms")
    if info is not None:
        breakdown["ticks"] = info.view(-1, 4)[:, 3]
    return pm, int((ok == 0).sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    _lib.load()
    t0 = time.time()
    mats, shapes, sigmas, kinds = I.training_batch(args.count, seed=args.seed)
    print(f"training set: {len(mats)} matrices ({time.time() - t0:.1f} s)", flush=True)
    configs, ticks, ok = sweep(mats, shapes, sigmas)
    lab = labels_from_sweep(configs, ticks, ok)
    b = Batch([(m, n) for m, n, _ in shapes])
    b.load(mats)
    plan = BatchPlan(b)
    feats = plan.features()
    torch.cuda.synchronize()
    params, norm, losses = train(feats, targets(lab), epochs=args.epochs)
    out = args.out or model_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    dflt = configs.tolist().index(list(DEFAULT))
    np.savez(out, params=params, norm=norm, losses=np.array(losses), label_tau=lab[:, 0], label_delta=lab[:, 1],
             label_k=lab[:, 2], ticks=ticks, ok=ok, configs=configs)
    lab_ticks = np.array([ticks[configs.tolist().index(list(l)), i] for i, l in enumerate(lab)])
    print(f"saved {out}; sum of ticks at the labels / at the default: "
          f"{lab_ticks.sum() / max(ticks[dflt].sum(), 1):.3f}; labels meeting the rule at default: "
          f"{ok[dflt].mean():.3f}", flush=True)


if __name__ == "__main__":
    main()
