"""Parameter study of Section 5 on the GPU path: the (tau, delta) grid of
Fig. 3 and the block size k_DM, with synthetic stand-ins for the paper's
matrix collections.

  grid   G(i, j) = (delta_i, tau_j) = (0.05 i, 0.05 j), i, j = 0..20.  Every
         matrix of a batch is factored to the end (no stopping criterion, as
         the grid study reads the whole R factor) by the batched path at each
         grid point; per point the report holds the minimum over the matrices
         of min_{i < n_r} |r_ii| / sigma_i (Fig. 3a; n_r = #{sigma_i > eps n
         sigma_1}) and the GPU time of the whole batch (Fig. 3b).
  k_DM   the single-matrix path at k_DM = 32, 64, 128 on larger matrices, and
         the batched path at k_DM = 16, 32, 64 on the grid's batch: time, rank
         and the same ratio.

    python -m paper_2106_03138_amd.grid [--count 256] [--json OUT] [--md OUT]

Every factorization runs in the library's kernels; this module times them,
reads the diagonals back and tabulates.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import _lib
from . import inputs as I
from .api import Batch, BatchPlan, batch_params, device_matrix, qrdm_factor

STEP = 0.05
NGRID = 21


def numerical_rank(sigma: np.ndarray, n: int) -> int:
    """n_r = #{sigma_i > eps n sigma_1} (Section 5)."""
    if len(sigma) == 0 or sigma[0] == 0:
        return 0
    return int(np.sum(sigma > np.finfo(np.float64).eps * n * sigma[0]))


def min_ratio(rdiag: np.ndarray, sigma: np.ndarray, n: int) -> float:
    """min_{i < n_r} |r_ii| / sigma_i, diagonal entries in their positions."""
    nr = numerical_rank(sigma, n)
    if nr == 0:
        return float("inf")
    return float(np.min(np.abs(rdiag[:nr]) / sigma[:nr]))


def _diag_index(batch: Batch):
    idx = []
    for i, (m, n) in enumerate(batch.shapes):
        p = min(m, n)
        idx.append(int(batch.off[i]) + np.arange(p) * (batch.lda[i] + 1))
    return idx


def run_grid(mats, sigmas, taus=None, deltas=None, kmax: int = 64, verbose: bool = True):
    """Returns dict(taus, deltas, ratio [tau, delta], ms [tau, delta])."""
    import torch
    taus = [STEP * j for j in range(NGRID)] if taus is None else list(taus)
    deltas = [STEP * i for i in range(NGRID)] if deltas is None else list(deltas)
    b = Batch([a.shape for a in mats])
    b.load(mats)
    pristine = b.data.clone()
    plan = BatchPlan(b, kmax=kmax, stop_rule=_lib.STOP_NONE)
    didx = _diag_index(b)
    flat = torch.as_tensor(np.concatenate(didx)).cuda()
    cuts = np.cumsum([0] + [len(x) for x in didx])
    ratio = np.zeros((len(taus), len(deltas)))
    ms = np.zeros((len(taus), len(deltas)))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nb = len(mats)
    for jt, t in enumerate(taus):
        for idl, d in enumerate(deltas):
            pm = batch_params([t] * nb, [d] * nb, [kmax] * nb)
            b.data.copy_(pristine)
            ev0.record()
            plan.factor(params=pm)
            ev1.record()
            torch.cuda.synchronize()
            ms[jt, idl] = ev0.elapsed_time(ev1)
            diag = b.data[flat].cpu().numpy()
            ratio[jt, idl] = min(min_ratio(diag[cuts[i]: cuts[i + 1]], sigmas[i], a.shape[1])
                                 for i, a in enumerate(mats))
        if verbose:
            print(f"tau {t:.2f}: min ratio over delta {np.min(ratio[jt]):.2e}, "
                  f"time {ms[jt].min():.1f}..{ms[jt].max():.1f} ms", flush=True)
    plan.close()
    return {"taus": taus, "deltas": deltas, "ratio": ratio.tolist(), "ms": ms.tolist(), "count": nb,
            "kmax": kmax}


def run_kdm_single(cases, ks=(32, 64, 128), reps: int = 3):
    """Single-matrix path: per case and k_DM the median time of `reps` runs,
    the rank (stopping criterion of eq. (practical stopping criterion)) and the
    ratio over min(rank, n_r)."""
    import torch
    out = []
    for name, a, sigma in cases:
        n = a.shape[1]
        for k in ks:
            times = []
            for _ in range(reps + 1):
                A = device_matrix(a)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f = qrdm_factor(A, kmax=k)
                torch.cuda.synchronize()
                times.append(1e3 * (time.perf_counter() - t0))
            d = np.abs(np.diag(A[: min(a.shape), : min(a.shape)].cpu().numpy()))
            nr = min(numerical_rank(sigma, n), f.rank)
            q = float(np.min(d[:nr] / sigma[:nr])) if nr else float("inf")
            out.append({"case": name, "kmax": k, "ms": float(np.median(times[1:])), "rank": f.rank,
                        "n_r": numerical_rank(sigma, n), "ratio": q})
    return out


def run_kdm_batched(mats, sigmas, ks=(16, 32, 64), tau=0.15, delta=0.9):
    g = [run_grid(mats, sigmas, taus=[tau], deltas=[delta], kmax=k, verbose=False) for k in ks]
    return [{"kmax": k, "ms": r["ms"][0][0], "ratio": r["ratio"][0][0]} for k, r in zip(ks, g)]


def stand_in_collection(count: int, seed: int = 5):
    """Synthetic stand-in for the paper's collection of small matrices: the
    shapes of the uneven batch (m in [32, 512]) with the four spectrum
    families of the training set (geometric, stairs, flat with a gap, two
    clusters).  Returns (mats, sigmas)."""
    mats, shapes, sigmas, kinds = I.training_batch(count, seed=seed)
    return mats, sigmas


def markdown(rep: dict, kd_single, kd_batched, command: str) -> str:
    taus, deltas = rep["taus"], rep["deltas"]
    ratio, ms = np.array(rep["ratio"]), np.array(rep["ms"])
    head = "| tau \\ delta | " + " | ".join(f"{d:.2f}" for d in deltas) + " |"
    sep = "|---" * (len(deltas) + 1) + "|"
    lines = [f"# (tau, delta) grid and k_DM study, batched QRDM, {rep['count']} matrices", "",
             f"Command: `{command}`", "",
             "## floor(log10(min over matrices of min_{i<n_r} |r_ii| / sigma_i)) (Fig. 3a analogue)", "",
             head, sep]
    for j, t in enumerate(taus):
        cells = [("inf" if not np.isfinite(v) else ("-inf" if v <= 0 else str(int(np.floor(np.log10(v))))))
                 for v in ratio[j]]
        lines.append(f"| {t:.2f} | " + " | ".join(cells) + " |")
    lines += ["", f"## GPU time of the whole batch, ms (Fig. 3b analogue; k_DM = {rep['kmax']})", "", head, sep]
    for j, t in enumerate(taus):
        lines.append(f"| {t:.2f} | " + " | ".join(f"{v:.1f}" for v in ms[j]) + " |")
    lines += ["", "## k_DM, single-matrix path (stopping criterion on)", "",
              "| case | k_DM | ms | rank | n_r | min ratio |", "|---|---|---|---|---|---|"]
    for r in kd_single:
        lines.append(f"| {r['case']} | {r['kmax']} | {r['ms']:.1f} | {r['rank']} | {r['n_r']} | {r['ratio']:.3g} |")
    lines += ["", "## k_DM, batched path (tau 0.15, delta 0.9, full factorization)", "",
              "| k_DM | ms | min ratio |", "|---|---|---|"]
    for r in kd_batched:
        lines.append(f"| {r['kmax']} | {r['ms']:.1f} | {r['ratio']:.3g} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--kdm-n", type=int, default=2048, help="size of the single-matrix k_DM cases")
    ap.add_argument("--json", default="")
    ap.add_argument("--md", default="")
    args = ap.parse_args()
    _lib.load()
    mats, sigmas = stand_in_collection(args.count, args.seed)
    print(f"collection: {len(mats)} matrices", flush=True)
    rep = run_grid(mats, sigmas)
    n = args.kdm_n
    cases = [("half_rank", I.half_rank_noise(n, 1), np.concatenate([np.geomspace(1, 1e-8, n // 2),
                                                                     np.zeros(n - n // 2)])),
             ("geometric", I.from_spectrum(n, n, np.geomspace(1, 1e-16, n), 2), np.geomspace(1, 1e-16, n))]
    kd_single = run_kdm_single(cases)
    kd_batched = run_kdm_batched(mats, sigmas)
    for r in kd_single + kd_batched:
        print(json.dumps(r), flush=True)
    cmd = f"python -m paper_2106_03138_amd.grid --count {args.count} --seed {args.seed} --kdm-n {args.kdm_n}"
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"grid": rep, "kdm_single": kd_single, "kdm_batched": kd_batched}, f)
    if args.md:
        with open(args.md, "w") as f:
            f.write(markdown(rep, kd_single, kd_batched, cmd))


if __name__ == "__main__":
    main()
