"""Benchmark: QRDM on one MI355X vs the GPU QRP baseline, 8192 x 8192 FP64.

    python bench.py [--steps K] [--warmup W] [--size 8192] [--spectrum geometric]
                    [--precision fp64|mixed] [--qrp-runs 2] [--cpu-sample-cols 192]

A step is one full QRDM factorization (Algorithm 4 of arXiv 2106.03138, the
whole hot path: norms, DM selection, swaps, Householder panel with break,
compact-WY trailing update, norm downdate) of a device-resident matrix that is
first restored from a pristine device copy (the restore is inside the timed
step).  The stopping criterion is off (full factorization) so QRDM and QRP do
equal work; TFLOP/s uses the algorithmic count F = 2mn^2 - 2n^3/3.

One JSON line is printed.  Besides the contract fields it carries:
  roofline      the kernel with the largest summed time, its average launch
                duration measured live with HIP events inside the library, against
                the roofline that bounds it (HBM bandwidth or FP64 MFMA);
  cpu_baseline  the CPU oracle timed on the host cores on a bounded sample (the
                first columns of the same matrix);
  qrp           the GPU QRP baseline on the same matrix and its speedup.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def flops_full(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def flops_cols(m, n, r):
    s = np.arange(r, dtype=np.float64)
    return float(np.sum(4.0 * (m - s) * (n - s)))


KERNEL_SOURCES = {"k_gemm1": "k_trail.hip", "k_gemm2": "k_trail.hip", "k_gemm2p": "k_trail.hip",
                  "k_qp_run": "k_qp3.hip", "k_qp_tail": "k_qp3.hip"}


def source_sha(kernel):
    import hashlib
    path = os.path.join(ROOT, "paper_2106_03138_amd", "csrc", KERNEL_SOURCES[kernel])
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic(kernel, workload_tag):
    """HBM bytes per launch from the committed counter summary of this kernel and
    workload (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or
    None when there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_tag}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != source_sha(kernel):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(prof, prec, Q, workload_tag=None, kmax=64):
    """Roofline of the kernel with the largest summed time among the column-
    pivoting kernel and the two trailing GEMMs (the panel and the DM selection
    are chains of short single-workgroup and grid launches, reported in
    phase_ms).  The column-pivoting kernel (one matrix-vector product over the
    trailing matrix per pivot: 2 flop per 8 B) is HBM-bound; at 8192^2 the whole
    tail is one launch of the register-resident k_qp_tail, otherwise block launches
    of k_qp_run.  The trailing GEMMs are timed alone (the partial sum and
    Z = T^T Y of k_zsum between them is reported apart); GEMM1 (8 B read per
    2 l flop) is MFMA-bound, GEMM2 (16 B per 2 l flop) close to the ridge.  GEMM2 is the
    persistent k_gemm2p for FP64 blocks of at most 64 reflectors, k_gemm2
    otherwise."""
    qp_name = "k_qp_tail" if int(prof.get("nqp3_tail", 0)) > 0 and int(prof.get("nqp3_launch", 0)) == 1 \
        else "k_qp_run"
    g2_name = "k_gemm2p" if prec != Q.PREC_MIXED and kmax <= 64 else "k_gemm2"
    times = {qp_name: prof.get("qp3_run_ms", 0.0), "k_gemm1": prof["gemm1_ms"], g2_name: prof["gemm2_ms"]}
    dom = max(times, key=times.get)
    nlaunch = max(int(prof["npanel"]), 1)  # one launch of each GEMM per block
    if dom in ("k_qp_run", "k_qp_tail"):
        nlaunch = max(int(prof["nqp3_launch"]), 1)
        bound, unit, peak = "hbm", "GB/s", PEAK_HBM_GBS
        work = prof["qp3_bytes"]
        achieved = work / (times[dom] * 1e-3) / 1e9
    elif dom == g2_name and prec != Q.PREC_MIXED:
        # FP64 GEMM2: 2 l flop per 16 B of A (8 flop/B at l = 64) is below the
        # ridge (78.6 TFLOP/s over 8 TB/s = 9.8 flop/B), so HBM bounds it
        bound, unit, peak = "hbm", "GB/s", PEAK_HBM_GBS
        work = prof["gemm2_bytes"]
        achieved = work / (times[dom] * 1e-3) / 1e9
    else:
        bound, unit = "mfma", "TFLOP/s"
        peak = PEAK_FP32_TFLOPS if prec == Q.PREC_MIXED else PEAK_FP64_TFLOPS
        work = prof["gemm_flop"]
        achieved = work / (times[dom] * 1e-3) / 1e12
    traffic = measured_traffic(dom, workload_tag) if workload_tag else None
    return {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "traffic": traffic,
            "launches": nlaunch, "avg_launch_us": round(1e3 * times[dom] / nlaunch, 2),
            "algorithmic_per_launch": work / nlaunch,
            "phase_ms": {"dm_select": round(prof["dm_ms"], 3), "panel": round(prof["panel_ms"], 3),
                         "gemm1": round(prof["gemm1_ms"], 3), "zsum": round(prof.get("zsum_ms", 0.0), 3),
                         "gemm2": round(prof["gemm2_ms"], 3),
                         "downdate": round(prof["downdate_ms"], 3), "qp3_tail": round(prof["qp3_ms"], 3),
                         "qp3_kernel": round(prof.get("qp3_run_ms", 0.0), 3),
                         "loop_total": round(prof["total_ms"], 3)},
            "gemm_tflops": {"gemm1": round(prof["gemm_flop"] / (prof["gemm1_ms"] * 1e-3) / 1e12, 3)
                            if prof["gemm1_ms"] > 0 else None,
                            "gemm1_with_zsum": round(prof["gemm_flop"] / ((prof["gemm1_ms"] + prof.get("zsum_ms", 0.0))
                                                                          * 1e-3) / 1e12, 3)
                            if prof["gemm1_ms"] > 0 else None,
                            "gemm2": round(prof["gemm_flop"] / (prof["gemm2_ms"] * 1e-3) / 1e12, 3)
                            if prof["gemm2_ms"] > 0 else None}}


def batched_leg(args, torch, Q):
    """The uneven batch: 2048 matrices, m ~ U{32..512}, n ~ U{16..m}, rank
    r ~ U{n/4..n} with singular values 10^(-14 (j-1)/(r-1)); the paper's stop
    rule and default parameters; launch per size class from the autotuner's
    cache.  Times graph replays (inputs restored before each, outside the
    timed region) and reports matrices/s."""
    from paper_2106_03138_amd import autotune
    from paper_2106_03138_amd import inputs as I
    mats, shapes = I.batch(args.batched_count, seed=args.seed)
    b = Q.Batch([(m, n) for m, n, _ in shapes])
    b.load(mats)
    pristine = b.data.clone()
    tune = autotune.load()
    plan = Q.BatchPlan(b, tau=args.tau, delta=args.delta, kmax=min(args.kmax, 64), tune=tune)
    plan.factor(use_graph=True)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.batched_reps):
        b.data.copy_(pristine)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.factor(use_graph=True)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    rank = b.rank.cpu().numpy()
    flop = sum(flops_cols(m, n, int(r)) for (m, n, _), r in zip(shapes, rank))
    # quality at the stated rule: rank against the numerical rank fixed by construction,
    # and the factor-10 band d_i / sigma_i (Section 5) on the first n_r diagonal entries
    host = b.data.cpu().numpy()
    exact, over, worst = 0, 0, np.inf
    for i, (m, n, r) in enumerate(shapes):
        sig = np.logspace(0.0, -14.0, r) if r > 1 else np.ones(1)
        nr = int(np.sum(sig > np.finfo(np.float64).eps * n * sig[0]))
        exact += int(rank[i] == nr)
        over = max(over, int(rank[i]) - nr)
        seg = host[int(b.off[i]): int(b.off[i]) + m * n].reshape((m, n), order="F")
        d = np.sort(np.abs(np.diag(seg)[:nr]))[::-1]
        worst = min(worst, float(np.min(d / sig[:nr])))
    solve = lstsq_leg(args, torch, Q, b, plan, shapes, ms)
    plan.close()
    learned = learned_leg(args, torch, Q, b, pristine, shapes, ms) if args.learned else None
    return {"metric": "batched QRDM matrices/s", "matrices": len(shapes), "ms": round(ms, 3),
            "matrices_per_s": round(len(shapes) / (ms * 1e-3), 1),
            "tflops": round(flop / (ms * 1e-3) / 1e12, 4), "flop": flop,
            "roofline": {"bound": "mfma", "kernel": "k_qrdm_batched", "achieved": round(flop / (ms * 1e-3) / 1e12, 4),
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flop / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 5)},
            "tune": [list(t) for t in tune], "launch": "hipGraph replay",
            "quality": {"rank_equals_numerical_rank": exact, "max_rank_over": over,
                        "min_d_over_sigma": round(worst, 4)},
            "lstsq": solve, "learned": learned}


def lstsq_leg(args, torch, Q, b, plan, shapes, factor_ms):
    """After the batched factorization: the basic least-squares solution for one
    seeded right-hand side per matrix (qrdm_batch_lstsq) and the post-hoc rank
    truncation (qrdm_batch_truncate_rank), each timed with HIP events (median of
    the reps; B restored outside the timed region).  The truncated ranks are
    compared with the numerical rank fixed by construction."""
    rng = np.random.default_rng(args.seed + 1)
    rhs = Q.BatchRHS(b, 1)
    rhs.load([rng.standard_normal(m) for m, _, _ in shapes])
    b0 = rhs.b.clone()
    times, ttr = [], []
    for _ in range(args.batched_reps):
        rhs.b.copy_(b0)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        plan.lstsq(rhs)
        e1.record()
        tr = plan.truncate_rank()
        e2.record()
        e2.synchronize()
        times.append(e0.elapsed_time(e1))
        ttr.append(e1.elapsed_time(e2))
    ms = float(np.median(times))
    tr = tr.cpu().numpy()
    exact, over = 0, 0
    for i, (m, n, r) in enumerate(shapes):
        sig = np.logspace(0.0, -14.0, r) if r > 1 else np.ones(1)
        nr = int(np.sum(sig > np.finfo(np.float64).eps * n * sig[0]))
        exact += int(tr[i] == nr)
        over = max(over, int(tr[i]) - nr)
    return {"nrhs": 1, "ms": round(ms, 3), "truncate_ms": round(float(np.median(ttr)), 3),
            "factor_plus_solve_matrices_per_s": round(len(shapes) / ((factor_ms + ms) * 1e-3), 1),
            "truncated_rank_equals_numerical_rank": exact, "truncated_max_rank_over": over,
            "timing": "HIP events around the launch on the current stream"}


def quality_of(b, shapes):
    """Rank against the numerical rank fixed by construction, and the factor-10
    band d_i / sigma_i on the first n_r diagonal entries (host, from R)."""
    rank = b.rank.cpu().numpy()
    host = b.data.cpu().numpy()
    exact, over, worst, below = 0, 0, np.inf, 0
    for i, (m, n, r) in enumerate(shapes):
        sig = np.logspace(0.0, -14.0, r) if r > 1 else np.ones(1)
        nr = int(np.sum(sig > np.finfo(np.float64).eps * n * sig[0]))
        exact += int(rank[i] == nr)
        over = max(over, int(rank[i]) - nr)
        seg = host[int(b.off[i]): int(b.off[i]) + m * n].reshape((m, n), order="F")
        d = np.sort(np.abs(np.diag(seg)[:nr]))[::-1]
        w = float(np.min(d / sig[:nr]))
        worst = min(worst, w)
        below += int(w < 0.1)
    return {"rank_equals_numerical_rank": exact, "max_rank_over": over, "min_d_over_sigma": round(worst, 4),
            "matrices_below_factor_10": below}


def learned_leg(args, torch, Q, b, pristine, shapes, default_ms):
    """Per-matrix (tau, delta, k_DM) from the trained MLP: features, forward pass,
    grid snap, then the factorization with the online condition check and the
    default re-runs of the matrices that fail it in one launch, all timed
    together; compared with the default parameters on the same batch."""
    from paper_2106_03138_amd import learned as Ld
    model = Ld.Model.load()
    if model is None:
        return None
    plan = Q.BatchPlan(b, tune=autotune_load())
    # the default parameters, eager and timed the same way (wall clock with a sync)
    eager = []
    for _ in range(args.batched_reps):
        b.data.copy_(pristine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.factor()
        torch.cuda.synchronize()
        eager.append(1e3 * (time.perf_counter() - t0))
    eager_ms = float(np.median(eager))
    b.data.copy_(pristine)
    ptrs = b.pointers(pristine)
    Ld.predict_factor(b, plan, model, pristine, pristine_ptrs=ptrs)  # warm up
    times, nfb = [], 0
    for _ in range(args.batched_reps):
        b.data.copy_(pristine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, nfb = Ld.predict_factor(b, plan, model, pristine, pristine_ptrs=ptrs)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    ms = float(np.median(times))
    # the breakdown: each stage between synchronizations, and the per-matrix
    # clock ticks of the batched kernel with the predicted and the default
    # parameters (the persistent launch lasts as long as its longest workgroup)
    bd = {}
    b.data.copy_(pristine)
    Ld.predict_factor(b, plan, model, pristine, breakdown=bd, pristine_ptrs=ptrs)
    tk_p = bd.pop("ticks").double()
    b.data.copy_(pristine)
    info = torch.zeros(4 * max(len(b), 1), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.factor(info=info)
    torch.cuda.synchronize()
    dflt_ms = 1e3 * (time.perf_counter() - t0)
    tk_d = info.view(-1, 4)[:, 3].double()
    breakdown = {k: round(v, 3) for k, v in bd.items()}
    breakdown.update({"default_factor_ms": round(dflt_ms, 3),
                      "ticks_sum_predicted_over_default": round(float(tk_p.sum() / tk_d.sum()), 4),
                      "ticks_max_predicted_over_default": round(float(tk_p.max() / tk_d.max()), 4)})
    pm = Ld.predict_params(plan, model).cpu().numpy().view(
        np.dtype([("tau", "<f8"), ("delta", "<f8"), ("kmax", "<i4"), ("pad", "<i4")]))
    import collections
    common = collections.Counter(zip(pm["tau"].round(3), pm["delta"].round(3), pm["kmax"])).most_common(3)
    qual = quality_of(b, shapes)
    plan.close()
    return {"ms": round(ms, 3), "default_eager_ms": round(eager_ms, 3),
            "gain_vs_default": round(eager_ms / ms, 4), "gain_vs_default_graph": round(default_ms / ms, 4),
            "fallbacks": nfb,
            "matrices_per_s": round(len(shapes) / (ms * 1e-3), 1), "quality": qual,
            "most_common_params": [[float(t), float(d), int(k), c] for (t, d, k), c in common],
            "breakdown": breakdown,
            "timing": "wall clock around features + MLP + checked factorization (eager)"}


def _qt_sampled_residual(a, qr, tau, perm, nref, cols):
    """Estimate of ||A P - Q R||_F / ||A||_F from the columns `cols` of A P
    (LAPACK dormqr applies Q^T; host numpy/scipy, not the oracle)."""
    from scipy.linalg import lapack
    y = np.asfortranarray(a[:, perm[cols]])
    if nref > 0:
        y, _, info = lapack.dormqr("L", "T", np.asfortranarray(qr[:, :nref]), np.ascontiguousarray(tau[:nref]), y,
                                   max(1, 64 * y.shape[1]))
        assert info == 0
    r = np.array(qr[:, cols], copy=True)
    for c, j in enumerate(cols):
        if j < nref:
            r[j + 1:, c] = 0.0
    return float(np.sqrt(a.shape[1] / len(cols) * np.sum((y - r) ** 2)) / np.linalg.norm(a))


def _quality(a, qr, tau, perm, rank, sigma, full, eps_w=np.finfo(np.float64).eps):
    """Rank against n_r = #{sigma_i > eps_w n sigma_1} (eps_w = 2^-52, or 2^-23 for
    mixed precision, whose trailing data carry FP32 rounding), min/max d_i / sigma_i
    over the first n_r (d_i = i-th largest |r_ii|, Section 5), sampled backward error."""
    m, n = a.shape
    nref = min(m, n) if full else rank
    cols = np.random.default_rng(1).choice(n, min(n, 64), replace=False)
    q = {"rank": int(rank), "residual": float(f"{_qt_sampled_residual(a, qr, tau, perm, nref, cols):.3e}")}
    if sigma is not None:
        sg = np.sort(sigma)[::-1]
        nr = int(np.sum(sg > eps_w * n * sg[0]))
        d = np.sort(np.abs(np.diag(qr)[:nr]))[::-1] / sg[:nr]
        q.update({"n_r": nr, "d_over_sigma": [round(float(d.min()), 4), round(float(d.max()), 4)]})
    return q


def configs_leg(args, torch, Q):
    """The workloads of every configuration besides the headline: one timed line
    each (median of `reps` runs, the input restored from a device copy inside each
    run, wall clock around a synchronized call), with the quality at the stated
    rule.  Per matrix: QRDM with the paper's stopping rule (its rank is the
    numerical rank the method reports), QRDM and GPU QRP at equal work (stop
    off), and QRDM with the stop against full QRP (the comparison of the paper's
    Fig. 7).  The 8192^2 spectra also run in mixed precision, with the gap of its
    R diagonal to the FP64 run's."""
    from paper_2106_03138_amd import inputs as I
    out = []

    def timed(A, a0, fn, reps):
        ts = []
        res = None
        for _ in range(reps + 1):
            A.copy_(a0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn(A)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        return float(np.median(ts[1:])), res

    def one(name, a0, sigma, qp, reps, mixed):
        m, n = a0.shape
        A = torch.empty_like(a0.t().contiguous()).t()
        th = torch.empty(min(m, n), dtype=torch.float64, device="cuda")
        pm = torch.empty(n, dtype=torch.int32, device="cuda")
        host = np.asfortranarray(a0.t().contiguous().cpu().numpy().T)
        row = {"config": name, "m": m, "n": n, "tau": qp[0], "delta": qp[1], "k_DM": qp[2]}
        kw = dict(tau=qp[0], delta=qp[1], kmax=qp[2], tau_house=th, perm=pm)
        for label, stop, prec in [("qrdm_stop", Q.STOP_PAPER, Q.PREC_FP64), ("qrdm_full", Q.STOP_NONE, Q.PREC_FP64)] + \
                ([("qrdm_full_mixed", Q.STOP_NONE, Q.PREC_MIXED), ("qrdm_stop_mixed", Q.STOP_PAPER, Q.PREC_MIXED)]
                 if mixed else []):
            ms, o = timed(A, a0, lambda X: Q.qrdm_factor(X, stop_rule=stop, precision=prec, **kw), reps)
            full = stop == Q.STOP_NONE
            r = o.rank
            F = flops_full(m, n) if full else flops_cols(m, n, r)
            qr = Q.host_matrix(A)
            e = {"ms": round(ms, 3), "tflops": round(F / (ms * 1e-3) / 1e12, 3)}
            e.update(_quality(host, qr, th.cpu().numpy(), pm.cpu().numpy(), r, sigma, full,
                              2.0 ** -23 if prec == Q.PREC_MIXED else np.finfo(np.float64).eps))
            if label == "qrdm_full":
                d64 = np.sort(np.abs(np.diag(qr)))[::-1]
            if label == "qrdm_full_mixed":
                dmx = np.sort(np.abs(np.diag(qr)))[::-1]
                e["max_diag_gap_to_fp64_over_norm"] = float(f"{np.max(np.abs(dmx - d64)) / abs(d64[0]):.3e}")
            row[label] = e
        for label, stop in [("qrp_full", Q.STOP_NONE), ("qrp_stop", Q.STOP_PAPER)]:
            ms, o = timed(A, a0, lambda X: Q.qrp_factor(X, stop_rule=stop, tau_house=th, perm=pm), max(1, reps // 3))
            row[label] = {"ms": round(ms, 3), "rank": int(o.rank)}
        row["speedup_equal_work"] = round(row["qrp_full"]["ms"] / row["qrdm_full"]["ms"], 3)
        row["speedup_fig7"] = round(row["qrp_full"]["ms"] / row["qrdm_stop"]["ms"], 3)
        row["speedup_both_stopped"] = round(row["qrp_stop"]["ms"] / row["qrdm_stop"]["ms"], 3)
        print(f"[bench configs] {name}: qrdm full {row['qrdm_full']['ms']} ms, qrp full {row['qrp_full']['ms']} ms",
              file=sys.stderr, flush=True)
        out.append(row)
        del A

    a0 = torch.from_numpy(np.ascontiguousarray(I.small_rank64(0).T)).cuda().t()
    one("256x256 rank 64 (sigma 1 -> 1e-3, then 1e-15)", a0, I.geometric_rank(256, 64, 1.0, 1e-3, 1e-15),
        (0.9, 0.9, 32), 10, False)
    for spec, label in [("half_rank", "4096x4096 numerical rank 2048 (sigma 1 -> 1e-8, then 1e-16 noise)"),
                        ("kahan", "Kahan 4096 (theta = 1.2)")]:
        a0 = I.device_matrix(4096, spec, args.seed, torch)
        one(label, a0, I.device_spectrum(4096, spec, args.seed) if spec != "kahan" else None,
            (args.tau, args.delta, args.kmax), 3, False)
        del a0
    for spec in ["geometric", "stairs", "gaussian"]:
        a0 = I.device_matrix(8192, spec, args.seed, torch)
        one(f"8192x8192 {spec}", a0, I.device_spectrum(8192, spec) if spec != "gaussian" else None,
            (args.tau, args.delta, args.kmax), 3, True)
        del a0
    torch.cuda.empty_cache()
    return out


def autotune_load():
    from paper_2106_03138_amd import autotune
    return autotune.load()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--spectrum", default="geometric", choices=["geometric", "stairs", "gaussian"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tau", type=float, default=0.15)
    ap.add_argument("--delta", type=float, default=0.9)
    ap.add_argument("--kmax", type=int, default=64)
    ap.add_argument("--qrp-runs", type=int, default=2)  # timed runs; the fastest is reported
    ap.add_argument("--cpu-sample-cols", type=int, default=1536)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain elementwise copy of this many MiB (for counter calibration)")
    ap.add_argument("--no-profile-run", action="store_true")
    ap.add_argument("--batched-count", type=int, default=2048, help="0 skips the batched leg")
    ap.add_argument("--batched-reps", type=int, default=5)
    ap.add_argument("--learned", type=int, default=1, help="1 = also time the learned-parameter path")
    ap.add_argument("--input-cache", default="",
                    help=".npy file holding the input: loaded if present, else written after generation")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--configs", type=int, default=1,
                    help="1 = also time the other configurations (256^2, 4096^2, the 8192^2 spectra, mixed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is "
              "described in the design notes, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2106_03138_amd as Q
    from paper_2106_03138_amd import inputs as I

    Q.load()
    torch.cuda.set_device(0)
    n = m = args.size
    prec = Q.PREC_MIXED if args.precision == "mixed" else Q.PREC_FP64
    if args.copy_calibration_mb > 0:
        # a plain copy kernel of known traffic: reads and writes N float64 once each
        cnt = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(cnt, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.input_cache and os.path.exists(args.input_cache):
        a0 = torch.from_numpy(np.load(args.input_cache)).cuda().t()  # stored as the (n, m) row-major A^T
    else:
        a0 = I.device_matrix(n, args.spectrum, args.seed, torch)
        if args.input_cache:
            np.save(args.input_cache, a0.t().contiguous().cpu().numpy())
    A = torch.empty_like(a0.t().contiguous()).t()
    tau_h = torch.empty(n, dtype=torch.float64, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    kw = dict(tau=args.tau, delta=args.delta, kmax=args.kmax, stop_rule=Q.STOP_NONE, precision=prec,
              tau_house=tau_h, perm=perm)

    def step(**extra):
        A.copy_(a0)
        return Q.qrdm_factor(A, **kw, **extra)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    F = flops_full(m, n)
    value = F / (ms * 1e-3) / 1e12

    # per-phase times from HIP events on the library's stream; the dominant kernel
    # is the single kernel with the largest summed time
    tag = f"qrdm{m}_{args.spectrum}_{args.precision}"
    roof = None
    if not args.no_profile_run:
        prof = step(profile=True).stats
        roof = roofline(prof, prec, Q, tag, args.kmax)
    rank = outs[-1].rank
    st = outs[-1].stats

    # GPU QRP baseline on the same matrix
    qrp = None
    if args.qrp_runs > 0:
        times = []
        for _ in range(args.qrp_runs):
            A.copy_(a0)
            torch.cuda.synchronize()
            q0 = time.perf_counter()
            qo = Q.qrp_factor(A, stop_rule=Q.STOP_NONE, tau_house=tau_h, perm=perm)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - q0)
        qms = 1e3 * min(times)
        qrp = {"ms": round(qms, 3), "tflops": round(F / (qms * 1e-3) / 1e12, 3),
               "speedup_qrdm_over_qrp": round(qms / ms, 3), "rank": qo.rank}

    # CPU oracle on a bounded sample: the first columns of the same matrix
    cpu = None
    if args.cpu_sample_cols > 0:
        import oracle
        host = np.asfortranarray(a0.t().contiguous().cpu().numpy().T)
        cores = oracle.threads()
        c0 = time.perf_counter()
        res = oracle.qrdm(host, tau=args.tau, delta=args.delta, kmax=args.kmax, stop_rule=oracle.STOP_NONE,
                          max_ns=args.cpu_sample_cols, log_cap=args.cpu_sample_cols + 2)
        ct = time.perf_counter() - c0
        done_cols = int(sum(b.l for b in res.blocks))
        cf = flops_cols(m, n, done_cols)
        cpu = {"value": round(cf / ct / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
               "sample": f"first {done_cols} of {n} columns of the same {m}x{n} {args.spectrum} matrix "
                         f"({cf / 1e9:.1f} GFLOP in {ct:.1f} s)"}

    batched = batched_leg(args, torch, Q) if args.batched_count > 0 else None
    del A
    torch.cuda.empty_cache()
    per_config = configs_leg(args, torch, Q) if args.configs else None

    line = {
        "metric": "QRDM TFLOP/s vs GPU QRP at 8192^2 (full factorization, FP64), at stated RR quality",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == Q.PREC_FP64 else "f64+f32mfma",
        "data": "synthetic",
        "config": {"workload": f"qrdm {m}x{n} {args.spectrum} spectrum, tau={args.tau} delta={args.delta} "
                               f"k_DM={args.kmax}, stop off (full), {args.precision}",
                   "m": m, "n": n, "flop": F, "rank_paper_rule": rank,
                   "blocks": st["nblocks"], "breaks": st["nbreaks"], "recomputes": st["nrecompute"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "qrp": qrp,
        "batched": batched,
        "per_config": per_config,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
