"""The batched QRDM kernel (k_batched.hip) run on the CPU under a host
emulation of the HIP device interface (tests/emu): one host thread per GPU
thread, __syncthreads as a pthread barrier over the workgroup, and every
cross-lane operation (shuffle, ballot, FP64 MFMA) as an exchange between two
barriers over the wavefront.  The emulation is built with ThreadSanitizer, so
any hand-off between threads that the kernel does not fence (an LDS or global
value read or written by two threads with no barrier or cross-lane operation
between them) fails the run, and its result is compared with the oracle:
the rank (the paper's stopping test, and a full factorization that passes
through the scalar-pivoting switch), a permutation, the backward error.

Variants 0-2 are the library's 256-thread forms (register panel with one or
two column tiles per wavefront, panel read from memory); 3 is the 512-thread
form, which the library does not offer (it spills on gfx950) but whose code
the emulation shows to be correct.
"""
import os
import shutil

import numpy as np
import pytest

import oracle
from emu import emurun
from oracle import metrics as M
from paper_2106_03138_amd import inputs as I

CXX = "/opt/rocm/lib/llvm/bin/clang++"
TSAN = {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"}


@pytest.fixture(scope="module")
def emu_exe(tmp_path_factory):
    if not os.path.exists(CXX) or shutil.which("g++") is None:
        pytest.skip("host clang++ not available")
    d = tmp_path_factory.mktemp("emu")
    return emurun.build(str(d / "batched_emu_tsan"), tsan=True), d


def _cases():
    """A 152 x 96 matrix of numerical rank 73 (the batch's spectrum family), a
    300 x 60 one (two panel rows per thread), a 600 x 40 one (the panel
    read from memory past 512 rows) and a 70 x 32 Gaussian one."""
    return [I.batch_matrix(152, 96, 73, np.random.SeedSequence(152096 + 73)),
            I.batch_matrix(300, 60, 50, np.random.SeedSequence(3)),
            I.batch_matrix(600, 40, 30, np.random.SeedSequence(4)),
            I.gaussian(70, 32, 3)]


@pytest.mark.parametrize("variant,rule", [(0, oracle.STOP_PAPER), (0, oracle.STOP_NONE), (1, oracle.STOP_PAPER),
                                          (2, oracle.STOP_NONE), (3, oracle.STOP_NONE)])
def test_batched_kernel_emulated(emu_exe, variant, rule):
    exe, d = emu_exe
    mats = _cases()
    res, _ = emurun.run(exe, mats, str(d), variant=variant, stop_rule=rule, env=TSAN, timeout=900)
    for a, r in zip(mats, res):
        m, n = a.shape
        ref = oracle.qrdm(a, stop_rule=rule)
        assert r["status"] == 0
        assert r["rank"] == ref.rank, (a.shape, r["rank"], ref.rank)
        assert sorted(r["perm"].tolist()) == list(range(n))
        nref = min(m, n) if rule == oracle.STOP_NONE else r["rank"]
        assert M.residual(a, r["qr"], r["tau"], r["perm"], nref) <= 1e-13
        steps, breaks, fallback = r["info"][:3]
        assert steps >= 1 and breaks <= steps
        if rule == oracle.STOP_NONE and ref.rank < min(m, n):
            assert fallback > 0  # the full run passes through the scalar-pivoting switch


def test_emulation_catches_unfenced_handoff(tmp_path):
    """The harness itself: ThreadSanitizer reports an LDS value written by one
    thread and read by the others without a barrier, and not with one; the
    emulated shuffles, ballot and MFMA follow their lane definitions."""
    if not os.path.exists(CXX):
        pytest.skip("host clang++ not available")
    import subprocess
    exe = str(tmp_path / "probe")
    subprocess.run([CXX, "-std=c++17", "-O1", "-g", "-pthread", "-w", "-fsanitize=thread", "-I", emurun.HERE, "-x",
                    "c++", os.path.join(emurun.HERE, "probe.cpp"), "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, **TSAN)
    ok = subprocess.run([exe, "fenced"], env=env, capture_output=True, text=True, timeout=120)
    assert ok.returncode == 0, ok.stderr[-2000:]
    bad = subprocess.run([exe, "racy"], env=env, capture_output=True, text=True, timeout=120)
    assert bad.returncode == 66 and "data race" in bad.stderr
    lanes = subprocess.run([exe, "lanes"], env=env, capture_output=True, text=True, timeout=120)
    assert lanes.returncode == 0 and "lanes ok" in lanes.stdout, lanes.stdout + lanes.stderr[-2000:]


def test_checked_form_emulated(emu_exe):
    """The checked form (per-matrix parameters, the online check, the re-run of
    a failure from its pristine copy with the launch's parameters, all in the
    workgroup's loop) under ThreadSanitizer: a matrix it keeps equals the run
    with its per-matrix parameters alone, a matrix it factors again equals the
    run with the launch's parameters, bit for bit; the ok flags follow the
    oracle's condition estimate where it is not at the threshold."""
    from oracle import learned as Lr
    exe, d = emu_exe
    mats = _cases() + [I.batch_matrix(120, 90, 80, np.random.SeedSequence(7)),
                       I.from_spectrum(96, 96, np.geomspace(1.0, 1e-12, 96), 8)]
    # aggressive parameters (tau = 0, delta = 1 admits almost any block) for some
    params = [(0.0, 1.0, 64) if i % 2 == 0 else (0.3, 0.7, 32) for i in range(len(mats))]
    own, _ = emurun.run(exe, mats, str(d), variant=1, params=params, env=TSAN, timeout=900)
    # a band between two of the estimate-to-diagonal ratios, so that some
    # matrices pass the check and some are factored again
    ratios = []
    for o in own:
        r = int(o["rank"])
        if r > 0:
            R = np.triu(o["qr"][:r, :r])
            ratios.append(Lr.ice_sigma_min(R) / np.min(np.abs(np.diag(R))))
    ratios = np.sort(ratios)
    h = len(ratios) // 2
    band = float(np.sqrt(ratios[h - 1] * ratios[h]))
    chk, _ = emurun.run(exe, mats, str(d), variant=1, params=params, band=band, env=TSAN, timeout=900)
    dflt, _ = emurun.run(exe, mats, str(d), variant=1, env=TSAN, timeout=900)
    kept = redo = 0
    for i, (c, o, f) in enumerate(zip(chk, own, dflt)):
        ref = o if c["ok"] == 1 else f
        kept += c["ok"] == 1
        redo += c["ok"] == 0
        assert c["ok"] in (0, 1)
        for key in ("rank", "status"):
            assert c[key] == ref[key], (i, key)
        for key in ("tau", "perm", "qr"):
            assert np.array_equal(c[key], ref[key]), (i, key)
        r = int(o["rank"])
        if r > 0:
            R = np.triu(o["qr"][:r, :r])
            est = Lr.ice_sigma_min(R)
            thr = band * np.min(np.abs(np.diag(R)))
            scale = np.max(np.abs(np.diag(R)))
            if abs(est - thr) > 1e-8 * max(est, thr) + 1e-12 * scale:
                assert c["ok"] == int(est >= thr), (i, est, thr)
    assert kept >= 1 and redo >= 1, (kept, redo)
