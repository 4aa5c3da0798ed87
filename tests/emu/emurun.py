"""Input and output files of the batched-kernel emulation (tests/emu/batched_emu.cpp)."""
import os
import struct
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def build(out, tsan=False):
    """Compile the emulation with the host clang (its vector types match the kernel's)."""
    cxx = "/opt/rocm/lib/llvm/bin/clang++"
    flags = ["-std=c++17", "-O1", "-g", "-pthread", "-w"]
    if tsan:
        flags.append("-fsanitize=thread")
    cmd = [cxx] + flags + ["-I", HERE, "-I", os.path.join(ROOT, "paper_2106_03138_amd", "csrc"), "-I",
                           os.path.join(ROOT, "include"), "-x", "c++", os.path.join(HERE, "batched_emu.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def run(exe, mats, workdir, variant=0, grid=1, tau=0.15, delta=0.9, kmax=64, stop_rule=0, eps1_scale=0.0,
        certified=0, env=None, timeout=600, params=None, band=None):
    """Factor `mats` (float64 arrays) with the emulated kernel; returns one dict per matrix.
    params: per-matrix (tau, delta, kmax); with band also the online check and
    the re-run of the failures with the launch's parameters (the checked form)."""
    fin, fout = os.path.join(workdir, "in.bin"), os.path.join(workdir, "out.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("<iiiddiidi", len(mats), variant, grid, tau, delta, kmax, stop_rule, eps1_scale,
                            certified))
        for a in mats:
            m, n = a.shape
            f.write(struct.pack("<ii", m, n))
            f.write(np.asfortranarray(a, dtype=np.float64).tobytes(order="F"))
        if params is not None:
            f.write(struct.pack("<id", 2 if band is not None else 1, float(band or 0.0)))
            for t, d, k in params:
                f.write(struct.pack("<ddii", t, d, k, 0))
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout,
                       env=dict(os.environ, **(env or {})))
    if r.returncode != 0:
        raise RuntimeError(f"emulation exit {r.returncode}:\n{r.stderr[-4000:]}")
    out = []
    with open(fout, "rb") as f:
        for a in mats:
            m, n = a.shape
            p = min(m, n)
            rank, status = struct.unpack("<qi", f.read(12))
            tau_h = np.frombuffer(f.read(8 * p), dtype=np.float64).copy()
            perm = np.frombuffer(f.read(4 * n), dtype=np.int32).copy()
            qr = np.frombuffer(f.read(8 * m * n), dtype=np.float64).reshape((m, n), order="F").copy()
            info = np.frombuffer(f.read(32), dtype=np.int64).copy()
            ok = struct.unpack("<i", f.read(4))[0]
            out.append(dict(rank=rank, status=status, tau=tau_h, perm=perm, qr=qr, info=info, ok=ok))
    return out, r.stderr
