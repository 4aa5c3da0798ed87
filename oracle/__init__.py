"""CPU oracle for QRDM / QRP (TEST INFRASTRUCTURE ONLY).

ctypes bindings to oracle/liboracle.so (plain C, FP64, built from
oracle/qrdm_oracle.c) plus host-side quality metrics.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

STOP_PAPER, STOP_MAXNORM, STOP_NONE = 0, 1, 2
# deliberate mistakes for the tests of the checks (oracle_params.plant)
PLANT_SINGLE, PLANT_TRUNC, PLANT_ACCEPT, PLANT_NOBREAK, PLANT_FBSCALE, PLANT_DNORM, PLANT_REJECT = range(1, 8)

_LIB = None


class OracleBlock(ctypes.Structure):
    _fields_ = [
        ("ns", ctypes.c_int64), ("ncand", ctypes.c_int32), ("nL", ctypes.c_int32),
        ("ks", ctypes.c_int32), ("l", ctypes.c_int32), ("fallback", ctypes.c_int32),
        ("jmax", ctypes.c_int32), ("umax", ctypes.c_double), ("eps_s", ctypes.c_double),
        ("m_order", ctypes.c_double), ("m_thr", ctypes.c_double), ("m_cos", ctypes.c_double),
        ("m_break", ctypes.c_double), ("m_stop", ctypes.c_double), ("m_fb", ctypes.c_double),
        ("m_recomp", ctypes.c_double), ("gamma", ctypes.c_double), ("sigma_bound", ctypes.c_double),
    ]


class OracleParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("delta", ctypes.c_double), ("kmax", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("eps1_scale", ctypes.c_double),
                ("max_ns", ctypes.c_int64), ("certified", ctypes.c_int32), ("plant", ctypes.c_int32)]


def lib():
    global _LIB
    if _LIB is None:
        path = build_oracle.ensure_built()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_qrdm.restype = ctypes.c_int
        L.oracle_qrdm.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.POINTER(OracleParams), dp, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(OracleBlock),
                                  ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_dm_step.restype = ctypes.c_int
        L.oracle_dm_step.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     dp, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), dp,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        L.oracle_block_size.restype = ctypes.c_size_t
        assert L.oracle_block_size() == ctypes.sizeof(OracleBlock)
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Result:
    """Output of one oracle factorization."""

    def __init__(self, qr, tau, perm, rank, blocks, code):
        self.qr, self.tau, self.perm, self.rank, self.blocks, self.code = qr, tau, perm, rank, blocks, code

    @property
    def R(self):
        return np.triu(self.qr[: min(self.qr.shape), :])

    def first_low_margin_block(self, eta=1e-10):
        """Index of the first block where any decision margin is below eta (len if none)."""
        for i, b in enumerate(self.blocks):
            if min(b.m_order, b.m_thr, b.m_cos, b.m_break, b.m_stop, b.m_fb, b.m_recomp) < eta:
                return i
        return len(self.blocks)


def qrdm(a: np.ndarray, tau: float = 0.15, delta: float = 0.9, kmax: int = 64,
         stop_rule: int = STOP_PAPER, eps1_scale: float = 0.0, max_ns: int = -1,
         log_cap: int | None = None, certified: bool = False, plant: int = 0) -> Result:
    """Oracle QRDM2 (Algorithm 4) on a copy of a (m x n float64).  plant != 0
    (tests of the checks only) runs one of the deliberate mistakes PLANT_*."""
    a = np.array(a, dtype=np.float64, order="F", copy=True)
    m, n = a.shape
    p = min(m, n)
    tau_h = np.zeros(max(p, 1))
    perm = np.zeros(max(n, 1), dtype=np.int32)
    rank = ctypes.c_int64(-1)
    cap = log_cap if log_cap is not None else max(n, 1) + 2
    blocks = (OracleBlock * cap)()
    nb = ctypes.c_int64(0)
    prm = OracleParams(tau, delta, kmax, stop_rule, eps1_scale, max_ns, 1 if certified else 0, int(plant))
    code = lib().oracle_qrdm(_dp(a), m, n, max(m, 1), ctypes.byref(prm), _dp(tau_h),
                             perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(rank),
                             blocks, cap, ctypes.byref(nb))
    nb_used = min(nb.value, cap)
    return Result(a, tau_h[:p], perm[:n], rank.value, [blocks[i] for i in range(nb_used)], code)


def qrp(a: np.ndarray, stop_rule: int = STOP_PAPER, eps1_scale: float = 0.0, max_ns: int = -1) -> Result:
    """Oracle QRP (Algorithm 2): QRDM2 with a single arg-max pivot per step."""
    return qrdm(a, tau=1.0, delta=0.0, kmax=1, stop_rule=stop_rule, eps1_scale=eps1_scale, max_ns=max_ns)


def dm_step(a: np.ndarray, vn1: np.ndarray, ns: int, tau: float, delta: float, cap: int, plant: int = 0):
    """One DM selection (Algorithm 1) on [A]_{ns:m, ns:n}: returns (L, theta, J)."""
    a = np.asfortranarray(a, dtype=np.float64)
    m, n = a.shape
    vn1 = np.ascontiguousarray(vn1, dtype=np.float64)
    L = np.zeros(cap, dtype=np.int64)
    J = np.zeros(cap, dtype=np.int64)
    th = np.zeros(cap * cap)
    nl = ctypes.c_int32(0)
    ks = ctypes.c_int32(0)
    code = lib().oracle_dm_step(_dp(a), m, n, m, ns, _dp(vn1), tau, delta, cap,
                                L.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(nl), _dp(th),
                                J.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(ks), int(plant))
    if code != 0:
        raise RuntimeError(f"oracle_dm_step failed: {code}")
    k = nl.value
    return L[:k].copy(), th[: k * k].reshape(k, k).copy(), J[: ks.value].copy()


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())
