"""Torch-facing wrappers of the C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _lib


def _torch():
    import torch
    return torch


def device_matrix(a: np.ndarray, device: str = "cuda"):
    """Copy a host matrix to the GPU as a float64 column-major (Fortran) tensor of
    shape (m, n) with strides (1, m)."""
    torch = _torch()
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)  # (n, m) row-major == (m, n) col-major
    return t.t()


def host_matrix(t) -> np.ndarray:
    """Column-major device tensor -> Fortran-ordered numpy array."""
    return np.asfortranarray(t.t().contiguous().cpu().numpy().T)


def _check_matrix(A):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.dtype != torch.float64 or A.dim() != 2:
        raise TypeError("A must be a 2-D float64 torch tensor")
    if not A.is_cuda:
        raise ValueError("A must live on the GPU")
    m, n = A.shape
    if m > 1 and n > 0 and A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1)")
    lda = A.stride(1) if n > 1 else max(m, 1)
    return m, n, max(lda, max(m, 1))


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class Factorization:
    """Result of a pivoted QR: A holds R and the reflectors in place."""
    tau_house: object
    perm: object
    rank: int
    stats: dict = field(default_factory=dict)
    blocks: list = field(default_factory=list)


def _params(tau, delta, kmax, stop_rule, precision, poll_lag, eps1_scale, profile=False):
    p = _lib.Params()
    _lib.load().qrdm_default_params(ctypes.byref(p))
    p.tau, p.delta, p.kmax = float(tau), float(delta), int(kmax)
    p.stop_rule, p.precision, p.poll_lag = int(stop_rule), int(precision), int(poll_lag)
    p.eps1_scale = float(eps1_scale)
    p.profile = 1 if profile else 0
    return p


def qrdm_factor(A, tau: float = 0.15, delta: float = 0.9, kmax: int = 64, stop_rule: int = _lib.STOP_PAPER,
                precision: int = _lib.PREC_FP64, poll_lag: int = 4, eps1_scale: float = 0.0,
                log: bool = False, profile: bool = False, stream=None, tau_house=None,
                perm=None) -> Factorization:
    """QRDM (Algorithm 4 with Algorithm 1) of A in place."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    p = _params(tau, delta, kmax, stop_rule, precision, poll_lag, eps1_scale, profile)
    if tau_house is None:
        tau_house = torch.empty(max(min(m, n), 1), dtype=torch.float64, device=A.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    rank = ctypes.c_int64(-1)
    st = _lib.Stats()
    cap = (min(m, n) + 2) if log else 0
    blocks = (_lib.Block * max(cap, 1))()
    nlog = ctypes.c_int64(0)
    code = _lib.load().qrdm_factor_ex(
        ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.byref(p), ctypes.c_void_p(tau_house.data_ptr()),
        ctypes.c_void_p(perm.data_ptr()), ctypes.byref(rank), ctypes.byref(st),
        blocks if log else None, cap, ctypes.byref(nlog), _stream_ptr(stream))
    _lib.check("qrdm_factor_ex", code)
    stats = {k: getattr(st, k) for k, _ in _lib.Stats._fields_}
    bl = [(b.ns, b.nL, b.ks, b.l, b.fallback) for b in list(blocks)[: min(nlog.value, cap)]] if log else []
    return Factorization(tau_house[: min(m, n)], perm[:n], rank.value, stats, bl)


def qrp_factor(A, stop_rule: int = _lib.STOP_PAPER, nb: int = 32, poll_lag: int = 4, eps1_scale: float = 0.0,
               stream=None, tau_house=None, perm=None) -> Factorization:
    """QRP (Algorithm 2, blocked like xgeqp3) of A in place."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    p = _params(0.15, 0.9, 64, stop_rule, 0, poll_lag, eps1_scale)
    if tau_house is None:
        tau_house = torch.empty(max(min(m, n), 1), dtype=torch.float64, device=A.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    rank = ctypes.c_int64(-1)
    st = _lib.Stats()
    code = _lib.load().qrp_factor_ex(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.byref(p), int(nb),
                                     ctypes.c_void_p(tau_house.data_ptr()), ctypes.c_void_p(perm.data_ptr()),
                                     ctypes.byref(rank), ctypes.byref(st), _stream_ptr(stream))
    _lib.check("qrp_factor_ex", code)
    stats = {k: getattr(st, k) for k, _ in _lib.Stats._fields_}
    return Factorization(tau_house[: min(m, n)], perm[:n], rank.value, stats, [])


def colnorms(A, stream=None):
    torch = _torch()
    m, n, lda = _check_matrix(A)
    out = torch.empty(max(n, 1), dtype=torch.float64, device=A.device)
    code = _lib.load().qrdm_colnorms(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(out.data_ptr()),
                                     _stream_ptr(stream))
    _lib.check("qrdm_colnorms", code)
    return out[:n]


def dm_step(A, ns: int, vn1, tau: float, delta: float, kmax: int, stream=None):
    """One DM selection on [A]_{ns:m, ns:n}: returns (L, theta, J) as numpy arrays."""
    m, n, lda = _check_matrix(A)
    L = (ctypes.c_int32 * kmax)()
    J = (ctypes.c_int32 * kmax)()
    th = (ctypes.c_double * (kmax * kmax))()
    nL = ctypes.c_int32(0)
    ks = ctypes.c_int32(0)
    code = _lib.load().qrdm_dm_step(ctypes.c_void_p(A.data_ptr()), m, n, lda, int(ns),
                                    ctypes.c_void_p(vn1.data_ptr()), float(tau), float(delta), int(kmax),
                                    L, ctypes.byref(nL), th, J, ctypes.byref(ks), _stream_ptr(stream))
    _lib.check("qrdm_dm_step", code)
    k = nL.value
    return (np.array(L[:k], dtype=np.int64), np.array(th[: k * k]).reshape(k, k),
            np.array(J[: ks.value], dtype=np.int64))
