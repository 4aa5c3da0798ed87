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
    if m == 0 or n <= 1:
        return m, n, max(m, 1)  # no second column: the stride is never used
    lda = A.stride(1)
    if lda < max(m, 1):
        raise ValueError(f"A's column stride {lda} is below its {m} rows (columns would overlap)")
    return m, n, lda


def _out_vector(t, name, dtype, count, A):
    """A caller-supplied output vector: the dtype, at least `count` contiguous
    elements, on A's device."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != dtype:
        raise TypeError(f"{name} must be a {dtype} torch tensor")
    if t.device != A.device:
        raise ValueError(f"{name} must live on {A.device}")
    if not t.is_contiguous() or t.numel() < max(count, 1):
        raise ValueError(f"{name} must be contiguous with at least {max(count, 1)} elements")
    return t


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


def _params(tau, delta, kmax, stop_rule, precision, poll_lag, eps1_scale, profile=False, certified=False):
    p = _lib.Params()
    _lib.load().qrdm_default_params(ctypes.byref(p))
    p.tau, p.delta, p.kmax = float(tau), float(delta), int(kmax)
    p.stop_rule, p.precision, p.poll_lag = int(stop_rule), int(precision), int(poll_lag)
    p.eps1_scale = float(eps1_scale)
    p.profile = 1 if profile else 0
    p.certified = 1 if certified else 0
    return p


def _outputs(A, m, n, tau_house, perm):
    torch = _torch()
    if tau_house is None:
        tau_house = torch.empty(max(min(m, n), 1), dtype=torch.float64, device=A.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    return (_out_vector(tau_house, "tau_house", torch.float64, min(m, n), A),
            _out_vector(perm, "perm", torch.int32, n, A))


def workspace_size(m: int, n: int, kmax: int = 64) -> int:
    """Bytes of device workspace qrdm_factor_ws needs (qrdm_workspace_size)."""
    p = _lib.Params()
    _lib.load().qrdm_default_params(ctypes.byref(p))
    p.kmax = int(kmax)
    return int(_lib.load().qrdm_workspace_size(int(m), int(n), ctypes.byref(p)))


def qrdm_factor_ws(A, workspace, rank_out, tau: float = 0.15, delta: float = 0.9, kmax: int = 64,
                   stop_rule: int = _lib.STOP_PAPER, precision: int = _lib.PREC_FP64, poll_lag: int = 4,
                   eps1_scale: float = 0.0, stream=None, tau_house=None, perm=None, certified: bool = False,
                   stats: bool = False) -> Factorization:
    """QRDM of A in place in a caller-owned workspace (a uint8 device tensor of at
    least workspace_size(m, n, kmax) bytes); the rank goes to rank_out (an int64
    device tensor with one element) in stream order.  The returned
    Factorization's rank is -1 (it stays on the device)."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    p = _params(tau, delta, kmax, stop_rule, precision, poll_lag, eps1_scale, False, certified)
    tau_house, perm = _outputs(A, m, n, tau_house, perm)
    rank_out = _out_vector(rank_out, "rank_out", torch.int64, 1, A)
    if not isinstance(workspace, torch.Tensor) or workspace.device != A.device or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous tensor on A's device")
    nbytes = workspace.numel() * workspace.element_size()
    st = _lib.Stats()
    code = _lib.load().qrdm_factor_ws(
        ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.byref(p), ctypes.c_void_p(tau_house.data_ptr()),
        ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(rank_out.data_ptr()), ctypes.byref(st) if stats else None,
        ctypes.c_void_p(workspace.data_ptr()), nbytes, _stream_ptr(stream))
    _lib.check("qrdm_factor_ws", code)
    sd = {k: getattr(st, k) for k, _ in _lib.Stats._fields_} if stats else {}
    return Factorization(tau_house[: min(m, n)], perm[:n], -1, sd, [])


def qrdm_factor_noalloc(A, rank_out, tau: float = 0.15, delta: float = 0.9, kmax: int = 64,
                        stop_rule: int = _lib.STOP_PAPER, precision: int = _lib.PREC_FP64, eps1_scale: float = 0.0,
                        stream=None, tau_house=None, perm=None, certified: bool = False) -> Factorization:
    """QRDM of A in place in the library's fixed device scratch (no allocation by
    the library; tau_house and perm must be passed in to keep the call free of
    allocations here too).  The rank goes to rank_out (an int64 device tensor
    with one element) in stream order; the returned Factorization's rank is -1."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    p = _params(tau, delta, kmax, stop_rule, precision, 0, eps1_scale, False, certified)
    tau_house, perm = _outputs(A, m, n, tau_house, perm)
    rank_out = _out_vector(rank_out, "rank_out", torch.int64, 1, A)
    code = _lib.load().qrdm_factor_noalloc(
        ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.byref(p), ctypes.c_void_p(tau_house.data_ptr()),
        ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(rank_out.data_ptr()), _stream_ptr(stream))
    _lib.check("qrdm_factor_noalloc", code)
    return Factorization(tau_house[: min(m, n)], perm[:n], -1, {}, [])


def qrdm_factor(A, tau: float = 0.15, delta: float = 0.9, kmax: int = 64, stop_rule: int = _lib.STOP_PAPER,
                precision: int = _lib.PREC_FP64, poll_lag: int = 4, eps1_scale: float = 0.0,
                log: bool = False, profile: bool = False, stream=None, tau_house=None,
                perm=None, certified: bool = False) -> Factorization:
    """QRDM (Algorithm 4 with Algorithm 1) of A in place.  With log=True,
    blocks holds (ns, nL, ks, l, fallback, gamma, sigma_bound, umax) per step of
    the DM loop; a last record with fallback = 1 and l = 0 marks the hand-over
    to column pivoting at column ns (eq. column_norm_bound_DM)."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    p = _params(tau, delta, kmax, stop_rule, precision, poll_lag, eps1_scale, profile, certified)
    tau_house, perm = _outputs(A, m, n, tau_house, perm)
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
    bl = [(b.ns, b.nL, b.ks, b.l, b.fallback, b.gamma, b.sigma_bound, b.umax)
          for b in list(blocks)[: min(nlog.value, cap)]] if log else []
    return Factorization(tau_house[: min(m, n)], perm[:n], rank.value, stats, bl)


def qrp_factor(A, stop_rule: int = _lib.STOP_PAPER, nb: int = 32, poll_lag: int = 4, eps1_scale: float = 0.0,
               stream=None, tau_house=None, perm=None) -> Factorization:
    """QRP (Algorithm 2, blocked like xgeqp3) of A in place."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    p = _params(0.15, 0.9, 64, stop_rule, 0, poll_lag, eps1_scale)
    tau_house, perm = _outputs(A, m, n, tau_house, perm)
    rank = ctypes.c_int64(-1)
    st = _lib.Stats()
    code = _lib.load().qrp_factor_ex(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.byref(p), int(nb),
                                     ctypes.c_void_p(tau_house.data_ptr()), ctypes.c_void_p(perm.data_ptr()),
                                     ctypes.byref(rank), ctypes.byref(st), _stream_ptr(stream))
    _lib.check("qrp_factor_ex", code)
    stats = {k: getattr(st, k) for k, _ in _lib.Stats._fields_}
    return Factorization(tau_house[: min(m, n)], perm[:n], rank.value, stats, [])


def lstsq(A, fac: Factorization, B, rank: int | None = None, stream=None):
    """Basic least-squares solution from a factorization of A (qrdm_lstsq).
    B (m x nrhs column-major float64 device tensor, or a vector of length m) is
    overwritten as qrdm_lstsq describes.  Returns (X [n x nrhs] or [n], resid)."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    vec = B.dim() == 1
    Bm = B.view(-1, 1) if vec else B
    if Bm.dtype != torch.float64 or not Bm.is_cuda or Bm.shape[0] != m:
        raise ValueError("B must be a float64 GPU tensor with m rows")
    nrhs = Bm.shape[1]
    if m > 1 and nrhs > 0 and Bm.stride(0) != 1:
        raise ValueError("B must be column-major (stride(0) == 1)")
    ldb = max(Bm.stride(1) if nrhs > 1 else m, m, 1)
    X = torch.empty((max(nrhs, 1), max(n, 1)), dtype=torch.float64, device=A.device).t()
    resid = torch.empty(max(nrhs, 1), dtype=torch.float64, device=A.device)
    r = fac.rank if rank is None else int(rank)
    code = _lib.load().qrdm_lstsq(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(fac.tau_house.data_ptr()),
                                  ctypes.c_void_p(fac.perm.data_ptr()), r, ctypes.c_void_p(Bm.data_ptr()), ldb, nrhs,
                                  ctypes.c_void_p(X.data_ptr()), max(n, 1), ctypes.c_void_p(resid.data_ptr()),
                                  _stream_ptr(stream))
    _lib.check("qrdm_lstsq", code)
    X = X[:n, :nrhs]
    return (X[:, 0] if vec else X), resid[:nrhs]


def truncate_rank(A, rank: int, eps1_scale: float = 0.0, stream=None) -> int:
    """Post-hoc truncated rank from the diagonal of a factored A (qrdm_truncate_rank);
    synchronizes the stream to return a host integer."""
    torch = _torch()
    m, n, lda = _check_matrix(A)
    out = torch.empty(1, dtype=torch.int64, device=A.device)
    code = _lib.load().qrdm_truncate_rank(ctypes.c_void_p(A.data_ptr()), m, n, lda, int(rank), float(eps1_scale),
                                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _lib.check("qrdm_truncate_rank", code)
    return int(out.item())


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


# ---------------------------------------------------------------- batched
def batch_size_class(m: int) -> int:
    """Size class of a batched matrix (the classes of qrdm_batch_plan_create)."""
    return 0 if m <= 64 else 1 if m <= 128 else 2 if m <= 256 else 3


class Batch:
    """Device storage for a batch of matrices: one packed float64 buffer (each
    matrix column-major with lda = max(1, m)), packed tau_house and perm buffers,
    rank and status arrays, and the device pointer arrays the C ABI takes."""

    def __init__(self, shapes, device: str = "cuda"):
        torch = _torch()
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.lda = [max(1, m) for m, _ in self.shapes]
        sizes = [ld * n for ld, (_, n) in zip(self.lda, self.shapes)]
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        psz = [min(m, n) for m, n in self.shapes]
        self.toff = np.concatenate([[0], np.cumsum(psz)]).astype(np.int64)
        self.poff = np.concatenate([[0], np.cumsum([n for _, n in self.shapes])]).astype(np.int64)
        self.data = torch.zeros(max(int(self.off[-1]), 1), dtype=torch.float64, device=device)
        self.tau = torch.zeros(max(int(self.toff[-1]), 1), dtype=torch.float64, device=device)
        self.perm = torch.zeros(max(int(self.poff[-1]), 1), dtype=torch.int32, device=device)
        b = len(self.shapes)
        self.rank = torch.full((max(b, 1),), -2, dtype=torch.int64, device=device)
        self.status = torch.full((max(b, 1),), -1, dtype=torch.int32, device=device)

        def ptrs(t, offs, esize):
            base = t.data_ptr()
            return torch.tensor([base + esize * int(o) for o in offs[:-1]] or [0], dtype=torch.int64,
                                device=device)
        self.a_ptr = ptrs(self.data, self.off, 8)
        self.t_ptr = ptrs(self.tau, self.toff, 8)
        self.p_ptr = ptrs(self.perm, self.poff, 4)

    def __len__(self):
        return len(self.shapes)

    def pointers(self, t):
        """Device array of per-matrix pointers into t, a tensor laid out like
        self.data (e.g. a pristine copy made with data.clone())."""
        torch = _torch()
        base = t.data_ptr()
        return torch.tensor([base + 8 * int(o) for o in self.off[:-1]] or [0], dtype=torch.int64, device=t.device)

    def load(self, mats):
        """Copy host matrices (numpy, any order) into the device buffer."""
        torch = _torch()
        host = np.zeros(max(int(self.off[-1]), 1))
        for i, a in enumerate(mats):
            m, n = self.shapes[i]
            a = np.asarray(a, dtype=np.float64)
            assert a.shape == (m, n)
            host[self.off[i]: self.off[i] + m * n] = a.reshape(-1, order="F")
        self.data.copy_(torch.from_numpy(host))

    def matrix(self, i):
        m, n = self.shapes[i]
        seg = self.data[int(self.off[i]): int(self.off[i]) + m * n].cpu().numpy()
        return seg.reshape((m, n), order="F")

    def tau_house(self, i):
        return self.tau[int(self.toff[i]): int(self.toff[i + 1])].cpu().numpy()

    def subset(self, idx):
        """A batch over some of these matrices, sharing their storage (the
        device pointer arrays are gathered; rank and status are new)."""
        torch = _torch()
        return _SubBatch(self, [int(i) for i in idx])

    def permutation(self, i):
        return self.perm[int(self.poff[i]): int(self.poff[i + 1])].cpu().numpy().astype(np.int64)


class _SubBatch:
    def __init__(self, parent, idx):
        torch = _torch()
        dev = parent.data.device
        self.shapes = [parent.shapes[i] for i in idx]
        self.lda = [parent.lda[i] for i in idx]
        sel = torch.as_tensor(idx or [0], dtype=torch.int64, device=dev)
        self.a_ptr = parent.a_ptr[sel].contiguous()
        self.t_ptr = parent.t_ptr[sel].contiguous()
        self.p_ptr = parent.p_ptr[sel].contiguous()
        self.rank = torch.full((max(len(idx), 1),), -2, dtype=torch.int64, device=dev)
        self.status = torch.full((max(len(idx), 1),), -1, dtype=torch.int32, device=dev)
        self.data = parent.data

    def __len__(self):
        return len(self.shapes)


class BatchRHS:
    """Right-hand sides and solutions of a batch: packed float64 buffers with
    B[i] m_i x nrhs (leading dimension max(1, m_i)) and X[i] n_i x nrhs
    (leading dimension max(1, n_i)), the device pointer arrays, and resid."""

    def __init__(self, batch, nrhs: int):
        torch = _torch()
        dev = batch.data.device
        self.shapes = list(batch.shapes)
        self.nrhs = int(nrhs)
        bsz = [max(1, m) * self.nrhs for m, _ in self.shapes]
        xsz = [max(1, n) * self.nrhs for _, n in self.shapes]
        self.boff = np.concatenate([[0], np.cumsum(bsz)]).astype(np.int64)
        self.xoff = np.concatenate([[0], np.cumsum(xsz)]).astype(np.int64)
        self.b = torch.zeros(max(int(self.boff[-1]), 1), dtype=torch.float64, device=dev)
        self.x = torch.zeros(max(int(self.xoff[-1]), 1), dtype=torch.float64, device=dev)
        self.resid = torch.zeros(max(len(self.shapes) * self.nrhs, 1), dtype=torch.float64, device=dev)
        mk = lambda t, offs: torch.tensor([t.data_ptr() + 8 * int(o) for o in offs[:-1]] or [0],  # noqa: E731
                                          dtype=torch.int64, device=dev)
        self.b_ptr = mk(self.b, self.boff)
        self.x_ptr = mk(self.x, self.xoff)

    def load(self, rhs):
        """Host right-hand sides: per matrix an (m,) or (m, nrhs) array."""
        torch = _torch()
        host = np.zeros(max(int(self.boff[-1]), 1))
        for i, b in enumerate(rhs):
            m = self.shapes[i][0]
            if m == 0:
                continue
            b = np.asarray(b, dtype=np.float64).reshape(m, -1)
            assert b.shape[1] == self.nrhs
            host[self.boff[i]: self.boff[i] + m * self.nrhs] = b.reshape(-1, order="F")
        self.b.copy_(torch.from_numpy(host))

    def rhs(self, i):
        m = self.shapes[i][0]
        seg = self.b[int(self.boff[i]): int(self.boff[i]) + m * self.nrhs].cpu().numpy()
        return seg.reshape((m, self.nrhs), order="F")

    def solution(self, i):
        n = self.shapes[i][1]
        seg = self.x[int(self.xoff[i]): int(self.xoff[i]) + n * self.nrhs].cpu().numpy()
        return seg.reshape((n, self.nrhs), order="F")

    def residual(self, i):
        return self.resid[i * self.nrhs: (i + 1) * self.nrhs].cpu().numpy()


class BatchPlan:
    """qrdm_batch_plan: size classes, longest-first order, launch variant per class."""

    def __init__(self, batch: Batch, tau: float = 0.15, delta: float = 0.9, kmax: int = 64,
                 stop_rule: int = _lib.STOP_PAPER, eps1_scale: float = 0.0, tune=None, certified: bool = False):
        lib = _lib.load()
        p = _params(tau, delta, kmax, stop_rule, _lib.PREC_FP64, 4, eps1_scale, certified=certified)
        b = len(batch)
        arr = lambda v: (ctypes.c_int32 * max(b, 1))(*v)  # noqa: E731
        m = arr([s[0] for s in batch.shapes])
        n = arr([s[1] for s in batch.shapes])
        ld = arr(batch.lda)
        tn = None
        if tune is not None:
            tn = (_lib.BatchTune * _lib.BATCH_CLASSES)(*[_lib.BatchTune(int(v), int(w)) for v, w in tune])
        self._ptr = ctypes.c_void_p()
        code = lib.qrdm_batch_plan_create(m, n, ld, b, ctypes.byref(p), tn, ctypes.byref(self._ptr))
        _lib.check("qrdm_batch_plan_create", code)
        self.batch = batch

    def factor(self, params=None, use_graph: bool = False, stream=None, info=None):
        """Factor every matrix of the batch in place (enqueued on the stream).
        info: optional int64 device tensor of 4 * batch entries (outer steps,
        early-stopped panels, scalar-pivoting steps, clock ticks per matrix)."""
        bt = self.batch
        pm = ctypes.c_void_p(params.data_ptr()) if params is not None else None
        inf = ctypes.c_void_p(info.data_ptr()) if info is not None else None
        code = _lib.load().qrdm_batch_factor(self._ptr, ctypes.c_void_p(bt.a_ptr.data_ptr()),
                                             ctypes.c_void_p(bt.t_ptr.data_ptr()),
                                             ctypes.c_void_p(bt.p_ptr.data_ptr()),
                                             ctypes.c_void_p(bt.rank.data_ptr()),
                                             ctypes.c_void_p(bt.status.data_ptr()), pm, inf, 1 if use_graph else 0,
                                             _stream_ptr(stream))
        _lib.check("qrdm_batch_factor", code)

    def factor_checked(self, params, pristine_ptrs, band: float = 0.1, stream=None, info=None):
        """Factor with per-matrix parameters and the online check in the same
        launch (qrdm_batch_factor_checked): a matrix that fails the check is
        restored from pristine and factored again with the plan's parameters.
        pristine_ptrs: Batch.pointers(pristine).  Returns ok (int32 device
        tensor: 1 = kept, 0 = factored again)."""
        torch = _torch()
        bt = self.batch
        ok = torch.zeros(max(len(bt), 1), dtype=torch.int32, device=bt.data.device)
        inf = ctypes.c_void_p(info.data_ptr()) if info is not None else None
        code = _lib.load().qrdm_batch_factor_checked(self._ptr, ctypes.c_void_p(bt.a_ptr.data_ptr()),
                                                     ctypes.c_void_p(bt.t_ptr.data_ptr()),
                                                     ctypes.c_void_p(bt.p_ptr.data_ptr()),
                                                     ctypes.c_void_p(bt.rank.data_ptr()),
                                                     ctypes.c_void_p(bt.status.data_ptr()),
                                                     ctypes.c_void_p(params.data_ptr()),
                                                     ctypes.c_void_p(pristine_ptrs.data_ptr()), float(band),
                                                     ctypes.c_void_p(ok.data_ptr()), inf, _stream_ptr(stream))
        _lib.check("qrdm_batch_factor_checked", code)
        return ok[: len(bt)]

    def lstsq(self, rhs: BatchRHS, stream=None):
        """Basic least-squares solutions of the factored batch (qrdm_batch_lstsq)."""
        bt = self.batch
        code = _lib.load().qrdm_batch_lstsq(self._ptr, ctypes.c_void_p(bt.a_ptr.data_ptr()),
                                            ctypes.c_void_p(bt.t_ptr.data_ptr()), ctypes.c_void_p(bt.p_ptr.data_ptr()),
                                            ctypes.c_void_p(bt.rank.data_ptr()), ctypes.c_void_p(rhs.b_ptr.data_ptr()),
                                            ctypes.c_void_p(rhs.x_ptr.data_ptr()), rhs.nrhs,
                                            ctypes.c_void_p(rhs.resid.data_ptr()), _stream_ptr(stream))
        _lib.check("qrdm_batch_lstsq", code)

    def truncate_rank(self, eps1_scale: float = 0.0, out=None, stream=None):
        """Post-hoc truncated ranks (int64 device tensor) of the factored batch."""
        torch = _torch()
        bt = self.batch
        if out is None:
            out = torch.empty(max(len(bt), 1), dtype=torch.int64, device=bt.data.device)
        code = _lib.load().qrdm_batch_truncate_rank(self._ptr, ctypes.c_void_p(bt.a_ptr.data_ptr()),
                                                    ctypes.c_void_p(bt.rank.data_ptr()), float(eps1_scale),
                                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        _lib.check("qrdm_batch_truncate_rank", code)
        return out[: len(bt)]

    def features(self, out=None, stream=None):
        """Per-matrix features (float64 device tensor [batch, 16])."""
        torch = _torch()
        bt = self.batch
        if out is None:
            out = torch.zeros((max(len(bt), 1), _lib.NFEAT), dtype=torch.float64, device=bt.data.device)
        code = _lib.load().qrdm_batch_features(self._ptr, ctypes.c_void_p(bt.a_ptr.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        _lib.check("qrdm_batch_features", code)
        return out[: len(bt)]

    def check(self, band: float = 0.1, stream=None):
        """Online quality check of the current factorization: (ok int32, est float64)."""
        torch = _torch()
        bt = self.batch
        dev = bt.data.device
        ok = torch.zeros(max(len(bt), 1), dtype=torch.int32, device=dev)
        est = torch.zeros(max(len(bt), 1), dtype=torch.float64, device=dev)
        code = _lib.load().qrdm_batch_check(self._ptr, ctypes.c_void_p(bt.a_ptr.data_ptr()),
                                            ctypes.c_void_p(bt.rank.data_ptr()), float(band),
                                            ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(ok.data_ptr()),
                                            _stream_ptr(stream))
        _lib.check("qrdm_batch_check", code)
        return ok[: len(bt)], est[: len(bt)]

    def close(self):
        if self._ptr:
            _lib.load().qrdm_batch_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_params(tau, delta, kmax, device: str = "cuda"):
    """Per-matrix (tau, delta, kmax) as the device array of qrdm_batch_params."""
    torch = _torch()
    b = len(tau)
    raw = np.zeros(b, dtype=[("tau", "<f8"), ("delta", "<f8"), ("kmax", "<i4"), ("pad", "<i4")])
    raw["tau"], raw["delta"], raw["kmax"] = tau, delta, kmax
    return torch.from_numpy(raw.view(np.uint8).copy()).to(device)


# ---------------------------------------------------------------- MLP
def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def mlp_forward(params, features, norm=None, h1=None, h2=None, stream=None):
    """y [B, 3] (float32 device) for features [B, 16] (float64 device)."""
    torch = _torch()
    b = features.shape[0]
    dev = features.device
    y = torch.empty((max(b, 1), _lib.MLP_OUT), dtype=torch.float32, device=dev)
    code = _lib.load().qrdm_mlp_forward(_vp(params), _vp(norm), _vp(features.contiguous()), b, _vp(h1), _vp(h2),
                                        _vp(y), _stream_ptr(stream))
    _lib.check("qrdm_mlp_forward", code)
    return y[:b]


def mlp_gradient(params, features, target, norm=None, stream=None):
    """(grad [5443], y [B, 3], sqerr [B]) of the squared loss, all float32 device."""
    torch = _torch()
    b = features.shape[0]
    dev = features.device
    feats = features.contiguous()
    h1 = torch.empty((b, _lib.MLP_HIDDEN), dtype=torch.float32, device=dev)
    h2 = torch.empty_like(h1)
    y = torch.empty((b, _lib.MLP_OUT), dtype=torch.float32, device=dev)
    lib = _lib.load()
    code = lib.qrdm_mlp_forward(_vp(params), _vp(norm), _vp(feats), b, _vp(h1), _vp(h2), _vp(y), _stream_ptr(stream))
    _lib.check("qrdm_mlp_forward", code)
    work = torch.empty(b * _lib.MLP_NDELTA, dtype=torch.float32, device=dev)
    grad = torch.empty(_lib.MLP_NPARAM, dtype=torch.float32, device=dev)
    sq = torch.empty(b, dtype=torch.float32, device=dev)
    code = lib.qrdm_mlp_gradient(_vp(params), _vp(norm), _vp(feats), _vp(h1), _vp(h2), _vp(y),
                                 _vp(target.contiguous()), b, _vp(work), _vp(grad), _vp(sq), _stream_ptr(stream))
    _lib.check("qrdm_mlp_gradient", code)
    return grad, y, sq


def mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    code = _lib.load().qrdm_mlp_adam(_vp(params), _vp(grad), _vp(m), _vp(v), int(t), float(lr), float(beta1),
                                     float(beta2), float(eps), _stream_ptr(stream))
    _lib.check("qrdm_mlp_adam", code)


def mlp_to_params(y, stream=None):
    """MLP outputs [B, 3] -> device array of qrdm_batch_params (24 bytes each)."""
    torch = _torch()
    b = y.shape[0]
    out = torch.zeros(max(b, 1) * 24, dtype=torch.uint8, device=y.device)
    code = _lib.load().qrdm_mlp_to_params(_vp(y.contiguous()), b, _vp(out), _stream_ptr(stream))
    _lib.check("qrdm_mlp_to_params", code)
    return out
