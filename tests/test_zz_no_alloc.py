"""qrdm_factor_noalloc, the entry point for callers that cannot allocate: it runs
in the library's fixed device scratch and must give exactly what
qrdm_factor_ws gives in a caller-owned workspace (same kernels; the host only
polls differently), on consecutive calls whose scratch holds the previous
call's contents, the second call on a smaller matrix.  After a first call on
the device, further calls leave the device's free memory unchanged."""
import numpy as np
import pytest

import oracle
from paper_2106_03138_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[noalloc] {msg}", flush=True)


def _gpu():
    import paper_2106_03138_amd as Q
    Q.load()
    return Q


CASES = [
    # (name, matrix, parameters): a geometric spectrum into the noise level (DM
    # blocks, then the switch to scalar pivoting), then a smaller matrix
    ("geometric_1500x1300", lambda: I.from_spectrum(1500, 1300, np.geomspace(1.0, 1e-16, 1300), 31),
     dict(tau=0.15, delta=0.9, kmax=64, stop_rule=oracle.STOP_NONE)),
    ("rank64_256", lambda: I.small_rank64(3),
     dict(tau=0.9, delta=0.9, kmax=32, stop_rule=oracle.STOP_PAPER)),
    ("gaussian_300x200", lambda: I.gaussian(300, 200, 32),
     dict(tau=0.15, delta=0.9, kmax=64, stop_rule=oracle.STOP_PAPER)),
]


def _ws_reference(Q, a, kw):
    import torch
    dev = torch.device("cuda")
    A = Q.device_matrix(a)
    ws = torch.empty(Q.api.workspace_size(*a.shape, kw["kmax"]), dtype=torch.uint8, device=dev)
    rk = torch.full((1,), -7, dtype=torch.int64, device=dev)
    o = Q.api.qrdm_factor_ws(A, ws, rk, **kw)
    torch.cuda.synchronize()
    return Q.host_matrix(A), o.tau_house.cpu().numpy(), o.perm.cpu().numpy(), int(rk.item())


def test_noalloc_matches_workspace_entry_on_consecutive_calls():
    import torch
    Q = _gpu()
    dev = torch.device("cuda")
    mats = [(name, make(), kw) for name, make, kw in CASES]
    refs = []
    for name, a, kw in mats:
        _say(f"qrdm_factor_ws {name}")
        refs.append(_ws_reference(Q, a, kw))
    # every tensor of the calls below exists before the first of them
    inputs = [Q.device_matrix(a) for _, a, _ in mats]
    work = [torch.empty_like(x.t().contiguous()).t() for x in inputs]
    taus = [torch.empty(min(a.shape), dtype=torch.float64, device=dev) for _, a, _ in mats]
    perms = [torch.empty(a.shape[1], dtype=torch.int32, device=dev) for _, a, _ in mats]
    ranks = [torch.full((1,), -7, dtype=torch.int64, device=dev) for _ in mats]
    torch.cuda.synchronize()
    free = []
    for rep in range(2):
        for i, (name, a, kw) in enumerate(mats):
            _say(f"qrdm_factor_noalloc {name} (pass {rep})")
            work[i].copy_(inputs[i])
            ranks[i].fill_(-7)
            torch.cuda.synchronize()
            before = torch.cuda.mem_get_info()[0]
            Q.api.qrdm_factor_noalloc(work[i], ranks[i], tau_house=taus[i], perm=perms[i], **kw)
            torch.cuda.synchronize()
            after = torch.cuda.mem_get_info()[0]
            if rep > 0 or i > 0:
                free.append(after - before)
            qr, tau, perm, rank = refs[i]
            assert int(ranks[i].item()) == rank, (name, int(ranks[i].item()), rank)
            assert np.array_equal(perms[i].cpu().numpy(), perm), name
            assert np.array_equal(taus[i].cpu().numpy(), tau), name
            assert np.array_equal(Q.host_matrix(work[i]), qr), name
    assert all(d == 0 for d in free), free


def test_noalloc_rejects_shapes_beyond_the_scratch():
    import ctypes
    Q = _gpu()
    assert Q.api.workspace_size(16384, 16384, 64) > Q._lib.NOALLOC_WS_MAX
    d = ctypes.c_void_p(4096)  # never dereferenced: the size is refused before any launch
    p = Q._lib.Params()
    Q.load().qrdm_default_params(ctypes.byref(p))
    assert Q.load().qrdm_factor_noalloc(d, 16384, 16384, 16384, ctypes.byref(p), d, d, d, None) == Q._lib.ERR_SCRATCH
