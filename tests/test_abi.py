"""The C ABI without a GPU: libqrdm.so loads, exports every function that
include/qrdm.h declares, and the ctypes mirrors of the header's structs have
the header's layout.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qrdm.h")
LIB = os.path.join(ROOT, "paper_2106_03138_amd", "libqrdm.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("QRDM")))


def _struct_sizes():
    """sizeof/offsetof of the header's structs, from a host C compiler."""
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "qrdm.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(qrdm_params), sizeof(qrdm_stats), sizeof(qrdm_block));
  printf("%zu %zu %zu\n", offsetof(qrdm_params, eps1_scale), offsetof(qrdm_params, profile),
         offsetof(qrdm_stats, total_ms));
  printf("%zu %zu\n", offsetof(qrdm_block, fallback), offsetof(qrdm_block, umax));
  printf("%zu %zu %zu\n", offsetof(qrdm_params, certified), offsetof(qrdm_block, gamma),
         offsetof(qrdm_block, sigma_bound));
  printf("%zu %zu %zu\n", sizeof(qrdm_batch_params), offsetof(qrdm_batch_params, kmax), sizeof(qrdm_batch_tune));
  printf("%zu\n", offsetof(qrdm_stats, qp3_start));
  return 0;
}
"""
    return src


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libqrdm.so not built (python -m paper_2106_03138_amd.build)")
    import torch  # noqa: F401  (same HIP runtime as the library)
    return ctypes.CDLL(LIB)


def test_header_declares_the_expected_entry_points():
    names = _declared_functions()
    for want in ["qrdm_factor", "qrdm_factor_ex", "qrdm_factor_ws", "qrdm_factor_noalloc", "qrdm_workspace_size",
                 "qrp_factor", "qrp_factor_ex", "qrdm_colnorms",
                 "qrdm_dm_step", "qrdm_default_params", "qrdm_release", "qrdm_strerror", "qrdm_lstsq",
                 "qrdm_batch_lstsq", "qrdm_truncate_rank", "qrdm_batch_truncate_rank"]:
        assert want in names, names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2106_03138_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared_functions()


def test_struct_layouts_match_the_header(tmp_path):
    from paper_2106_03138_amd import _lib
    c = tmp_path / "sizes.c"
    c.write_text(_struct_sizes())
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = [int(x) for x in out]
    want = [ctypes.sizeof(_lib.Params), ctypes.sizeof(_lib.Stats), ctypes.sizeof(_lib.Block),
            _lib.Params.eps1_scale.offset, _lib.Params.profile.offset, _lib.Stats.total_ms.offset,
            _lib.Block.fallback.offset, _lib.Block.umax.offset,
            _lib.Params.certified.offset, _lib.Block.gamma.offset, _lib.Block.sigma_bound.offset,
            ctypes.sizeof(_lib.BatchParams), _lib.BatchParams.kmax.offset, ctypes.sizeof(_lib.BatchTune),
            _lib.Stats.qp3_start.offset]
    assert got == want


def test_defaults_and_error_strings_without_a_device(lib):
    from paper_2106_03138_amd import _lib
    lib.qrdm_default_params.argtypes = [ctypes.POINTER(_lib.Params)]
    p = _lib.Params()
    lib.qrdm_default_params(ctypes.byref(p))
    assert (p.tau, p.delta, p.kmax, p.stop_rule, p.precision, p.certified) == (0.15, 0.9, 64, 0, 0, 0)
    lib.qrdm_strerror.restype = ctypes.c_char_p
    lib.qrdm_strerror.argtypes = [ctypes.c_int]
    for code in (0, 1, 2, 3, 4, 5, -1, 1001):
        assert lib.qrdm_strerror(code)


def test_invalid_arguments_are_rejected_before_any_launch(lib):
    """Argument checks run on the host and return -i without touching the device."""
    from paper_2106_03138_amd import _lib
    f = lib.qrdm_factor_ex
    f.restype, f.argtypes = _lib.SIGNATURES["qrdm_factor_ex"]
    p = _lib.Params()
    lib.qrdm_default_params(ctypes.byref(p))
    rank = ctypes.c_int64(0)
    nlog = ctypes.c_int64(0)
    dummy = ctypes.c_void_p(16)
    # m < 0
    assert f(dummy, -1, 4, 4, ctypes.byref(p), dummy, dummy, ctypes.byref(rank), None, None, 0,
             ctypes.byref(nlog), None) == -2
    # lda < m
    assert f(dummy, 8, 4, 4, ctypes.byref(p), dummy, dummy, ctypes.byref(rank), None, None, 0,
             ctypes.byref(nlog), None) == -4
    # kmax beyond the supported limit
    p.kmax = 129
    assert f(dummy, 8, 4, 8, ctypes.byref(p), dummy, dummy, ctypes.byref(rank), None, None, 0,
             ctypes.byref(nlog), None) == -5


def test_batched_plan_rejects_bad_arguments_on_the_host(lib):
    """Plan creation validates sizes and parameters before touching the device."""
    from paper_2106_03138_amd import _lib
    f = lib.qrdm_batch_plan_create
    f.restype, f.argtypes = _lib.SIGNATURES["qrdm_batch_plan_create"]
    p = _lib.Params()
    lib.qrdm_default_params(ctypes.byref(p))
    arr = lambda *v: (ctypes.c_int32 * len(v))(*v)  # noqa: E731
    plan = ctypes.c_void_p()
    # n beyond the batched limit
    assert f(arr(600, 8), arr(600, 4), arr(600, 8), 2, ctypes.byref(p), None, ctypes.byref(plan)) == 3
    # lda < m
    assert f(arr(8), arr(4), arr(4), 1, ctypes.byref(p), None, ctypes.byref(plan)) == -3
    # negative m, negative batch
    assert f(arr(-1), arr(4), arr(4), 1, ctypes.byref(p), None, ctypes.byref(plan)) == -1
    assert f(arr(8), arr(4), arr(8), -1, ctypes.byref(p), None, ctypes.byref(plan)) == -4
    # k_DM beyond the batched limit; mixed precision is not offered for batches
    p.kmax = 65
    assert f(arr(8), arr(4), arr(8), 1, ctypes.byref(p), None, ctypes.byref(plan)) == 3
    p.kmax, p.precision = 64, 1
    assert f(arr(8), arr(4), arr(8), 1, ctypes.byref(p), None, ctypes.byref(plan)) == -5
    # an unknown launch variant
    p.precision = 0
    tune = (_lib.BatchTune * 4)(*[_lib.BatchTune(9, 0)] * 4)
    assert f(arr(8), arr(4), arr(8), 1, ctypes.byref(p), tune, ctypes.byref(plan)) == -6
    assert not plan.value


def test_lstsq_and_truncation_reject_bad_arguments_on_the_host(lib):
    from paper_2106_03138_amd import _lib
    f = lib.qrdm_lstsq
    f.restype, f.argtypes = _lib.SIGNATURES["qrdm_lstsq"]
    d = ctypes.c_void_p(16)
    assert f(d, -1, 4, 4, d, d, 2, d, 4, 1, d, 4, None, None) == -2
    assert f(d, 8, 4, 4, d, d, 2, d, 8, 1, d, 4, None, None) == -4
    assert f(d, 8, 4, 8, d, d, 2, d, 4, 1, d, 4, None, None) == -9
    assert f(d, 8, 4, 8, d, d, 2, d, 8, -1, d, 4, None, None) == -10
    assert f(d, 8, 4, 8, d, d, 2, d, 8, 1, d, 2, None, None) == -12
    assert f(d, 8, 4, 8, d, d, 2, None, 8, 1, d, 4, None, None) == -8
    assert f(d, 8, 4, 8, d, d, 2, d, 8, 0, d, 4, None, None) == 0  # nothing to solve
    t = lib.qrdm_truncate_rank
    t.restype, t.argtypes = _lib.SIGNATURES["qrdm_truncate_rank"]
    assert t(d, 8, 4, 4, 2, 0.0, d, None) == -4
    assert t(d, 8, 4, 8, 2, 0.0, None, None) == -7
    assert t(d, 8, 4, 8, 2, float("nan"), d, None) == -6


def test_workspace_size_and_ws_arguments_on_the_host(lib):
    """qrdm_workspace_size is a host computation; qrdm_factor_ws rejects a missing,
    misaligned or short workspace before touching the device."""
    from paper_2106_03138_amd import _lib
    ws = lib.qrdm_workspace_size
    ws.restype, ws.argtypes = _lib.SIGNATURES["qrdm_workspace_size"]
    p = _lib.Params()
    lib.qrdm_default_params(ctypes.byref(p))
    assert ws(-1, 4, ctypes.byref(p)) == 0
    small, big = ws(256, 256, ctypes.byref(p)), ws(8192, 8192, ctypes.byref(p))
    assert 0 < small < big
    assert ws(256, 256, None) == small  # NULL = the defaults (k_DM = 64)
    # the largest parts grow with k_DM: partial products of V^T A and the Gram partials
    p.kmax = 128
    assert ws(4096, 4096, ctypes.byref(p)) > ws(4096, 4096, None)
    p.kmax = 64
    # 8192^2 with k_DM = 64 stays under 100 MB (about 0.03% of the device memory)
    assert big < 100 * 2 ** 20
    f = lib.qrdm_factor_ws
    f.restype, f.argtypes = _lib.SIGNATURES["qrdm_factor_ws"]
    d = ctypes.c_void_p(4096)
    need = ws(64, 48, ctypes.byref(p))
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, d, None, None, need, None) == -10
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, ctypes.c_void_p(4096 + 8), None, ctypes.c_void_p(4104),
             need, None) == -10  # misaligned workspace
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, d, None, d, need - 1, None) == _lib.ERR_WORKSPACE
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, None, None, d, need, None) == -8
    assert f(d, 64, 48, 32, ctypes.byref(p), d, d, d, None, d, need, None) == -4
    p.profile = 1
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, d, None, d, need, None) == -5


def test_noalloc_arguments_and_size_limit_on_the_host(lib):
    """qrdm_factor_noalloc checks its arguments and the scratch limit before it
    touches the device: shapes whose workspace exceeds QRDM_NOALLOC_WS_MAX are
    refused with QRDM_ERR_SCRATCH."""
    from paper_2106_03138_amd import _lib
    ws = lib.qrdm_workspace_size
    ws.restype, ws.argtypes = _lib.SIGNATURES["qrdm_workspace_size"]
    f = lib.qrdm_factor_noalloc
    f.restype, f.argtypes = _lib.SIGNATURES["qrdm_factor_noalloc"]
    p = _lib.Params()
    lib.qrdm_default_params(ctypes.byref(p))
    text = open(HEADER).read()
    assert re.search(r"#define QRDM_NOALLOC_WS_MAX \(\(size_t\)96 << 20\)", text)
    assert _lib.NOALLOC_WS_MAX == 96 << 20
    assert ws(8192, 8192, ctypes.byref(p)) <= _lib.NOALLOC_WS_MAX  # the benchmark's shape fits
    d = ctypes.c_void_p(4096)
    assert ws(16384, 16384, ctypes.byref(p)) > _lib.NOALLOC_WS_MAX
    assert f(d, 16384, 16384, 16384, ctypes.byref(p), d, d, d, None) == _lib.ERR_SCRATCH
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, None, None) == -8
    assert f(d, 64, 48, 32, ctypes.byref(p), d, d, d, None) == -4
    assert f(d, 64, 48, 64, ctypes.byref(p), None, d, d, None) == -6
    assert f(d, 64, 48, 64, ctypes.byref(p), d, None, d, None) == -7
    p.profile = 1
    assert f(d, 64, 48, 64, ctypes.byref(p), d, d, d, None) == -5
    msg = lib.qrdm_strerror
    msg.restype, msg.argtypes = _lib.SIGNATURES["qrdm_strerror"]
    assert b"QRDM_NOALLOC_WS_MAX" in msg(_lib.ERR_SCRATCH)
