"""The C-ABI library loads without a GPU, exports every function that
include/ttsh.h declares, and rejects invalid arguments before any device work."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_2304_03306_amd import ttsh

ROOT = Path(__file__).resolve().parents[1]


def declared(header):
    text = (ROOT / "include" / header).read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:ttsh|fno)_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not ttsh.LIB_PATH.exists():
        from paper_2304_03306_amd import build
        build.build(verbose=False)
    return ttsh.lib()


@pytest.mark.parametrize("header", ["ttsh.h", "fno.h"])
def test_exports_every_declared_symbol(lib, header):
    names = declared(header)
    assert len(names) >= (15 if header == "ttsh.h" else 10)
    for n in names:
        assert hasattr(lib, n), n


def test_rejects_bad_arguments_before_device_work(lib):
    p = ttsh.make_params(type("P", (), dict(alpha=-1.0, beta=1.0, gamma0=-1.0, gamma2=1.0, lambda0=3.0,
                                            lambda1=0.0, gamma_v=100.0, gamma_w=0.0, dt=0.01))())
    ctx = ctypes.c_void_p()
    N = (ctypes.c_int * 1)(100)
    L = (ctypes.c_double * 1)(10.0)
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 32, None) == ttsh.TTSH_EUNSUPPORTED
    assert "N must be" in ttsh.ttsh_last_error()
    N[0] = 16384
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 64, None) == ttsh.TTSH_EUNSUPPORTED
    assert "N must be" in ttsh.ttsh_last_error()
    N[0] = 8192  # FP64 transforms of 8192 points do not fit one workgroup's LDS
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 64, None) == ttsh.TTSH_EUNSUPPORTED
    assert "FP32 transforms" in ttsh.ttsh_last_error()
    N[0] = 64
    assert lib.ttsh_create(ctypes.byref(ctx), 0, N, L, ctypes.byref(p), 32, None) == ttsh.TTSH_EINVAL
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 16, None) == ttsh.TTSH_EINVAL
    L[0] = -1.0
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 32, None) == ttsh.TTSH_EINVAL
    L[0] = 10.0
    p.dt = float("nan")
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 32, None) == ttsh.TTSH_EINVAL
    p.dt = 0.01
    p.scheme = 7
    assert lib.ttsh_create(ctypes.byref(ctx), 1, N, L, ctypes.byref(p), 32, None) == ttsh.TTSH_EINVAL
    assert lib.ttsh_step(None, 1) == ttsh.TTSH_EINVAL
    assert lib.ttsh_sync(None) == ttsh.TTSH_EINVAL
    assert lib.ttsh_fft2(None, None, 64, 1, 0, 64) == ttsh.TTSH_EINVAL
    assert lib.ttsh_set_option(None, 1, 1) == ttsh.TTSH_EINVAL
