"""CPU checks of the HIP library's host side: it builds, loads, exports every
entry point the header declares, and rejects bad limits before touching the
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gsta.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsta_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    syms = declared_symbols()
    assert len(syms) >= 11
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(_lib.EXPORTS)


def test_create_rejects_bad_limits_without_device():
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    bad = [
        _lib.Limits(0, 1, 64, 64, 100, 16, 16, 1),        # no Gaussians
        _lib.Limits(10, 9, 64, 64, 100, 16, 16, 1),       # too many views
        _lib.Limits(10, 1, 64, 64, 100, 8, 8, 1),         # tile size
        _lib.Limits(10, 1, 64, 64, 1 << 33, 16, 16, 1),   # capacity beyond 32-bit
        _lib.Limits(10, 8, 4096, 4096, 100, 16, 16, 1),   # tile keys beyond 16 bits
    ]
    for lim in bad:
        h = ctypes.c_void_p()
        st = L.gsta_create(ctypes.byref(lim), ctypes.byref(h))
        assert st == _lib.GSTA_ERR_INVALID
        assert L.gsta_last_error(h)
        L.gsta_destroy(h)


def test_null_context_is_invalid():
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    assert L.gsta_render_forward(None, None, None, 1, None, None, 0, None) == _lib.GSTA_ERR_INVALID
    assert L.gsta_check(None, None, None) == _lib.GSTA_ERR_INVALID


def test_product_path_fails_loudly_without_library(tmp_path):
    from paper_2504_06716_amd import _lib
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(RuntimeError):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved


def test_noalloc_loss_validates_on_the_host():
    """The context-free loss rejects counts beyond its stated maximum and
    NULL pointers before touching the device, with a message for
    gsta_last_error(NULL)."""
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    p = ctypes.c_void_p(16)          # never dereferenced: the call is rejected first
    for count in (0, -1, _lib.L1_NOALLOC_MAX_COUNT + 1):
        assert L.gsta_l1_loss_noalloc(p, p, count, p, p, None) == _lib.GSTA_ERR_INVALID
        assert b"outside" in L.gsta_last_error(None)
    assert L.gsta_l1_loss_noalloc(p, None, 10, p, p, None) == _lib.GSTA_ERR_INVALID
    assert b"NULL" in L.gsta_last_error(None)
