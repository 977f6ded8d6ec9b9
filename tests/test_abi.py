"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/scs.h declares, and reports errors instead of
crashing when no device is present."""
import ctypes as C
import os

import pytest

from paper_2408_13170_amd import _binding as B


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = B.header_symbols()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert set(B.header_symbols()) <= set(B._SIGS)


def test_null_arguments_are_rejected_without_device():
    L = B.lib()
    assert L.scs_ctx_create(None, 0) == -1
    assert "NULL" in B.scs_last_error()
    assert L.scs_ctx_destroy(None) == 0
    assert L.scs_evaluate(None, 1, None, 0, None, None, 0, None) == -1
    assert L.scs_footprint(None, 1, 1, 0, None) == -1
    assert L.scs_pso_step(None, None, 0, None) == -1


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_context_creation_fails_cleanly_without_gpu():
    h = C.c_void_p()
    rc = B.lib().scs_ctx_create(C.byref(h), 0)
    assert rc == -3 and not h.value
    assert B.scs_last_error()


def test_server_arguments_are_checked_before_any_device_work():
    L = B.lib()
    h = C.c_void_p()
    assert L.scs_server_create(None, 0, 4, 1 << 30, 2) == -1
    assert L.scs_server_create(C.byref(h), 0, 0, 1 << 30, 2) == -1  # no request slot
    assert L.scs_server_create(C.byref(h), 0, 4, 0, 2) == -1        # no memory budget
    assert L.scs_server_create(C.byref(h), 0, 4, 1 << 30, 17) == -1  # too many streams
    assert not h.value
    n = C.c_int32()
    assert L.scs_server_submit(None, None, 1, 1, None, 0, None, None) == -1
    assert L.scs_server_poll(None, None, 0, 0, C.byref(n)) == -1
    assert L.scs_server_destroy(None) == 0
    assert B.scs_server_clock(None) == 0.0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libscs.so the binding raises instead of computing anything
    another way: the product path has no CPU fallback."""
    monkeypatch.setattr(B, "LIBPATH", str(tmp_path / "libscs.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError, match="missing"):
        B.lib()
    with pytest.raises(ImportError):
        B.scs_ctx_create(0)
