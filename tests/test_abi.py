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


class _NoLibrary:
    """Stands in for libscs.so: any call into it fails the test, so a check
    that raises ValueError is shown to act before the library is reached."""

    def __getattr__(self, name):
        raise AssertionError(f"the binding called {name} with arguments it should have refused")


@pytest.fixture
def fake_ctx(monkeypatch):
    info = {"theta_dim": 7, "N": 4, "n_chan": 2, "K": 100}
    monkeypatch.setattr(B, "scs_ctx_info", lambda ctx: dict(info))
    monkeypatch.setattr(B, "_lib", _NoLibrary())
    return C.c_void_p(1)


def test_binding_refuses_wrong_buffers(fake_ctx):
    """dtype, theta width and buffer lengths are checked against the context
    before a raw pointer goes to the kernels (which would index past a short
    or narrow buffer)."""
    import numpy as np

    ctx = fake_ctx
    P = 5
    good_th, good_u = np.zeros((P, 7)), np.zeros(P)
    bad = [
        lambda: B.scs_evaluate(ctx, good_th.astype(np.float32), good_u),       # float32 theta
        lambda: B.scs_evaluate(ctx, np.zeros((P, 8)), good_u),                 # 8 entries on a 7-entry context
        lambda: B.scs_evaluate(ctx, good_th, np.zeros(P - 1)),                 # short ups
        lambda: B.scs_evaluate(ctx, good_th, good_u.astype(np.float32)),       # float32 ups
        lambda: B.scs_evaluate(ctx, good_th, good_u, seg=np.zeros((P, 3, 3))),  # seg rows for another N
        lambda: B.scs_evaluate_stats(ctx, good_th, np.zeros((P, 4))),          # stats rows too narrow
        lambda: B.scs_loglike(ctx, np.zeros((P, 5)), np.ones(P - 1)),          # amp too short
        lambda: B.scs_load_data(ctx, np.zeros((2, 99, 2)), np.ones((2, 100)), 0.016, 1e-6),  # data / psd shapes
        lambda: B.scs_waveform(ctx, np.zeros(7), np.zeros((1, 100, 2))),       # h for another channel count
        lambda: B.scs_waveform(ctx, np.zeros(6), np.zeros((2, 100, 2))),       # short theta
        lambda: B.scs_swarm_create(ctx, 8, np.zeros(6), np.ones(6)),           # prior box of 6 entries
        lambda: B.scs_server_submit(None, ctx, 4, np.zeros((P, 8)), good_u),   # theta width
    ]
    for i, f in enumerate(bad):
        with pytest.raises(ValueError):
            f()


def test_binding_refuses_host_buffers_for_device_only_calls(fake_ctx):
    torch = pytest.importorskip("torch")
    ctx = fake_ctx
    th = torch.zeros((3, 7), dtype=torch.float64)  # CPU tensors: host memory
    u = torch.zeros(3, dtype=torch.float64)
    with pytest.raises(ValueError):
        B.scs_evaluate_batched([(ctx, 4, th, u)])
    with pytest.raises(ValueError):
        B.scs_pso_move(th, torch.zeros((3, 6), dtype=torch.float64), th, torch.zeros(7, dtype=torch.float64),
                       None, None, None, None, 0, 0, 0)
