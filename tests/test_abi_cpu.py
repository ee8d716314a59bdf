"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point the header declares, describes plans exactly as the oracle's
radix rule does, and rejects invalid arguments before touching the device
(the paper's step C-2, section 3.4: a mismatched interface is reported, not
coerced)."""
import ctypes
import os
import re

import pytest

import oracle
from paper_2004_09883_amd import fb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "fb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = fb.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(fb.EXPORTS) == names


def test_version():
    assert fb.fb_version() >= 100


SHAPES = [(512, 256, 256), (256, 256, 128), (64, 64, 64), (32, 32, 32), (128, 256, 512), (1, 512, 512),
          (1, 1, 1), (3, 6, 12), (4096, 2, 1), (768, 96, 24), (1, 3072, 48), (2, 1, 1536),
          (9, 27, 81), (2187, 1, 18), (2304, 3456, 3888), (729, 1458, 2916), (144, 36, 2592)]


@pytest.mark.parametrize("shape", SHAPES)
def test_describe_matches_oracle(shape):
    for dt in (fb.FB_C128, fb.FB_C64, fb.FB_C64_SPLITBF16):
        assert fb.fb_describe_shape(*shape, dt) == oracle.describe(*shape)


def _is_2a3b(n):
    while n % 2 == 0:
        n //= 2
    while n % 3 == 0:
        n //= 3
    return n == 1


ALL_LENGTHS = [n for n in range(2, 4097) if _is_2a3b(n)]


def test_every_supported_length_has_a_pass_on_every_axis():
    """Every axis length 2^a 3^b up to 4096 (55 of them) describes on every
    axis and in every dtype: the host-side lookup finds an instantiated pass
    (the lookup a plan makes), and the radix list equals the oracle's."""
    assert len(ALL_LENGTHS) == 55
    for n in ALL_LENGTHS:
        for shape in ((1, 1, n), (1, n, 2), (n, 2, 1)):
            for dt in (fb.FB_C128, fb.FB_C64, fb.FB_C64_SPLITBF16):
                assert fb.fb_describe_shape(*shape, dt) == oracle.describe(*shape), (shape, dt)


@pytest.mark.parametrize("shape,code", [((0, 4, 4), fb.FB_ERR_INVALID_ARG), ((4, -1, 4), fb.FB_ERR_INVALID_ARG),
                                        ((5, 4, 4), fb.FB_ERR_UNSUPPORTED_SIZE),
                                        ((4, 4, 8192), fb.FB_ERR_UNSUPPORTED_SIZE),
                                        ((4, 7, 4), fb.FB_ERR_UNSUPPORTED_SIZE),
                                        ((4, 4, 6561), fb.FB_ERR_UNSUPPORTED_SIZE),
                                        ((10, 4, 4), fb.FB_ERR_UNSUPPORTED_SIZE),
                                        ((4, 4, 6144), fb.FB_ERR_UNSUPPORTED_SIZE)])
def test_describe_rejects_shapes(shape, code):
    with pytest.raises(fb.FbError) as e:
        fb.fb_describe_shape(*shape)
    assert e.value.code == code
    assert fb.fb_last_error()[0] == code


def test_describe_rejects_dtype():
    with pytest.raises(fb.FbError) as e:
        fb.fb_describe_shape(8, 8, 8, 7)
    assert e.value.code == fb.FB_ERR_DTYPE
    assert "dtype" in e.value.msg


def test_plan_rejects_before_device():
    lib = fb.load()
    assert not lib.fb_fft3d_plan(6, 5, 4, 0)
    assert fb.fb_last_error()[0] == fb.FB_ERR_UNSUPPORTED_SIZE
    assert not lib.fb_fft3d_plan(8, 8, 8, 3)
    assert fb.fb_last_error()[0] == fb.FB_ERR_DTYPE


def test_null_plan_calls_are_rejected():
    lib = fb.load()
    assert lib.fb_fft3d_exec(None, 16, 16, -1, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_spectral_evolve(None, 16, 1e-6, 1.0, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_checksum(None, 16, 16, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_spectral_step(None, 16, 4096, 1e-6, 1.0, None, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_fill_uniform(None, 16, 1, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_plan_device_bytes(None) == 0
    assert lib.fb_server_set_policy(None, fb.FB_SERVE_DEADLINE) == fb.FB_ERR_INVALID_ARG
    lib.fb_fft3d_destroy(None)   # NULL-safe


def test_last_error_clears_on_success():
    fb.fb_describe_shape(8, 8, 8)
    assert fb.fb_last_error() == (0, "")


def test_batch_plan_rejects_before_device():
    lib = fb.load()
    import ctypes
    arr = (ctypes.c_int64 * 3)(256, 5, 1024)
    assert not lib.fb_batch_plan(arr, 3, 0, 0, fb.FB_C64)
    assert fb.fb_last_error()[0] == fb.FB_ERR_UNSUPPORTED_SIZE
    arr = (ctypes.c_int64 * 1)(1 << 22)
    assert not lib.fb_batch_plan(arr, 1, 0, 0, fb.FB_C64)
    assert fb.fb_last_error()[0] == fb.FB_ERR_UNSUPPORTED_SIZE
    assert not lib.fb_batch_plan(arr, 0, 0, 0, fb.FB_C64)
    assert fb.fb_last_error()[0] == fb.FB_ERR_INVALID_ARG
    assert not lib.fb_batch_plan(arr, 0, 2, 500, fb.FB_C64)
    assert fb.fb_last_error()[0] == fb.FB_ERR_UNSUPPORTED_SIZE
    assert not lib.fb_batch_plan(arr, 0, 2, 512, fb.FB_C128)
    assert fb.fb_last_error()[0] == fb.FB_ERR_DTYPE
    assert lib.fb_batch_exec(None, 16, 16, 256, 1 << 20, -1, 1, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_batch_elements(None) == 0
    lib.fb_batch_destroy(None)


def test_lu_and_steps_reject_before_device():
    """Argument checks of the LU block and the multi-step call run before any
    HIP call (no device here)."""
    lib = fb.load()
    assert lib.fb_lu_factor(16, 0, 0, 32, 64, None) == fb.FB_ERR_UNSUPPORTED_SIZE
    assert lib.fb_lu_factor(16, 4096, 4096, 32, 64, None) == fb.FB_ERR_UNSUPPORTED_SIZE
    assert lib.fb_lu_factor(16, 8, 4, 32 << 10, 64 << 10, None) == fb.FB_ERR_INVALID_ARG    # lda < n
    assert lib.fb_lu_factor(None, 8, 8, 32 << 10, 64 << 10, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_lu_factor(12, 8, 8, 32 << 10, 64 << 10, None) == fb.FB_ERR_INVALID_ARG   # misaligned
    assert lib.fb_lu_factor(1 << 20, 8, 8, (1 << 20) + 64, 64 << 20, None) == fb.FB_ERR_INVALID_ARG  # overlap
    ts = (ctypes.c_double * 2)(1.0, 2.0)
    assert lib.fb_spectral_steps(None, 16, 16, 1e-6, ts, 2, None, None) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_fft3d_exec_host(None, 16, 16, -1) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_fft3d_exec_host_noalloc(None, 16, 16, -1) == fb.FB_ERR_INVALID_ARG
    assert lib.fb_fft3d_forward_uniform(None, 1, 16, None) == fb.FB_ERR_INVALID_ARG


class _RecordingLib:
    """Stands in for libfb: records every entry point called."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def f(*args):
            self.calls.append(name)
            return 0
        return f


class _FakePlan:
    """A plan whose grid checks pass, so that only the checksum buffers are
    judged (no device here to make a real plan)."""
    shape = (4, 4, 4)
    handle = 1

    def check_tensor(self, x, name="x"):
        return None

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128


def _bad_sums():
    import torch
    return [
        ("cpu tensor", torch.zeros(2, dtype=torch.float64), fb.FB_ERR_INVALID_ARG),
        ("float32", torch.zeros(2, dtype=torch.float32), fb.FB_ERR_DTYPE),
        ("too small", torch.zeros(1, dtype=torch.float64), None),
        ("not contiguous", torch.zeros(4, dtype=torch.float64)[::2], None),
        ("not a tensor", [0.0, 0.0], fb.FB_ERR_INVALID_ARG),
    ]


@pytest.mark.parametrize("call", ["fb_checksum", "fb_spectral_step", "fb_spectral_steps"])
def test_binding_rejects_bad_checksum_buffers_before_any_call(monkeypatch, call):
    """A checksum destination that is on the host, of the wrong dtype, too
    small or strided raises FbError in the binding and nothing reaches the
    library (the kernel would otherwise write through a host pointer or past
    the allocation)."""
    rec = _RecordingLib()
    monkeypatch.setattr(fb, "_lib", rec)
    plan = _FakePlan()
    for label, sums, code in _bad_sums():
        with pytest.raises(fb.FbError) as e:
            if call == "fb_checksum":
                fb.fb_checksum(plan, 0, sums, stream=0)
            elif call == "fb_spectral_step":
                fb.fb_spectral_step(plan, 0, 0, 1e-6, 1.0, sums, stream=0)
            else:
                fb.fb_spectral_steps(plan, 0, 0, 1e-6, [1.0], sums, stream=0)
        if code is not None:
            assert e.value.code == code, label
        assert rec.calls == [], (label, rec.calls)
    if call == "fb_checksum":
        with pytest.raises(fb.FbError):
            fb.fb_checksum(plan, 0, None, stream=0)
    assert rec.calls == []


def test_binding_steps_sums_sized_for_every_step(monkeypatch):
    """fb_spectral_steps needs 2 values per step: a buffer of 2 values for
    3 steps is rejected before the call."""
    import torch
    rec = _RecordingLib()
    monkeypatch.setattr(fb, "_lib", rec)
    with pytest.raises(fb.FbError) as e:
        fb.fb_spectral_steps(_FakePlan(), 0, 0, 1e-6, [1.0, 2.0, 3.0], torch.zeros(2, dtype=torch.float64),
                             stream=0)
    assert "at least 6" in e.value.msg
    assert rec.calls == []
