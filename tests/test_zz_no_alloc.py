"""The allocation-free host-buffer transform (fb_fft3d_exec_host_noalloc)
against the allocating one (fb_fft3d_exec_host) through the C ABI: equal bit
for bit on two calls in a row, the second with a smaller grid, both
directions and both storage types; the largest grid the static buffer holds
(2048 x 2048 complex128) is accepted and a larger one is rejected before any
HIP call."""
import numpy as np
import pytest

from paper_2004_09883_amd import fb, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need a GPU"
    fb.load()


def host_grid(shape, dtype, seed):
    x = inputs.uniform_grid(shape, seed)
    return x if dtype == fb.FB_C128 else x.astype(np.complex64)


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
def test_noalloc_equals_exec_host_two_calls(dtype):
    for shape, seed in (((32, 48, 64), 3), ((8, 16, 12), 4)):   # the second call is smaller
        print(f"noalloc dtype={dtype} shape={shape}", flush=True)
        plan = fb.Plan(*shape, dtype)
        x = host_grid(shape, dtype, seed)
        for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
            want = np.empty_like(x)
            fb.fb_fft3d_exec_host(plan, x, want, direction)
            got = np.empty_like(x)
            fb.fb_fft3d_exec_host_noalloc(plan, x, got, direction)
            assert np.array_equal(got, want), (shape, direction)
            y = x.copy()                       # in place on the host
            fb.fb_fft3d_exec_host_noalloc(plan, y, y, direction)
            assert np.array_equal(y, want), (shape, direction)


def test_noalloc_largest_grid_and_limit():
    shape = (1, 2048, 2048)                    # exactly FB_STATIC_SCRATCH_BYTES in complex128
    print(f"noalloc largest grid {shape}", flush=True)
    plan = fb.Plan(*shape, fb.FB_C128)
    x = host_grid(shape, fb.FB_C128, 5)
    want = np.empty_like(x)
    fb.fb_fft3d_exec_host(plan, x, want, fb.FB_FORWARD)
    got = np.empty_like(x)
    fb.fb_fft3d_exec_host_noalloc(plan, x, got, fb.FB_FORWARD)
    assert np.array_equal(got, want)
    # a smaller call right after the largest one
    small = fb.Plan(4, 8, 16, fb.FB_C128)
    xs = host_grid((4, 8, 16), fb.FB_C128, 6)
    ws, gs = np.empty_like(xs), np.empty_like(xs)
    fb.fb_fft3d_exec_host(small, xs, ws, fb.FB_INVERSE)
    fb.fb_fft3d_exec_host_noalloc(small, xs, gs, fb.FB_INVERSE)
    assert np.array_equal(gs, ws)
    # one byte class above the limit: rejected, nothing transformed
    big = fb.Plan(1, 4096, 4096, fb.FB_C64)   # 128 MiB
    xb = np.zeros((1, 4096, 4096), np.complex64)
    with pytest.raises(fb.FbError) as e:
        fb.fb_fft3d_exec_host_noalloc(big, xb, xb, fb.FB_FORWARD)
    assert e.value.code == fb.FB_ERR_UNSUPPORTED_SIZE
    assert "static staging buffer" in e.value.msg
