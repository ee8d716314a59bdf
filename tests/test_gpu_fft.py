"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.

Bars (relative L2 over the whole grid, per step): complex128 path <= 1e-12,
complex64 path <= 1e-5; checksums are compared with the error normalised by
sum_j |x_ref[17 j]|.  The oracle follows the Fourier-transform block of the
paper (section 5.1(a)) re-created as the 3D spectral block.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2004_09883_amd import fb, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {fb.FB_C128: 1e-12, fb.FB_C64: 1e-5, fb.FB_C64_SPLITBF16: 1e-5}
DTYPES = [fb.FB_C128, fb.FB_C64, fb.FB_C64_SPLITBF16]
LENGTHS = [2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096]
# 2^a 3^b with b >= 2 (repeated radix-3 stages), every one up to 4096
LENGTHS_3B = [9, 18, 36, 72, 144, 288, 576, 1152, 2304, 27, 54, 108, 216, 432, 864, 1728, 3456, 81, 162, 324, 648,
              1296, 2592, 243, 486, 972, 1944, 3888, 729, 1458, 2916, 2187]


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x, dtype):
    t = torch.from_numpy(np.ascontiguousarray(x))
    t = t.to(torch.complex128 if dtype == fb.FB_C128 else torch.complex64)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def as_seen(x, dtype):
    """The values the device holds for a host grid (c64 rounds each part)."""
    return x if dtype == fb.FB_C128 else inputs.round_c64(x).astype(np.complex128)


def checksum_err(got, ref_grid):
    flat = ref_grid.reshape(-1)
    idx = (17 * np.arange(1024)) % flat.size
    return abs(got - oracle.checksum(ref_grid)) / np.sum(np.abs(flat[idx]))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need a GPU"
    fb.load()
    print("device:", torch.cuda.get_device_name(0), flush=True)


def run_fft(shape, dtype, seed=1, direction=fb.FB_FORWARD, inplace=False):
    x = inputs.uniform_grid(shape, seed)
    xs = as_seen(x, dtype)
    plan = fb.Plan(*shape, dtype)
    xin = dev(x, dtype)
    out = xin if inplace else torch.empty_like(xin)
    fb.fb_fft3d_exec(plan, xin, out, direction)
    got = host(out)
    ref = oracle.fft3d(xs, direction)
    return got, ref


# ---------------------------------------------------------------- one axis at a time

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", LENGTHS + LENGTHS_3B)
@pytest.mark.parametrize("axis", ["z", "y", "x"])
def test_single_axis_pass(axis, n, dtype):
    shape = {"z": (1, 3, n), "y": (2, n, 6), "x": (n, 3, 4)}[axis]
    print(f"axis={axis} n={n} dtype={dtype} shape={shape}", flush=True)
    for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
        got, ref = run_fft(shape, dtype, seed=n, direction=direction)
        assert rel_l2(got, ref) < TOL[dtype], (axis, n, direction)


# ---------------------------------------------------------------- whole 3D transforms

SHAPES_3D = [(64, 64, 64), (32, 48, 96), (12, 96, 24), (3, 6, 12), (1, 1, 1), (1, 1, 4096), (4096, 1, 2),
             (2, 4096, 1), (128, 256, 512), (256, 256, 128),
             # pencil counts that leave a part-filled last tile on every axis
             (3, 3, 256), (3, 256, 3), (256, 3, 3), (6, 3, 96),
             # repeated radix-3 stages on every axis
             (9, 27, 36), (18, 81, 54), (144, 9, 2304)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES_3D)
def test_fft3d(shape, dtype):
    print(f"fft3d shape={shape} dtype={dtype}", flush=True)
    for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
        got, ref = run_fft(shape, dtype, seed=7, direction=direction)
        assert rel_l2(got, ref) < TOL[dtype], direction


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
def test_fft3d_in_place_equals_out_of_place(dtype):
    shape = (32, 64, 48)
    a, ref = run_fft(shape, dtype, seed=3)
    b, _ = run_fft(shape, dtype, seed=3, inplace=True)
    assert np.array_equal(a, b)
    assert rel_l2(a, ref) < TOL[dtype]


def test_round_trip_c128():
    shape = (64, 32, 96)
    x = inputs.uniform_grid(shape, 5)
    plan = fb.Plan(*shape, fb.FB_C128)
    t = dev(x, fb.FB_C128)
    fb.fb_fft3d_exec(plan, t, t, fb.FB_FORWARD)
    fb.fb_fft3d_exec(plan, t, t, fb.FB_INVERSE)
    assert rel_l2(host(t), x) < 1e-14


def test_fft3d_config3_full_size_c128():
    """512 x 256 x 256 complex128, Gaussian input: the shape and launch
    configuration the benchmark times."""
    shape = (512, 256, 256)
    x = inputs.gaussian_grid(shape, 2)
    plan = fb.Plan(*shape, fb.FB_C128)
    t = dev(x, fb.FB_C128)
    out = torch.empty_like(t)
    fb.fb_fft3d_exec(plan, t, out, fb.FB_FORWARD)
    got = host(out)
    del out, t
    ref = oracle.fft3d(x, -1)
    assert rel_l2(got, ref) < 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
def test_paper_2d_2048(dtype):
    """The paper's own Fourier-transform size (section 5.1: a 2048 x 2048
    grid), as the benchmark runs it (the 3D plan with nx = 1): forward and
    inverse against the oracle on the same seeded input."""
    shape = (1, 2048, 2048)
    print(f"2048x2048 dtype={dtype}", flush=True)
    for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
        got, ref = run_fft(shape, dtype, seed=7, direction=direction)
        e = rel_l2(got, ref)
        assert e < TOL[dtype], (direction, e)


def test_headline_block_as_benchmarked():
    """The benchmark's headline block at full size and in its launch
    configuration (512 x 256 x 256 complex128, N(0,1) input seed 2, forward
    + 10 fused steps, captured in a HIP graph and replayed): every step's
    checksum and the last step's grid against the oracle."""
    import bench
    shape, steps = bench.SHAPE, bench.T_STEPS
    x0 = inputs.gaussian_grid(shape, bench.SEED)
    blk = bench.SpectralBlock(torch, fb, shape, fb.FB_C128, steps, host_x0=x0, schedule=bench.HEADLINE_SCHEDULE)
    t = bench.time_replays(torch, blk.run, warmup=1, reps=2)
    del t
    sums = blk.sums.cpu().numpy()
    last = host(blk.out if blk.schedule != "fused_steps" else blk.out[steps - 1])
    del blk
    torch.cuda.empty_cache()
    X0 = oracle.fft3d(x0, -1)
    for j in range(steps):
        ref = oracle.fft3d(oracle.evolve(X0, bench.ALPHA, j + 1), +1)
        assert checksum_err(complex(sums[j, 0], sums[j, 1]), ref) < 1e-12, j
        if j == steps - 1:
            assert rel_l2(last, ref) < 1e-12


# ---------------------------------------------------------------- evolve / checksum / inputs

@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
def test_evolve_standalone(dtype):
    shape = (16, 24, 32)
    u = inputs.uniform_grid(shape, 9)
    plan = fb.Plan(*shape, dtype)
    t = dev(u, dtype)
    fb.fb_spectral_evolve(plan, t, 1e-3, 2.5)
    ref = oracle.evolve(as_seen(u, dtype), 1e-3, 2.5)
    assert rel_l2(host(t), ref) < (1e-15 if dtype == fb.FB_C128 else 1e-6)


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
@pytest.mark.parametrize("shape", [(32, 32, 32), (4, 4, 4), (512, 256, 256)])
def test_checksum(shape, dtype):
    x = inputs.uniform_grid(shape, 4)
    plan = fb.Plan(*shape, dtype)
    t = dev(x, dtype)
    out2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    fb.fb_checksum(plan, t, out2)
    got = complex(*out2.cpu().numpy())
    assert checksum_err(got, as_seen(x, dtype)) < 1e-15


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
@pytest.mark.parametrize("shape", [(32, 32, 32), (4, 4, 4), (3, 4, 8)])
def test_checksum_summation_order(shape, dtype):
    """The device sums the 1024 samples by a fixed binary64 tree (level h adds
    sample j + h into sample j for j < h, h = 512 .. 1): equal bit for bit to
    that tree evaluated here, whatever the grid size (small grids wrap the
    sample index)."""
    x = as_seen(inputs.uniform_grid(shape, 6), dtype)
    plan = fb.Plan(*shape, dtype)
    out2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    fb.fb_checksum(plan, dev(x, dtype), out2)
    flat = x.reshape(-1)
    s = flat[(17 * np.arange(1024)) % flat.size].astype(np.complex128)
    re, im = s.real.copy(), s.imag.copy()
    h = 512
    while h > 0:
        re[:h] = re[:h] + re[h:2 * h]
        im[:h] = im[:h] + im[h:2 * h]
        h //= 2
    got = out2.cpu().numpy()
    assert got[0] == re[0] and got[1] == im[0]


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
def test_fill_uniform_bitwise(dtype):
    shape = (8, 12, 48)
    plan = fb.Plan(*shape, dtype)
    t = torch.empty(shape, dtype=plan.torch_dtype, device="cuda")
    fb.fb_fill_uniform(plan, t, 12345)
    want = inputs.uniform_grid(shape, 12345)
    if dtype == fb.FB_C64:
        want = inputs.round_c64(want)
    assert np.array_equal(t.cpu().numpy(), want)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(16, 32, 64), (6, 96, 1), (1, 1, 4096), (3, 1, 1), (1, 1, 1), (64, 256, 512)])
def test_forward_uniform_equals_fill_then_exec(dtype, shape):
    """The forward transform with the input generated inside the first pass
    is the fill followed by the transform, bit for bit; and it matches the
    oracle on the generated grid."""
    plan = fb.Plan(*shape, dtype)
    a = torch.empty(shape, dtype=plan.torch_dtype, device="cuda")
    fb.fb_fill_uniform(plan, a, 777)
    fb.fb_fft3d_exec(plan, a, a, fb.FB_FORWARD)
    b = torch.full(shape, 5.0, dtype=plan.torch_dtype, device="cuda")
    fb.fb_fft3d_forward_uniform(plan, 777, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    if math.prod(shape) <= 1 << 20:
        x = as_seen(inputs.uniform_grid(shape, 777), dtype)
        ref = oracle.fft3d(x, -1)
        assert rel_l2(host(b), ref) < (1e-12 if dtype == fb.FB_C128 else 1e-5)


# ---------------------------------------------------------------- the spectral block


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape,ts", [((16, 32, 64), list(range(1, 12))), ((6, 96, 1), [1, 2, 3]),
                                      ((1, 1, 256), [0.0, 2.5, 7.0]), ((12, 8, 48), [3.0] * 9),
                                      ((64, 64, 64), [1, 2, 3, 4, 5, 6])])
def test_spectral_steps_equal_single_steps(dtype, shape, ts):
    """Several steps from one read of the spectrum give, bit for bit, the
    grids and checksums of one fb_spectral_step per t (chunks of up to 8
    outputs per fused pass, ragged last chunk, nz = 1 fallback, repeated t);
    and they match the oracle."""
    alpha = 1e-3 if shape[0] < 64 else 1e-6
    plan = fb.Plan(*shape, dtype)
    x0 = as_seen(inputs.uniform_grid(shape, 21), dtype)
    u0 = dev(x0, dtype)
    fb.fb_fft3d_exec(plan, u0, u0, fb.FB_FORWARD)
    nt = len(ts)
    multi = torch.full((nt,) + shape, 3.0, dtype=plan.torch_dtype, device="cuda")
    msums = torch.zeros((nt, 2), dtype=torch.float64, device="cuda")
    fb.fb_spectral_steps(plan, u0, multi, alpha, ts, msums)
    one = torch.empty(shape, dtype=plan.torch_dtype, device="cuda")
    osums = torch.zeros((nt, 2), dtype=torch.float64, device="cuda")
    for j, t in enumerate(ts):
        fb.fb_spectral_step(plan, u0, one, alpha, float(t), osums[j])
        assert torch.equal(one, multi[j]), (j, t)
    assert torch.equal(osums, msums)
    X0 = oracle.fft3d(x0, -1)
    tol = 1e-12 if dtype == fb.FB_C128 else 1e-5
    for j in (0, nt - 1):
        ref = oracle.fft3d(oracle.evolve(X0, alpha, float(ts[j])), +1)
        assert rel_l2(host(multi[j]), ref) < tol, j


def test_spectral_steps_rejects_bad_arguments():
    plan = fb.Plan(8, 8, 8, fb.FB_C128)
    u0 = torch.zeros((8, 8, 8), dtype=torch.complex128, device="cuda")
    out = torch.zeros((2, 8, 8, 8), dtype=torch.complex128, device="cuda")
    for ts in ([], [1.0, -1.0], [float("nan")]):
        with pytest.raises(fb.FbError):
            fb.fb_spectral_steps(plan, u0, out[: max(1, len(ts))] if ts else out[:1], 1e-6, ts)
    # x_out overlapping uhat0
    with pytest.raises(fb.FbError):
        fb.fb_spectral_steps(plan, out[1], out, 1e-6, [1.0, 2.0])


def spectral_block_gpu(x0, dtype, alpha, steps, fused=True):
    shape = x0.shape
    plan = fb.Plan(*shape, dtype)
    u0 = dev(x0, dtype)
    fb.fb_fft3d_exec(plan, u0, u0, fb.FB_FORWARD)
    xt = torch.empty_like(u0)
    sums = torch.zeros((steps, 2), dtype=torch.float64, device="cuda")
    grids = []
    for t in range(1, steps + 1):
        if fused:
            fb.fb_spectral_step(plan, u0, xt, alpha, t, sums[t - 1])
        else:
            xt.copy_(u0)
            fb.fb_spectral_evolve(plan, xt, alpha, t)
            fb.fb_fft3d_exec(plan, xt, xt, fb.FB_INVERSE)
            fb.fb_checksum(plan, xt, sums[t - 1])
        grids.append(host(xt))
    s = sums.cpu().numpy()
    return s[:, 0] + 1j * s[:, 1], grids


def check_block(shape, dtype, seed, alpha, steps, fused=True, gaussian=False):
    x0 = inputs.gaussian_grid(shape, seed) if gaussian else inputs.uniform_grid(shape, seed)
    sums, grids = spectral_block_gpu(x0, dtype, alpha, steps, fused)
    X0 = oracle.fft3d(as_seen(x0, dtype), -1)
    worst = 0.0
    for t in range(1, steps + 1):
        ref = oracle.fft3d(oracle.evolve(X0, alpha, t), +1)
        e = rel_l2(grids[t - 1], ref)
        worst = max(worst, e)
        assert e < TOL[dtype], (t, e)
        assert checksum_err(sums[t - 1], ref) < TOL[dtype], t
    print(f"block shape={shape} dtype={dtype} worst rel L2 {worst:.3e}")


def test_block_64cube_c128_fused():
    check_block((64, 64, 64), fb.FB_C128, seed=1, alpha=1e-6, steps=6)


def test_block_64cube_c128_unfused():
    check_block((64, 64, 64), fb.FB_C128, seed=1, alpha=1e-6, steps=6, fused=False)


def test_block_strong_decay_and_nz1_fallback():
    check_block((32, 64, 1), fb.FB_C128, seed=8, alpha=1e-3, steps=3)
    check_block((24, 12, 48), fb.FB_C128, seed=8, alpha=1e-3, steps=3)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(3, 3, 256), (3, 256, 3), (6, 3, 96)])
def test_block_part_filled_tiles(shape, dtype):
    """The fused step (evolution in the first inverse pass) where the last
    tile of a pass holds fewer pencils than the others."""
    print(f"block shape={shape} dtype={dtype}", flush=True)
    check_block(shape, dtype, seed=4, alpha=1e-4, steps=3)


@pytest.mark.parametrize("dtype", [fb.FB_C64, fb.FB_C64_SPLITBF16])
def test_block_c64(dtype):
    check_block((64, 64, 64), dtype, seed=1, alpha=1e-6, steps=6)
    check_block((128, 64, 96), dtype, seed=2, alpha=1e-6, steps=3, gaussian=True)


@pytest.mark.parametrize("dtype", DTYPES)
def test_block_lengths_with_repeated_threes(dtype):
    """A spectral block whose axes have two or more radix-3 stages
    (36 = 3.3.4, 144 = 3.3.16, 27 = 3.3.3)."""
    check_block((36, 144, 27), dtype, seed=4, alpha=1e-4, steps=3)


def test_precision_forms_512x256x256():
    """The precision-form workload: 512 x 256 x 256, Gaussian N(0,1) input
    (seed 2), 10 evolve steps with alpha = 1e-6; every form against the
    binary64 oracle, every step."""
    shape, alpha, steps = (512, 256, 256), 1e-6, 10
    x0 = inputs.gaussian_grid(shape, 2)
    refs = {}
    for label, xs in (("exact", x0), ("c64", inputs.round_c64(x0).astype(np.complex128))):
        X0 = oracle.fft3d(xs, -1)
        refs[label] = X0
    report = {}
    for dtype in DTYPES:
        plan = fb.Plan(*shape, dtype)
        u0 = dev(x0, dtype)
        fb.fb_fft3d_exec(plan, u0, u0, fb.FB_FORWARD)
        xt = torch.empty_like(u0)
        sums = torch.zeros((steps, 2), dtype=torch.float64, device="cuda")
        X0 = refs["exact" if dtype == fb.FB_C128 else "c64"]
        worst = 0.0
        for t in range(1, steps + 1):
            fb.fb_spectral_step(plan, u0, xt, alpha, t, sums[t - 1])
            got = host(xt)
            ref = oracle.fft3d(oracle.evolve(X0, alpha, t), +1)
            e = rel_l2(got, ref)
            worst = max(worst, e)
            s = sums[t - 1].cpu().numpy()
            assert e < TOL[dtype], (dtype, t, e)
            assert checksum_err(complex(s[0], s[1]), ref) < TOL[dtype], (dtype, t)
        report[fb.DTYPE_NAMES[dtype]] = worst
        del u0, xt, plan
        torch.cuda.empty_cache()
    print("precision forms, worst rel L2 over 10 steps:", report, flush=True)


def test_block_256x256x128_c128_20_steps():
    """The 256 x 256 x 128 complex128 workload with 20 steps, alpha = 1e-6."""
    check_block((256, 256, 128), fb.FB_C128, seed=1, alpha=1e-6, steps=20)


def test_plan_describe_matches_oracle_on_device():
    plan = fb.Plan(256, 256, 128, fb.FB_C128)
    assert fb.fb_plan_describe(plan) == oracle.describe(256, 256, 128)
    assert fb.fb_plan_device_bytes(plan) > 0


def test_wrong_device_tensor_shape_rejected():
    plan = fb.Plan(8, 8, 8, fb.FB_C128)
    t = torch.zeros((8, 8, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(fb.FbError):
        fb.fb_fft3d_exec(plan, t, t)


def test_partial_overlap_rejected():
    plan = fb.Plan(8, 8, 8, fb.FB_C128)
    buf = torch.zeros(1024, dtype=torch.complex128, device="cuda")
    lib = fb.load()
    rc = lib.fb_fft3d_exec(plan.handle, buf.data_ptr(), buf.data_ptr() + 16 * 100, -1, None)
    assert rc == fb.FB_ERR_INVALID_ARG
    rc = lib.fb_fft3d_exec(plan.handle, buf.data_ptr() + 8, buf.data_ptr(), -1, None)
    assert rc == fb.FB_ERR_INVALID_ARG   # misaligned


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
@pytest.mark.parametrize("axes", range(8))
def test_exec_axes(axes, dtype):
    shape = (12, 16, 24)
    x = inputs.uniform_grid(shape, 30 + axes)
    plan = fb.Plan(*shape, dtype)
    for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
        xin = dev(x, dtype)
        out = torch.empty_like(xin)
        fb.fb_fft3d_exec_axes(plan, xin, out, direction, axes)
        ref = oracle.fft3d_axes(as_seen(x, dtype), direction, axes)
        assert rel_l2(host(out), ref) < TOL[dtype], (axes, direction)


def test_profile_hook_records_every_launch():
    shape = (32, 32, 32)
    plan = fb.Plan(*shape, fb.FB_C128)
    x = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    fb.fb_profile_enable(True)
    fb.fb_fft3d_exec(plan, x, x, fb.FB_FORWARD)
    fb.fb_spectral_step(plan, x, torch.empty_like(x), 1e-6, 1.0, torch.zeros(2, dtype=torch.float64, device="cuda"))
    rep = fb.fb_profile_report()
    fb.fb_profile_enable(False)
    names = [r["kernel"] for r in rep]
    assert "fft_pass<c128,n=32,contiguous>" in names
    assert "fft_pass<c128,n=32,contiguous,evolve>" in names
    assert "checksum<c128>" in names
    assert sum(r["launches"] for r in rep) == 3 + 3 + 1
    assert all(r["avg_ms"] > 0 for r in rep)


def test_graph_replays_match_eager():
    """The spectral block captured in a HIP graph: several replays, with eager
    work and synchronisations between them, each equal to the eager result."""
    shape, steps = (64, 32, 48), 4
    plan = fb.Plan(*shape, fb.FB_C128)
    x0 = torch.empty(shape, dtype=torch.complex128, device="cuda")
    fb.fb_fill_uniform(plan, x0, 21)
    u0 = torch.empty_like(x0)
    xt = torch.empty_like(x0)
    sums = torch.zeros((steps, 2), dtype=torch.float64, device="cuda")

    def block():
        fb.fb_fft3d_exec(plan, x0, u0, fb.FB_FORWARD)
        for t in range(1, steps + 1):
            fb.fb_spectral_step(plan, u0, xt, 1e-4, float(t), sums[t - 1])

    block()
    torch.cuda.synchronize()
    want_sums, want_x = sums.clone(), xt.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        block()
    for r in range(3):
        xt.zero_()
        sums.zero_()
        other = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(sums, want_sums), r
        assert torch.equal(xt, want_x), r
        del other


def test_offload_pattern_search():
    """The verification search of the paper's method on a small block: all
    16 placements of (forward, evolve, inverse, checksum) run end to end with
    the host/device copies they need, and every one gives the all-device
    checksums (host blocks in numpy, device blocks through libfb)."""
    from paper_2004_09883_amd import offload
    shape, alpha, steps = (32, 32, 32), 1e-3, 2
    rep = offload.search(torch, fb, shape=shape, alpha=alpha, steps=steps)
    print("offload search:", {k: rep[k] for k in ("greedy_pattern", "best_pattern", "x_vs_all_cpu")}, flush=True)
    assert len(rep["patterns"]) == 16
    assert rep["max_checksum_rel_err"] < 1e-12
    # every pattern's checksums, the all-device one included, against the
    # oracle's block on the same input (error normalised by sum_j |x[17 j]|)
    want_sums, grids = oracle.spectral_block(inputs.uniform_grid(shape, 1), alpha, steps,
                                             keep=set(range(1, steps + 1)))
    for label, sums in [("GGGG", rep["all_gpu_checksums"])] + [(r["pattern"], r["checksums"])
                                                                for r in rep["patterns"]]:
        assert len(sums) == steps, label
        for t in range(1, steps + 1):
            got = complex(*sums[t - 1])
            assert abs(got - want_sums[t - 1]) <= 1e-12 * abs(want_sums[t - 1]) or \
                checksum_err(got, grids[t]) <= 1e-12, (label, t, got, want_sums[t - 1])
    assert rep["best_seconds"] <= rep["all_cpu_seconds"]
    assert set(rep["greedy_pattern"]) <= {"C", "G"} and len(rep["greedy_pattern"]) == 4


@pytest.mark.parametrize("dtype", [fb.FB_C128, fb.FB_C64])
def test_exec_host_equals_device_exec(dtype):
    """The host-buffer form (copies in, transform, copies out) gives the
    device transform's values bit for bit, both directions, in place too."""
    shape = (8, 24, 32)
    plan = fb.Plan(*shape, dtype)
    x = as_seen(inputs.uniform_grid(shape, 31), dtype).astype(np.complex128 if dtype == fb.FB_C128 else np.complex64)
    for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
        d = dev(x, dtype)
        fb.fb_fft3d_exec(plan, d, d, direction)
        want = d.cpu().numpy()
        got = np.empty_like(x)
        fb.fb_fft3d_exec_host(plan, x, got, direction)
        assert np.array_equal(got, want)
        y = x.copy()
        fb.fb_fft3d_exec_host(plan, y, y, direction)
        assert np.array_equal(y, want)
