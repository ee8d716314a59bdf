"""GPU parity of the batched form: many independent complex64 1D transforms
of mixed lengths plus 2D transforms, as one launch per (length, pass) group
(mode 0), as a single persistent launch for the whole batch (mode 1) or as
one persistent launch per phase (mode 2), against the oracle transform by
transform (rel L2 <= 1e-5 each, on the complex64-rounded inputs); the three
modes run the same tile code and must agree bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2004_09883_amd import fb, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def packed_input(batch, seed):
    x = inputs.uniform_grid((batch.elements,), seed)
    return inputs.round_c64(x)


def ref_transform(batch, x, i, sign):
    o = batch.offsets[i]
    if i < len(batch.lens):
        seg = x[o:o + batch.lens[i]].astype(np.complex128)
        return oracle.fft1d_many(seg[None, :], sign)[0]
    s = batch.side2d
    seg = x[o:o + s * s].astype(np.complex128).reshape(s, s)
    return oracle.fft2d(seg, sign).reshape(-1)


def run(batch, x, direction, persistent, in_place):
    xin = torch.from_numpy(x).cuda()
    out = xin if in_place else torch.empty_like(xin)
    ws = torch.zeros(batch.workspace_bytes(in_place) + 256, dtype=torch.uint8, device="cuda")
    wsp = ws.data_ptr()
    wsp = (wsp + 255) // 256 * 256
    fb.fb_batch_exec(batch, xin, out, wsp, direction, persistent)
    torch.cuda.synchronize()
    return out.cpu().numpy()


MIXED = [256, 768, 4096, 3072, 6144, 8192, 24576, 65536, 196608, 12, 2, 3, 48, 512, 98304, 256, 12288, 16384,
         32768, 49152, 1536, 2048]


MODES = (0, 1, 2)


@pytest.mark.parametrize("persistent", MODES)
@pytest.mark.parametrize("in_place", [False, True])
@pytest.mark.parametrize("direction", [fb.FB_FORWARD, fb.FB_INVERSE])
def test_mixed_batch(persistent, in_place, direction):
    print(f"batch persistent={persistent} in_place={in_place} dir={direction}", flush=True)
    batch = fb.Batch(MIXED, n2d=3, side2d=64)
    x = packed_input(batch, 3)
    got = run(batch, x, direction, persistent, in_place)
    for i in range(len(MIXED) + 3):
        o = batch.offsets[i]
        n = MIXED[i] if i < len(MIXED) else 64 * 64
        e = rel_l2(got[o:o + n].astype(np.complex128), ref_transform(batch, x, i, direction))
        assert e < TOL, (i, n, e)


def test_persistent_equals_per_group_bitwise():
    batch = fb.Batch(MIXED, n2d=2, side2d=512)
    assert "onelaunch=1" in batch.description, batch.description
    x = packed_input(batch, 5)
    for in_place in (False, True):
        for direction in (fb.FB_FORWARD, fb.FB_INVERSE):
            a = run(batch, x, direction, 0, in_place)
            b = run(batch, x, direction, 1, in_place)
            assert np.array_equal(a, b), (in_place, direction)
            c = run(batch, x, direction, 2, in_place)
            assert np.array_equal(a, c), (in_place, direction)
    d = run(batch, x, fb.FB_FORWARD, 1, False)   # a second single launch on the same plan
    assert np.array_equal(d, run(batch, x, fb.FB_FORWARD, 0, False))


def test_batch_workload_4096_plus_64x512x512():
    """4096 1D lengths drawn from {2^k, 3*2^k : 8 <= k <= 16} (seed 3) plus
    64 2D 512 x 512 transforms; uniform inputs.  Checks a sample of
    transforms of every length (the smallest and the largest index of each)
    and two 2D transforms, in both execution modes."""
    lens = inputs.batch_lengths(4096, 3).tolist()
    batch = fb.Batch(lens, n2d=64, side2d=512)
    print("batch plan:", batch.description, flush=True)
    assert "onelaunch=1" in batch.description   # the workload runs in one launch
    x = packed_input(batch, 3)
    first = {}
    last = {}
    for i, n in enumerate(lens):
        first.setdefault(n, i)
        last[n] = i
    sample = sorted(set(first.values()) | set(last.values())) + [4096, 4096 + 63]
    outs = []
    for persistent in MODES:
        got = run(batch, x, fb.FB_FORWARD, persistent, False)
        outs.append(got)
        worst = 0.0
        for i in sample:
            o = batch.offsets[i]
            n = lens[i] if i < 4096 else 512 * 512
            e = rel_l2(got[o:o + n].astype(np.complex128), ref_transform(batch, x, i, fb.FB_FORWARD))
            worst = max(worst, e)
            assert e < TOL, (persistent, i, n, e)
        print(f"batch workload persistent={persistent}: {len(sample)} transforms checked, worst rel L2 {worst:.2e}",
              flush=True)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("lens,n2d,side", [([], 2, 64), ([196608], 0, 0), ([2], 0, 0), ([3] * 5, 0, 0),
                                           ([24576, 24576], 1, 512), ([4096] * 3 + [8], 0, 0)])
def test_batch_edge_shapes(lens, n2d, side):
    """Only 2D transforms, a single transform of the largest length, a single
    length-2 transform, several tiny transforms, one long length plus one 2D
    transform: both modes against the oracle, and equal to each other."""
    print(f"batch edge lens={lens[:4]} n2d={n2d} side={side}", flush=True)
    batch = fb.Batch(lens, n2d=n2d, side2d=side)
    x = packed_input(batch, 11)
    outs = []
    for persistent in MODES:
        got = run(batch, x, fb.FB_FORWARD, persistent, False)
        for i in range(len(lens) + n2d):
            o = batch.offsets[i]
            n = lens[i] if i < len(lens) else side * side
            e = rel_l2(got[o:o + n].astype(np.complex128), ref_transform(batch, x, i, fb.FB_FORWARD))
            assert e < TOL, (persistent, i, n, e)
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
