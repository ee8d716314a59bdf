"""GPU checks of the serving form: each request's result is the same alone
and in a mix of concurrent requests (bitwise: the kernels and their order do
not depend on the mix), results match the oracle, and admission never lets
device memory exceed the HBM budget."""
import math

import numpy as np
import pytest

import oracle
from paper_2004_09883_amd import fb, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ALPHA = 1e-6
SEED = 4

# (shape, dtype, steps, request key)
REQS = [((32, 32, 32), fb.FB_C64, 3, 0), ((64, 64, 64), fb.FB_C128, 5, 1), ((32, 32, 32), fb.FB_C128, 10, 2),
        ((128, 128, 128), fb.FB_C64, 2, 3), ((64, 64, 64), fb.FB_C64, 7, 4), ((128, 256, 512), fb.FB_C64, 1, 5),
        ((128, 128, 128), fb.FB_C128, 4, 6), ((32, 32, 32), fb.FB_C64, 1, 7), ((64, 64, 64), fb.FB_C128, 9, 8),
        ((256, 256, 256), fb.FB_C64, 2, 9), ((64, 64, 64), fb.FB_C64, 6, 10), ((32, 32, 32), fb.FB_C128, 4, 11)]


def nbytes(shape, dtype):
    return int(np.prod(shape)) * (16 if dtype == fb.FB_C128 else 8)


def wait_for(server, n, cap):
    out = {}
    while len(out) < n:
        r = server.poll(cap)
        if r is not None:
            out[r["id"]] = r
    return out


def as_grid(r, shape, dtype):
    return np.frombuffer(r["grid"], dtype=np.complex128 if dtype == fb.FB_C128 else np.complex64).reshape(shape)


def test_alone_equals_mix_and_oracle():
    cap = max(nbytes(s, d) for s, d, _, _ in REQS)
    alone = {}
    server = fb.Server(64 << 30, 8)
    for i, (shape, dt, steps, key) in enumerate(REQS):
        rid = server.submit(*shape, dt, steps, ALPHA, SEED, key, want_grid=True)
        alone[i] = wait_for(server, 1, cap)[rid]
        assert alone[i]["status"] == 0
    server.close()

    server = fb.Server(64 << 30, 8)
    ids = {}
    bg = 0
    for i, (shape, dt, steps, key) in enumerate(REQS):
        ids[server.submit(*shape, dt, steps, ALPHA, SEED, key, want_grid=True)] = i
        for _ in range(2):   # background requests between the checked ones
            server.submit(128, 128, 128, fb.FB_C64 if bg % 2 else fb.FB_C128, 3, ALPHA, SEED, 1000 + bg)
            bg += 1
    got = wait_for(server, len(REQS) + bg, cap)
    info = server.stats()
    server.close()
    assert info["max_concurrent"] > 1, "the mix did not overlap requests"
    for rid, i in ids.items():
        a, m = alone[i], got[rid]
        assert m["status"] == 0
        assert a["checksums"] == m["checksums"], i
        assert a["grid"] == m["grid"], i

    # against the oracle
    for i in (0, 1, 3, 6, 9):
        shape, dt, steps, key = REQS[i]
        x0 = inputs.request_grid(shape, SEED, key)
        if dt == fb.FB_C64:
            x0 = inputs.round_c64(x0).astype(np.complex128)
        sums, grids = oracle.spectral_block(x0, ALPHA, steps)
        tol = 1e-12 if dt == fb.FB_C128 else 1e-5
        ref = grids[steps]
        g = as_grid(alone[i], shape, dt).astype(np.complex128)
        assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < tol, i
        flat = ref.reshape(-1)
        norm = np.sum(np.abs(flat[(17 * np.arange(1024)) % flat.size]))
        for t in range(steps):
            assert abs(alone[i]["checksums"][t] - sums[t]) / norm < tol, (i, t)


def test_budget_admission():
    # a request holds its spectrum and min(steps, 8) output grids
    one = 9 * nbytes((128, 128, 128), fb.FB_C128) + 4096
    server = fb.Server(one, 4)
    for k in range(5):
        server.submit(128, 128, 128, fb.FB_C128, 10, ALPHA, SEED, 50 + k)
    res = wait_for(server, 5, 0)
    assert all(r["status"] == 0 for r in res.values())
    info = server.stats()
    assert info["peak_allocated"] <= one
    assert info["max_concurrent"] == 1
    with pytest.raises(fb.FbError) as e:
        server.submit(256, 256, 256, fb.FB_C128, 1, ALPHA, SEED, 99)
    assert e.value.code == fb.FB_ERR_BUDGET
    server.close()


@pytest.mark.parametrize("policy", [fb.FB_SERVE_FIFO, fb.FB_SERVE_DEADLINE])
def test_admission_policy_order(policy):
    """One stream slot, so admissions are strictly one after the other: a
    long request runs while a second long one and then a short one queue.
    FIFO admits them in arrival order; the deadline policy lets the short one
    (arrival + estimated service earlier) overtake.  Results do not depend on
    the order."""
    server = fb.Server(16 << 30, 1, policy)
    big = ((256, 256, 256), fb.FB_C64, 4)
    a = server.submit(*big[0], big[1], big[2], ALPHA, SEED, 200)
    while server.stats()["queued"] > 0:   # a is admitted (and runs for milliseconds)
        pass
    b = server.submit(*big[0], big[1], big[2], ALPHA, SEED, 201)
    c = server.submit(32, 32, 32, fb.FB_C128, 1, ALPHA, SEED, 202)
    res = wait_for(server, 3, 0)
    server.close()
    assert all(r["status"] == 0 for r in res.values())
    assert res[a]["t_admit"] <= min(res[b]["t_admit"], res[c]["t_admit"])
    if policy == fb.FB_SERVE_FIFO:
        assert res[b]["t_admit"] < res[c]["t_admit"]
    else:
        assert res[c]["t_admit"] < res[b]["t_admit"]
    # the same requests alone give the same checksums
    solo = fb.Server(16 << 30, 1)
    ids = {solo.submit(*big[0], big[1], big[2], ALPHA, SEED, 201): b, solo.submit(32, 32, 32, fb.FB_C128, 1, ALPHA, SEED, 202): c}
    ref = wait_for(solo, 2, 0)
    solo.close()
    for rid, orig in ids.items():
        assert ref[rid]["checksums"] == res[orig]["checksums"]
    with pytest.raises(fb.FbError):
        fb.Server(1 << 30, 1).set_policy(7)


def test_submit_validation():
    server = fb.Server(1 << 30, 2)
    for bad in (dict(nx=5, ny=4, nz=4, dtype=fb.FB_C64, steps=1), dict(nx=4, ny=4, nz=4, dtype=7, steps=1),
                dict(nx=4, ny=4, nz=4, dtype=fb.FB_C64, steps=0),
                dict(nx=4, ny=4, nz=4, dtype=fb.FB_C64, steps=fb.FB_SERVE_MAX_STEPS + 1)):
        with pytest.raises(fb.FbError):
            server.submit(bad["nx"], bad["ny"], bad["nz"], bad["dtype"], bad["steps"], ALPHA, SEED, 0)
    server.close()


def test_short_serving_run():
    from paper_2004_09883_amd import serve
    rep = serve.run_serving(rate=400.0, duration=1.0, warmup=0.2, budget_bytes=64e9)
    print("serving:", rep, flush=True)
    assert rep["failed"] == 0 and rep["requests"] > 200
    assert 0 < rep["p50_ms"] <= rep["p99_ms"]


def test_serving_workload_sample_against_oracle():
    """The first 160 requests of the serving workload (Poisson stream of
    seed 5: shapes, dtypes, step counts; inputs from seed 4 and the request
    index), submitted at once so that the loop runs them concurrently; every
    32^3 and 64^3 request and one in forty of the others is checked against
    the oracle (checksums of the first and the last step)."""
    count = 160
    w = inputs.serving_workload(count, 2000.0, 5)
    server = fb.Server(int(200e9), 8)
    ids = {}
    for j in range(count):
        shape = inputs.SERVING_SHAPES[int(w["shape"][j])]
        dt = fb.FB_C64 if bool(w["is_c64"][j]) else fb.FB_C128
        steps = int(w["steps"][j])
        ids[server.submit(*shape, dt, steps, ALPHA, SEED, j)] = (j, shape, dt, steps)
    got = wait_for(server, count, 0)
    info = server.stats()
    server.close()
    assert info["max_concurrent"] > 1
    others = checked = 0
    for rid, (j, shape, dt, steps) in sorted(ids.items()):
        r = got[rid]
        assert r["status"] == 0, j
        if math.prod(shape) > 64 ** 3:
            others += 1
            if others % 40 != 1:
                continue
        x0 = inputs.request_grid(shape, SEED, j)
        if dt == fb.FB_C64:
            x0 = inputs.round_c64(x0).astype(np.complex128)
        X0 = oracle.fft3d(x0, -1)
        tol = 1e-12 if dt == fb.FB_C128 else 1e-5
        for t in sorted({1, steps}):
            ref = oracle.fft3d(oracle.evolve(X0, ALPHA, t), +1)
            flat = ref.reshape(-1)
            norm = np.sum(np.abs(flat[(17 * np.arange(1024)) % flat.size]))
            assert abs(r["checksums"][t - 1] - oracle.checksum(ref)) / norm < tol, (j, t)
        checked += 1
    print(f"serving workload sample: {checked} of {count} requests checked against the oracle", flush=True)
    assert checked >= 10
