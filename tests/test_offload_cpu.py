"""Host logic of the offload-pattern verification search (no GPU): the
pattern space, the transfer accounting and the per-block choice."""
from paper_2004_09883_amd import offload


def test_sixteen_distinct_patterns():
    ps = offload.all_patterns()
    assert len(ps) == 16
    assert len({tuple(p[b] for b in offload.BLOCKS) for p in ps}) == 16
    assert all(set(p) == set(offload.BLOCKS) for p in ps)


def test_transfer_count():
    mk = lambda code: {b: ("gpu" if c == "G" else "cpu") for b, c in zip(offload.BLOCKS, code)}
    assert offload.transfers(mk("CCCC")) == 0
    assert offload.transfers(mk("GGGG")) == 1      # input to the device once
    assert offload.transfers(mk("GCGC")) == 4
    assert offload.transfers(mk("CCGG")) == 1
    assert offload.transfers(mk("GGGC")) == 2


def test_greedy_takes_each_faster_side():
    t = {"forward": {"cpu": 2.0, "gpu": 1.0}, "evolve": {"cpu": 0.5, "gpu": 0.7},
         "inverse": {"cpu": 3.0, "gpu": 0.1}, "checksum": {"cpu": 0.01, "gpu": 0.02}}
    assert offload.greedy_pattern(t) == {"forward": "gpu", "evolve": "cpu", "inverse": "gpu", "checksum": "cpu"}


def test_host_blocks_match_definitions():
    import numpy as np
    shape = (4, 6, 8)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    u = offload.cpu_forward(x)
    back = offload.cpu_inverse(u)
    assert np.allclose(back, x, rtol=1e-12, atol=1e-14)
    assert np.linalg.norm(back - x) <= 1e-14 * np.linalg.norm(x)
    k2 = offload._kgrid(shape)
    # k = 0 untouched; the Nyquist wavenumber of the first axis (2) squared is 4
    assert k2[0, 0, 0] == 0 and k2[2, 0, 0] == 4 and k2[3, 0, 0] == 1
    e = offload.cpu_evolve(u, 1e-3, 2.0, k2)
    assert np.allclose(e[1, 2, 3], u[1, 2, 3] * np.exp(-4 * np.pi ** 2 * 1e-3 * 2.0 * (1 + 4 + 9)),
                       rtol=1e-12, atol=0)
    flat = x.reshape(-1)
    ref = complex(sum(flat[(17 * j) % flat.size] for j in range(1024)))
    assert abs(offload.cpu_checksum(x) - ref) <= 1e-13 * sum(abs(flat[(17 * j) % flat.size]) for j in range(1024))


def test_host_blocks_match_the_oracle():
    """The host placements of the verification search (numpy) against the
    oracle on the same seeded grid: forward and inverse transforms and the
    evolution at relative L2 <= 1e-13, the checksum to rounding (the search
    then compares every placement's checksums with the oracle on the
    device)."""
    import numpy as np
    import oracle
    from paper_2004_09883_amd import inputs
    shape, alpha, t = (8, 12, 16), 1e-3, 3.0
    x = inputs.uniform_grid(shape, 5)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    u = offload.cpu_forward(x)
    assert rel(u, oracle.fft3d(x, -1)) <= 1e-13
    e = offload.cpu_evolve(u, alpha, t, offload._kgrid(shape))
    assert rel(e, oracle.evolve(oracle.fft3d(x, -1), alpha, t)) <= 1e-13
    xt = offload.cpu_inverse(e)
    assert rel(xt, oracle.fft3d(oracle.evolve(oracle.fft3d(x, -1), alpha, t), +1)) <= 1e-13
    ref = oracle.checksum(xt)
    flat = xt.reshape(-1)
    norm = np.sum(np.abs(flat[(17 * np.arange(1024)) % flat.size]))
    assert abs(offload.cpu_checksum(xt) - ref) <= 1e-14 * norm
