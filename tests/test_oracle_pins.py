"""Pins for the CPU oracle: each check ties it to something other than
itself -- the definition of the DFT written independently (numpy DFT
matrices), closed forms, invariants, a library FFT (pocketfft through
numpy.fft), and hand-computed worked examples under tests/golden/.

The oracle follows the block re-created from the paper's Fourier-transform
function block (section 5.1(a)); the evolution and checksum steps follow the
spectral-block definition (heat-equation decay of each Fourier mode and a
stride-17 sample sum).
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_2004_09883_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dft_matrix(n, sign=-1):
    """Independent definition: F[k, r] = exp(sign 2 pi i (r k mod n) / n)."""
    r = np.arange(n)
    ph = np.outer(r, r) % n
    return np.exp(sign * 2j * np.pi * ph / n)


def dft3d_matrix(x, sign=-1):
    """The 3D DFT as three dense matrix products (separability of the sum)."""
    nx, ny, nz = x.shape
    y = np.einsum("kr,abr->abk", dft_matrix(nz, sign), x)
    y = np.einsum("kr,arb->akb", dft_matrix(ny, sign), y)
    y = np.einsum("kr,rab->kab", dft_matrix(nx, sign), y)
    if sign > 0:
        y = y / x.size
    return y


def mode(shape, k0):
    """exp(2 pi i k0.r / n) with the phase reduced exactly (integer arithmetic)."""
    N = int(np.prod(shape))
    r = np.indices(shape)
    ph = sum((r[a] * (k0[a] % shape[a]) * (N // shape[a])) for a in range(3)) % N
    return np.exp(2j * np.pi * ph / N)


SMALL_AXES = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48]
SMALL_SHAPES = [s for s in itertools.product(SMALL_AXES, repeat=3) if np.prod(s) <= 2048]


# ---------------------------------------------------------------- generator

def test_splitmix64_known_answer():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    want = np.array([int(v) for _, v in rows], dtype=np.uint64)
    got = inputs.splitmix64(1234567, [int(c) for c, _ in rows])
    assert np.array_equal(got, want)


def test_uniform_range_and_moments():
    u = inputs.uniform_pm1(1, np.arange(1 << 20, dtype=np.uint64))
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 3e-3 and abs(u.var() - 1.0 / 3.0) < 3e-3
    # exactness: every value is a multiple of 2^-52
    assert np.all((u + 1.0) * 2.0**52 == np.floor((u + 1.0) * 2.0**52))


def test_uniform_grid_layout():
    g = inputs.uniform_grid((3, 4, 5), 7)
    flat = g.reshape(-1)
    i = 37
    assert flat[i].real == inputs.uniform_pm1(7, [2 * i])[0]
    assert flat[i].imag == inputs.uniform_pm1(7, [2 * i + 1])[0]


def test_gaussian_moments():
    g = inputs.gaussian_grid((64, 64, 64), 2).reshape(-1)
    for part in (g.real, g.imag):
        assert abs(part.mean()) < 5e-3 and abs(part.var() - 1.0) < 1e-2
    assert abs(np.mean(g.real * g.imag)) < 5e-3


def test_batch_lengths_set():
    lens = inputs.batch_lengths(4096, 3)
    allowed = {1 << k for k in range(8, 17)} | {3 << k for k in range(8, 17)}
    assert set(lens.tolist()) == allowed


# ---------------------------------------------------------------- plan

@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256, 512,
                               768, 1024, 2048, 3072, 4096, 9, 18, 27 * 16, 196608])
def test_radix_list(n):
    r = oracle.radices(n)
    assert int(np.prod(r)) == n
    threes = [v for v in r if v == 3]
    rest = r[len(threes):]
    assert all(v == 3 for v in r[: len(threes)])
    assert all(v in (2, 4, 8, 16) for v in rest)
    assert all(v == 16 for v in rest[:-1]) and rest.count(16) >= len(rest) - 1


def test_radix_list_rejects():
    for n in (0, 5, 7, 10, 20, 1000):
        with pytest.raises(ValueError):
            oracle.radices(n)


def test_describe():
    assert oracle.describe(512, 256, 256) == "z:16,16 y:16,16 x:16,16,2 order:zyx"
    assert oracle.describe(64, 64, 64) == "z:16,4 y:16,4 x:16,4 order:zyx"
    assert oracle.describe(1, 3, 768) == "z:3,16,16 y:3 x:- order:zyx"


# ---------------------------------------------------------------- twiddles

def test_omega_quadrants_exact():
    for n in (4, 8, 12, 16, 96, 4096, 3 * 4096):
        assert oracle.omega(n, 0) == 1
        assert oracle.omega(n, n // 4) == -1j
        assert oracle.omega(n, n // 2) == -1
        assert oracle.omega(n, 3 * n // 4) == 1j
        assert oracle.omega(n, n // 4, +1) == 1j


def test_omega_values_correctly_rounded():
    """Twiddles agree with a 40-digit evaluation (mpmath) to within half an ulp."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    for n in (3, 48, 1000, 196608):
        for m in (1, 2, 5, n // 3, n - 1):
            w = oracle.omega(n, m)
            th = -2 * mpmath.pi * mpmath.mpf(m) / n
            for got, ref in ((w.real, mpmath.cos(th)), (w.imag, mpmath.sin(th))):
                err = abs(mpmath.mpf(got) - ref)
                assert err <= 0.5 * np.spacing(abs(float(ref))) + 1e-300


# ---------------------------------------------------------------- FFT vs definition

def test_worked_example_dft4():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "dft4_worked_example.txt"))
            if l.strip() and not l.startswith("#")]
    want = np.array([float(a) + 1j * float(b) for _, a, b in rows])
    x = np.array([1, 2, 3, 4], dtype=np.complex128).reshape(1, 1, 4)
    assert np.array_equal(oracle.fft3d(x).reshape(-1), want)
    assert np.array_equal(oracle.dft3d_brute(x).reshape(-1), want)


@pytest.mark.parametrize("shape", SMALL_SHAPES[::7])
def test_fft_vs_dft_matrix(shape):
    x = inputs.uniform_grid(shape, 11)
    ref = dft3d_matrix(x)
    assert rel_l2(oracle.fft3d(x), ref) < 1e-14
    inv = dft3d_matrix(x, +1)
    assert rel_l2(oracle.fft3d(x, +1), inv) < 1e-14


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 16, 12), (8, 8, 8), (1, 48, 32), (2, 3, 96)])
def test_fft_vs_bruteforce_long_double(shape):
    x = inputs.uniform_grid(shape, 5)
    bf = oracle.dft3d_brute(x)
    assert rel_l2(oracle.fft3d(x), bf) < 1e-14
    assert rel_l2(dft3d_matrix(x), bf) < 1e-14
    assert rel_l2(oracle.fft3d(x, +1), oracle.dft3d_brute(x, +1)) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 8, 16, 48, 64, 96, 128, 256, 512, 768, 1024, 3072, 4096])
def test_fft1d_vs_dft_matrix(n):
    x = inputs.uniform_grid((2, n), 9)
    ref = x @ dft_matrix(n).T
    assert rel_l2(oracle.fft1d_many(x), ref) < 1e-14


@pytest.mark.parametrize("shape", [(64, 64, 64), (32, 64, 48), (256, 256, 128), (1, 512, 512)])
def test_fft_vs_pocketfft(shape):
    x = inputs.uniform_grid(shape, 1)
    assert rel_l2(oracle.fft3d(x), np.fft.fftn(x)) < 1e-13
    assert rel_l2(oracle.fft3d(x, +1), np.fft.ifftn(x)) < 1e-13


@pytest.mark.parametrize("n", [24576, 65536, 196608])
def test_long_1d_vs_pocketfft(n):
    x = inputs.uniform_grid((1, n), 4)
    assert rel_l2(oracle.fft1d_many(x), np.fft.fft(x, axis=-1)) < 1e-13


@pytest.mark.parametrize("axes", range(8))
def test_axes_subset_vs_dft_matrix(axes):
    """A transform along a subset of axes is the DFT along those axes only
    (numpy DFT matrices applied per selected axis)."""
    shape = (6, 8, 12)
    x = inputs.uniform_grid(shape, 17)
    for sign in (-1, +1):
        ref = x.copy()
        nsel = 1
        for bit, ax in ((1, 2), (2, 1), (4, 0)):
            if axes & bit:
                ref = np.moveaxis(np.tensordot(dft_matrix(shape[ax], sign), ref, axes=([1], [ax])), 0, ax)
                nsel *= shape[ax]
        if sign > 0:
            ref = ref / nsel
        got = oracle.fft3d_axes(x, sign, axes)
        assert rel_l2(got, ref) < 1e-14, (axes, sign)


# ---------------------------------------------------------------- closed forms

def test_delta_at_origin_is_all_ones():
    x = np.zeros((8, 12, 16), np.complex128)
    x[0, 0, 0] = 1
    assert np.array_equal(oracle.fft3d(x), np.ones_like(x))


def test_delta_at_r0_gives_phase_ramp():
    shape = (16, 24, 32)
    r0 = (3, 5, 7)
    x = np.zeros(shape, np.complex128)
    x[r0] = 1
    X = oracle.fft3d(x)
    k = np.indices(shape)
    ph = sum(((k[a] * r0[a]) % shape[a]) / shape[a] for a in range(3))
    assert np.max(np.abs(X - np.exp(-2j * np.pi * ph))) < 1e-14


def test_constant_maps_to_dc():
    c = 0.75 - 0.25j
    x = np.full((12, 16, 8), c)
    X = oracle.fft3d(x)
    assert abs(X[0, 0, 0] - c * x.size) < 1e-12
    X[0, 0, 0] = 0
    assert np.max(np.abs(X)) < 1e-12


@pytest.mark.parametrize("k0", [(1, 2, 3), (7, 0, 15), (15, 11, 1)])
def test_single_mode(k0):
    shape = (16, 12, 16)
    x = mode(shape, k0)
    X = oracle.fft3d(x)
    want = np.zeros(shape, np.complex128)
    want[k0] = x.size
    assert np.max(np.abs(X - want)) < 1e-14 * x.size


def test_round_trip_parseval_linearity():
    x = inputs.uniform_grid((32, 24, 16), 3)
    y = inputs.uniform_grid((32, 24, 16), 4)
    X, Y = oracle.fft3d(x), oracle.fft3d(y)
    assert rel_l2(oracle.fft3d(X, +1), x) < 1e-15
    assert abs(np.sum(abs(x) ** 2) - np.sum(abs(X) ** 2) / x.size) < 1e-12 * np.sum(abs(x) ** 2)
    a, b = 0.3 - 1.2j, -2.0 + 0.5j
    assert rel_l2(oracle.fft3d(a * x + b * y), a * X + b * Y) < 1e-15


def test_shift_theorem():
    shape = (16, 8, 12)
    x = inputs.uniform_grid(shape, 6)
    s = (3, 1, 5)
    X = oracle.fft3d(x)
    Xs = oracle.fft3d(np.roll(x, s, axis=(0, 1, 2)))
    k = np.indices(shape)
    ph = np.exp(-2j * np.pi * sum(((k[a] * s[a]) % shape[a]) / shape[a] for a in range(3)))
    assert rel_l2(Xs, X * ph) < 1e-14


def test_real_input_is_hermitian():
    shape = (12, 16, 8)
    x = inputs.uniform_grid(shape, 8).real.astype(np.complex128)
    X = oracle.fft3d(x)
    Xm = np.conj(np.roll(np.flip(X, axis=(0, 1, 2)), 1, axis=(0, 1, 2)))
    assert rel_l2(X, Xm) < 1e-15


# ---------------------------------------------------------------- evolution

FOUR_PI2 = 4.0 * np.pi**2


@pytest.mark.parametrize("k0", [(1, 2, 3), (5, 0, 2), (-3, 4, -7), (8, -8, 0)])
def test_evolve_single_mode_heat_equation(k0):
    """A mode exp(2 pi i k.r/n) on the unit periodic cube decays like the heat
    equation solution exp(-alpha (2 pi |k|)^2 t), with k the signed wavenumber
    (modes above n/2 are the negative ones)."""
    shape = (16, 16, 16)
    alpha, t = 1e-3, 2.5
    x0 = mode(shape, k0)
    xt = oracle.fft3d(oracle.evolve(oracle.fft3d(x0), alpha, t), +1)
    decay = np.exp(-alpha * FOUR_PI2 * sum(v * v for v in k0) * t)
    # error measured against the input's norm: rounding noise in the other
    # modes decays less than the chosen mode, so it is not relative to x_t
    assert np.linalg.norm(xt - decay * x0) < 1e-14 * np.linalg.norm(x0)
    assert abs(np.vdot(x0, xt) / np.vdot(x0, x0) - decay) < 1e-15


def test_evolve_identity_and_semigroup():
    u = inputs.uniform_grid((8, 12, 16), 2)
    assert np.array_equal(oracle.evolve(u, 1e-3, 0.0), u)
    assert np.array_equal(oracle.evolve(u, 0.0, 3.0), u)
    a = oracle.evolve(oracle.evolve(u, 1e-3, 1.0), 1e-3, 2.0)
    b = oracle.evolve(u, 1e-3, 3.0)
    assert rel_l2(a, b) < 1e-15


def test_evolve_conserves_mean_and_decays_energy():
    x0 = inputs.uniform_grid((16, 16, 16), 1)
    X0 = oracle.fft3d(x0)
    prev = np.sum(abs(x0) ** 2)
    for t in range(1, 6):
        xt = oracle.fft3d(oracle.evolve(X0, 1e-3, t), +1)
        assert abs(xt.sum() - x0.sum()) < 1e-12
        e = np.sum(abs(xt) ** 2)
        assert e < prev
        prev = e


def test_evolve_nyquist_uses_wrapped_wavenumber():
    shape = (8, 6, 4)
    u = np.ones(shape, np.complex128)
    e = oracle.evolve(u, 0.01, 1.0)
    c = FOUR_PI2 * 0.01
    # index 4 of 8 is -4, index 3 of 6 is -3, index 2 of 4 is -2; index 5 of 8 is -3
    assert abs(e[4, 3, 2] - np.exp(-c * (16 + 9 + 4))) < 1e-15
    assert abs(e[5, 1, 3] - np.exp(-c * (9 + 1 + 1))) < 1e-15
    assert abs(e[3, 2, 1] - np.exp(-c * (9 + 4 + 1))) < 1e-15


# ---------------------------------------------------------------- checksum

def test_checksum_constant():
    c = 0.5 - 1.5j
    assert oracle.checksum(np.full((32, 32, 32), c)) == 1024 * c


def test_checksum_bruteforce_loop():
    x = inputs.uniform_grid((32, 32, 32), 12)
    flat = x.reshape(-1)
    s = 0j
    for j in range(1024):
        s += flat[17 * j]
    assert oracle.checksum(x) == s


def test_checksum_wraps_on_tiny_grid():
    x = inputs.uniform_grid((4, 4, 4), 13)
    flat = x.reshape(-1)
    want = sum(flat[(17 * j) % 64] for j in range(1024))
    assert abs(oracle.checksum(x) - want) < 1e-12


# ---------------------------------------------------------------- the whole block

def test_block_single_mode_closed_form():
    shape = (32, 32, 32)
    k0 = (3, -5, 9)
    alpha = 1e-4
    x0 = mode(shape, k0)
    sums, grids = oracle.spectral_block(x0, alpha, 4, keep={2, 4})
    flat = x0.reshape(-1)
    base = sum(flat[17 * j] for j in range(1024))
    for t in (1, 2, 3, 4):
        d = np.exp(-alpha * FOUR_PI2 * sum(v * v for v in k0) * t)
        assert abs(sums[t - 1] - d * base) < 1e-11
    for t in (2, 4):
        d = np.exp(-alpha * FOUR_PI2 * sum(v * v for v in k0) * t)
        assert rel_l2(grids[t], d * x0) < 1e-14
