"""Seeded synthetic inputs for the FFT spectral block.

This module holds random-number generation only: it contains none of the
block's arithmetic (no transform, no evolution, no checksum).  Both the CPU
oracle's tests and the GPU path draw their inputs from here, so the two
sides consume bit-identical grids.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-based: the value at counter
``c`` of stream ``seed`` is ``mix64(seed + (c + 1) * GAMMA)``, i.e. the
(c+1)-th output of the sequential generator started at state ``seed``.

Uniform deviates: ``U(seed, c) = (h >> 11) * 2**-52 - 1`` with
``h = splitmix64(seed, c)``; this lies in [-1, 1) and is exact in binary64.
Element ``i`` of a complex grid takes ``U(seed, 2i)`` as its real part and
``U(seed, 2i + 1)`` as its imaginary part (C order, z fastest).

Gaussian deviates: Box-Muller on the pair of counters ``(2i, 2i + 1)``, with
``u1 = ((h0 >> 11) + 1) * 2**-53`` in (0, 1] and ``u2 = (h1 >> 11) * 2**-53``
in [0, 1); real part ``r cos(2 pi u2)``, imaginary part ``r sin(2 pi u2)``,
``r = sqrt(-2 ln u1)``, evaluated in binary64 on the host.

Per-request streams (serving): request ``rid`` of base seed ``s`` uses the
stream seed ``splitmix64(s, rid)``; the GPU kernel that generates request
inputs on the device implements the same definition independently.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, counters) -> np.ndarray:
    """SplitMix64 output at the given counters of stream ``seed`` (uint64)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GAMMA
        return _mix64(z)


def stream_seed(seed: int, rid: int) -> int:
    """Seed of the per-request stream ``rid`` derived from base ``seed``."""
    return int(splitmix64(seed, [rid])[0])


def uniform_pm1(seed: int, counters) -> np.ndarray:
    """U(seed, c) in [-1, 1), exact in binary64."""
    h = splitmix64(seed, counters)
    return (h >> np.uint64(11)).astype(np.float64) * 2.0**-52 - 1.0


def _chunks(n: int, chunk: int = 1 << 22):
    for lo in range(0, n, chunk):
        yield lo, min(n, lo + chunk)


def uniform_grid(shape, seed: int) -> np.ndarray:
    """Complex128 grid of the given shape, re/im i.i.d. U[-1, 1) from ``seed``."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.complex128)
    v = out.view(np.float64)
    for lo, hi in _chunks(2 * n):
        v[lo:hi] = uniform_pm1(seed, np.arange(lo, hi, dtype=np.uint64))
    return out.reshape(shape)


def gaussian_grid(shape, seed: int) -> np.ndarray:
    """Complex128 grid of the given shape, re/im i.i.d. N(0, 1) (Box-Muller)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.complex128)
    for lo, hi in _chunks(n):
        i = np.arange(lo, hi, dtype=np.uint64)
        h0 = splitmix64(seed, 2 * i)
        h1 = splitmix64(seed, 2 * i + np.uint64(1))
        u1 = ((h0 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53
        u2 = (h1 >> np.uint64(11)).astype(np.float64) * 2.0**-53
        r = np.sqrt(-2.0 * np.log(u1))
        th = 2.0 * np.pi * u2
        out[lo:hi].real = r * np.cos(th)
        out[lo:hi].imag = r * np.sin(th)
    return out.reshape(shape)


def request_grid(shape, seed: int, rid: int) -> np.ndarray:
    """Uniform grid of serving request ``rid`` (stream ``splitmix64(seed, rid)``)."""
    return uniform_grid(shape, stream_seed(seed, rid))


def batch_lengths(count: int, seed: int) -> np.ndarray:
    """``count`` 1D lengths drawn uniformly from {2^k, 3*2^k : 8 <= k <= 16}.

    Draw j uses ``splitmix64(seed, j) % 18`` as the index into the sorted set
    (the modulo bias is below 2^-59 and is ignored).
    """
    choices = np.array(sorted([1 << k for k in range(8, 17)]
                              + [3 << k for k in range(8, 17)]), dtype=np.int64)
    idx = splitmix64(seed, np.arange(count, dtype=np.uint64)) % np.uint64(len(choices))
    return choices[idx.astype(np.int64)]


def round_c64(x: np.ndarray) -> np.ndarray:
    """Round a complex128 grid to complex64 (round to nearest even, per part)."""
    return x.astype(np.complex64)


SERVING_SHAPES = ((32, 32, 32), (64, 64, 64), (128, 128, 128), (256, 256, 256), (128, 256, 512))


def unit_interval(seed: int, counters) -> np.ndarray:
    """(h >> 11) * 2**-53 in [0, 1) from SplitMix64."""
    h = splitmix64(seed, counters)
    return (h >> np.uint64(11)).astype(np.float64) * 2.0**-53


def serving_workload(count: int, rate: float, seed: int = 5):
    """Poisson request stream: for request j the counters 4j .. 4j+3 of stream
    ``seed`` give the exponential gap -ln(1 - u) / rate, the shape (uniform
    over SERVING_SHAPES), the dtype (complex64 with probability 0.7, else
    complex128) and the number of evolve steps (uniform in 1..10).

    Returns a dict of arrays: arrival (seconds from the start), shape index,
    is_c64, steps."""
    j = np.arange(count, dtype=np.uint64)
    u = [unit_interval(seed, 4 * j + np.uint64(k)) for k in range(4)]
    gaps = -np.log1p(-u[0]) / rate
    return {
        "arrival": np.cumsum(gaps),
        "shape": np.minimum((u[1] * len(SERVING_SHAPES)).astype(np.int64), len(SERVING_SHAPES) - 1),
        "is_c64": u[2] < 0.7,
        "steps": 1 + np.minimum((u[3] * 10).astype(np.int64), 9),
    }
