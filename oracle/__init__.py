"""CPU oracle for the FFT spectral block (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
this package.  It wraps ``liboracle.so`` (plain C, binary64, built from
``oracle.c`` with gcc) with numpy-friendly functions.  It shares no code with
the GPU library: the two meet only on the seeded inputs of
``paper_2004_09883_amd.inputs``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, no fused multiply-add)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, dp, i32 = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.orc_threads.restype = i32
    lib.orc_lu.argtypes = [i64, i64, dp, ctypes.POINTER(i32)]
    lib.orc_lu.restype = i32
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_radices.argtypes = [i64, ctypes.POINTER(i32), i32]
    lib.orc_describe.argtypes = [i64, i64, i64, ctypes.c_char_p, i32]
    lib.orc_omega.argtypes = [i64, i64, i32, dp, dp]
    lib.orc_fft3d.argtypes = [i64, i64, i64, i32, dp]
    lib.orc_fft3d_axes.argtypes = [i64, i64, i64, i32, i32, dp]
    lib.orc_fft1d_many.argtypes = [i64, i64, i32, dp]
    lib.orc_dft3d_brute.argtypes = [i64, i64, i64, i32, dp, dp]
    lib.orc_evolve.argtypes = [i64, i64, i64, dp, ctypes.c_double, ctypes.c_double]
    lib.orc_checksum.argtypes = [i64, i64, i64, dp, dp]
    for f in ("orc_radices", "orc_describe", "orc_fft3d", "orc_fft3d_axes", "orc_fft1d_many", "orc_dft3d_brute",
              "orc_evolve", "orc_checksum"):
        getattr(lib, f).restype = i32
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_grid(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    if a.ndim != 3:
        raise ValueError("expected a 3D grid (nx, ny, nz)")
    return a


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Threads used by later calls (timing only; results do not depend on it)."""
    _load().orc_set_threads(int(n))


def radices(n: int) -> list[int]:
    buf = (ctypes.c_int * 64)()
    c = _load().orc_radices(int(n), buf, 64)
    if c < 0:
        raise ValueError(f"length {n} is not of the form 2^a 3^b")
    return list(buf[:c])


def describe(nx: int, ny: int, nz: int) -> str:
    buf = ctypes.create_string_buffer(512)
    if _load().orc_describe(nx, ny, nz, buf, 512) < 0:
        raise ValueError("unsupported shape")
    return buf.value.decode()


def omega(n: int, m: int, sign: int = -1) -> complex:
    re, im = ctypes.c_double(), ctypes.c_double()
    _load().orc_omega(n, m, sign, ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def fft3d(x, sign: int = -1) -> np.ndarray:
    """Forward (sign -1, unscaled) or inverse (sign +1, / N) 3D DFT, z then y then x."""
    a = _as_grid(x).copy()
    nx, ny, nz = a.shape
    rc = _load().orc_fft3d(nx, ny, nz, sign, _dp(a))
    if rc:
        raise ValueError(f"orc_fft3d failed ({rc})")
    return a


def fft3d_axes(x, sign: int, axes: int) -> np.ndarray:
    """Transform along the axes selected by the mask (bit 0 z, bit 1 y, bit 2 x)."""
    a = _as_grid(x).copy()
    nx, ny, nz = a.shape
    rc = _load().orc_fft3d_axes(nx, ny, nz, sign, axes, _dp(a))
    if rc:
        raise ValueError(f"orc_fft3d_axes failed ({rc})")
    return a


def ifft3d(x) -> np.ndarray:
    return fft3d(x, +1)


def fft1d_many(x, sign: int = -1) -> np.ndarray:
    """Transform each row of a 2D array (howmany, n)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).copy()
    if a.ndim == 1:
        a = a[None, :]
    howmany, n = a.shape
    rc = _load().orc_fft1d_many(n, howmany, sign, _dp(a))
    if rc:
        raise ValueError(f"orc_fft1d_many failed ({rc})")
    return a


def fft2d(x, sign: int = -1) -> np.ndarray:
    """2D transform of (ny, nz) arrays, or of a stack (b, ny, nz)."""
    a = np.asarray(x, dtype=np.complex128)
    if a.ndim == 2:
        return fft3d(a[None], sign)[0]
    return np.stack([fft3d(p[None], sign)[0] for p in a])


def dft3d_brute(x, sign: int = -1) -> np.ndarray:
    """Definition tier: direct triple sum in long double (N <= 65536)."""
    a = _as_grid(x)
    out = np.empty_like(a)
    nx, ny, nz = a.shape
    rc = _load().orc_dft3d_brute(nx, ny, nz, sign, _dp(a), _dp(out))
    if rc:
        raise ValueError("grid too large for the brute-force DFT")
    return out


def evolve(u, alpha: float, t: float) -> np.ndarray:
    a = _as_grid(u).copy()
    nx, ny, nz = a.shape
    if _load().orc_evolve(nx, ny, nz, _dp(a), float(alpha), float(t)):
        raise ValueError("invalid evolve arguments")
    return a


def checksum(x) -> complex:
    a = _as_grid(x)
    out = np.zeros(2)
    nx, ny, nz = a.shape
    _load().orc_checksum(nx, ny, nz, _dp(a), _dp(out))
    return complex(out[0], out[1])


def spectral_block(x0, alpha: float, steps: int, keep=None):
    """Run the whole block: X0 = fft3d(x0); for t = 1..steps:
    x_t = ifft3d(evolve(X0, alpha, t)), C_t = checksum(x_t).

    Returns (checksums, grids) where grids maps t -> x_t for every t in
    ``keep`` (default: the last step only)."""
    if keep is None:
        keep = {steps}
    X0 = fft3d(x0, -1)
    sums, grids = [], {}
    for t in range(1, steps + 1):
        xt = fft3d(evolve(X0, alpha, t), +1)
        sums.append(checksum(xt))
        if t in keep:
            grids[t] = xt
    return np.array(sums), grids


def lu(a):
    """LU with partial pivoting of a square matrix (the paper's LU block,
    section 5.1(b)): returns (lu, ipiv, info) with the unit lower factor below
    the diagonal and the upper factor on and above it, row-major; ipiv[j] is
    the row swapped with row j at step j (0-based)."""
    m = np.ascontiguousarray(np.array(a, dtype=np.float64))
    if m.ndim != 2 or m.shape[0] != m.shape[1]:
        raise ValueError("expected a square matrix")
    n = m.shape[0]
    ipiv = np.zeros(max(1, n), dtype=np.int32)
    info = _load().orc_lu(n, n, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if info < 0:
        raise ValueError("bad arguments")
    return m, ipiv[:n], int(info)
