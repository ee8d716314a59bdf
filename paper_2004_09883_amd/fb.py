"""Python binding of libfb (ctypes; argument marshalling only).

Each function carries the name of the C entry point it calls (include/fb.h).
Grid arguments are torch tensors on the plan's device (complex128 for
FB_C128, complex64 otherwise, C-contiguous, shape (nx, ny, nz)) or raw
device addresses (int).  Work is enqueued on ``stream`` (a torch.cuda.Stream,
a raw hipStream_t int, or None for torch's current stream).  Every step of
the computation runs in libfb's HIP kernels; if the library is not built the
binding raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfb.so")

FB_C128, FB_C64, FB_C64_SPLITBF16 = 0, 1, 2
FB_FORWARD, FB_INVERSE = -1, +1
FB_OK = 0
FB_ERR_INVALID_ARG = -1
FB_ERR_UNSUPPORTED_SIZE = -2
FB_ERR_DTYPE = -3
FB_ERR_OOM = -4
FB_ERR_DEVICE = -5
FB_ERR_BUDGET = -6

DTYPE_NAMES = {FB_C128: "c128", FB_C64: "c64", FB_C64_SPLITBF16: "c64_splitbf16"}

# every entry point declared in include/fb.h
EXPORTS = ("fb_version", "fb_last_error", "fb_describe_shape", "fb_fft3d_plan", "fb_fft3d_destroy",
           "fb_plan_device_bytes", "fb_plan_describe", "fb_fft3d_exec", "fb_spectral_evolve",
           "fb_checksum", "fb_spectral_step", "fb_spectral_steps", "fb_fft3d_exec_host", "fb_fft3d_exec_host_noalloc", "fb_lu_factor", "fb_fill_uniform", "fb_fft3d_forward_uniform", "fb_fft3d_exec_axes",
           "fb_profile_enable", "fb_profile_report", "fb_batch_plan", "fb_batch_destroy", "fb_batch_elements",
           "fb_batch_offsets", "fb_batch_workspace_bytes", "fb_batch_launches", "fb_batch_describe",
           "fb_batch_exec", "fb_server_create", "fb_server_submit", "fb_server_poll",
           "fb_server_in_flight", "fb_server_stats", "fb_server_set_policy", "fb_server_destroy")


FB_SERVE_MAX_STEPS = 64
FB_SERVE_FIFO = 0
FB_SERVE_DEADLINE = 1


class FbRequest(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("dtype", ctypes.c_int),
                ("steps", ctypes.c_int), ("alpha", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("request_key", ctypes.c_int64), ("want_grid", ctypes.c_int)]


class FbResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("dtype", ctypes.c_int), ("steps", ctypes.c_int),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("grid_bytes", ctypes.c_int64)]


class FbServerInfo(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_size_t), ("bytes_allocated", ctypes.c_size_t),
                ("peak_allocated", ctypes.c_size_t), ("plans_cached", ctypes.c_int),
                ("max_concurrent", ctypes.c_int), ("queued", ctypes.c_int64)]


class FbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fb error {code}: {msg}")
        self.code = code
        self.msg = msg


_lib = None


def load():
    """Load libfb.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FbError(FB_ERR_DEVICE, f"{LIB_PATH} is not built (run __graft_entry__.build() or "
                                     "python -m paper_2004_09883_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, i32, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "fb_version": (i32, []),
        "fb_last_error": (i32, [ctypes.POINTER(ctypes.c_char_p)]),
        "fb_describe_shape": (i32, [i64, i64, i64, i32, ctypes.c_char_p, i32]),
        "fb_fft3d_plan": (vp, [i64, i64, i64, i32]),
        "fb_fft3d_destroy": (None, [vp]),
        "fb_plan_device_bytes": (ctypes.c_size_t, [vp]),
        "fb_plan_describe": (ctypes.c_char_p, [vp]),
        "fb_fft3d_exec": (i32, [vp, vp, vp, i32, vp]),
        "fb_spectral_evolve": (i32, [vp, vp, dbl, dbl, vp]),
        "fb_checksum": (i32, [vp, vp, vp, vp]),
        "fb_spectral_step": (i32, [vp, vp, vp, dbl, dbl, vp, vp]),
        "fb_fill_uniform": (i32, [vp, vp, ctypes.c_uint64, vp]),
        "fb_fft3d_exec_host": (i32, [vp, vp, vp, i32]),
        "fb_fft3d_exec_host_noalloc": (i32, [vp, vp, vp, i32]),
        "fb_lu_factor": (i32, [vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp]),
        "fb_spectral_steps": (i32, [vp, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double), i32, vp, vp]),
        "fb_fft3d_forward_uniform": (i32, [vp, ctypes.c_uint64, vp, vp]),
        "fb_fft3d_exec_axes": (i32, [vp, vp, vp, i32, i32, vp]),
        "fb_profile_enable": (i32, [i32]),
        "fb_profile_report": (i32, [ctypes.c_char_p, i32]),
        "fb_batch_plan": (vp, [ctypes.POINTER(i64), i32, i32, i64, i32]),
        "fb_batch_destroy": (None, [vp]),
        "fb_batch_elements": (i64, [vp]),
        "fb_batch_offsets": (i32, [vp, ctypes.POINTER(i64)]),
        "fb_batch_workspace_bytes": (ctypes.c_size_t, [vp, i32]),
        "fb_batch_launches": (i32, [vp]),
        "fb_batch_describe": (ctypes.c_char_p, [vp]),
        "fb_batch_exec": (i32, [vp, vp, vp, vp, ctypes.c_size_t, i32, i32, vp]),
        "fb_server_create": (vp, [ctypes.c_size_t, i32]),
        "fb_server_submit": (i64, [vp, ctypes.POINTER(FbRequest)]),
        "fb_server_poll": (i32, [vp, ctypes.POINTER(FbResult), ctypes.POINTER(dbl), i32, vp, ctypes.c_size_t]),
        "fb_server_in_flight": (i64, [vp]),
        "fb_server_stats": (i32, [vp, ctypes.POINTER(FbServerInfo)]),
        "fb_server_set_policy": (i32, [vp, i32]),
        "fb_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def fb_last_error():
    msg = ctypes.c_char_p()
    code = load().fb_last_error(ctypes.byref(msg))
    return code, (msg.value or b"").decode()


def _check(rc: int):
    if rc < 0:
        code, msg = fb_last_error()
        raise FbError(rc, msg)
    return rc


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _check_sums(t, need: int, name: str, allow_none: bool):
    """A checksum destination: a contiguous float64 device tensor of at least
    `need` values (or a raw device address, or None where the call allows
    it).  Checked here because the C side can only see the pointer."""
    if t is None:
        if allow_none:
            return
        raise FbError(FB_ERR_INVALID_ARG, f"{name} is required")
    if isinstance(t, int):
        if t == 0 and not allow_none:
            raise FbError(FB_ERR_INVALID_ARG, f"{name} is NULL")
        return
    import torch
    if not isinstance(t, torch.Tensor):
        raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a float64 device tensor")
    if t.dtype != torch.float64:
        raise FbError(FB_ERR_DTYPE, f"{name} is {t.dtype}, needs torch.float64")
    if t.numel() < need:
        raise FbError(FB_ERR_INVALID_ARG, f"{name} holds {t.numel()} values, needs at least {need}")
    if not t.is_contiguous():
        raise FbError(FB_ERR_INVALID_ARG, f"{name} must be contiguous")
    if not t.is_cuda:
        raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a device tensor")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def fb_version() -> int:
    return load().fb_version()


def fb_describe_shape(nx: int, ny: int, nz: int, dtype: int = FB_C128) -> str:
    buf = ctypes.create_string_buffer(256)
    _check(load().fb_describe_shape(nx, ny, nz, dtype, buf, 256))
    return buf.value.decode()


class Plan:
    """Owns an fb_plan*; destroyed with the object or by close()."""

    def __init__(self, nx: int, ny: int, nz: int, dtype: int = FB_C128):
        self._lib = load()
        h = self._lib.fb_fft3d_plan(nx, ny, nz, dtype)
        if not h:
            code, msg = fb_last_error()
            raise FbError(code, msg)
        self.handle = h
        self.shape = (nx, ny, nz)
        self.dtype = dtype

    def close(self):
        if getattr(self, "handle", None):
            self._lib.fb_fft3d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128 if self.dtype == FB_C128 else torch.complex64

    def check_tensor(self, x, name="x"):
        """Shape/dtype/contiguity check of a torch tensor argument."""
        if isinstance(x, int):
            return
        if tuple(x.shape) != self.shape:
            raise FbError(FB_ERR_INVALID_ARG, f"{name} has shape {tuple(x.shape)}, plan is {self.shape}")
        if x.dtype != self.torch_dtype:
            raise FbError(FB_ERR_DTYPE, f"{name} is {x.dtype}, plan needs {self.torch_dtype}")
        if not x.is_contiguous():
            raise FbError(FB_ERR_INVALID_ARG, f"{name} must be C-contiguous")
        if not x.is_cuda:
            raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a device tensor")


def fb_fft3d_plan(nx: int, ny: int, nz: int, dtype: int = FB_C128) -> Plan:
    return Plan(nx, ny, nz, dtype)


def fb_fft3d_destroy(plan: Plan):
    plan.close()


def fb_plan_device_bytes(plan: Plan) -> int:
    return int(load().fb_plan_device_bytes(plan.handle))


def fb_plan_describe(plan: Plan) -> str:
    return load().fb_plan_describe(plan.handle).decode()


def fb_fft3d_exec(plan: Plan, x_in, x_out, direction: int = FB_FORWARD, stream=None):
    plan.check_tensor(x_in, "in")
    plan.check_tensor(x_out, "out")
    _check(load().fb_fft3d_exec(plan.handle, _ptr(x_in), _ptr(x_out), direction, _stream(stream)))


def fb_fft3d_exec_axes(plan: Plan, x_in, x_out, direction: int, axes: int, stream=None):
    """Transform along the axes selected by the mask (bit 0 z, bit 1 y, bit 2 x)."""
    plan.check_tensor(x_in, "in")
    plan.check_tensor(x_out, "out")
    _check(load().fb_fft3d_exec_axes(plan.handle, _ptr(x_in), _ptr(x_out), direction, axes, _stream(stream)))


def fb_profile_enable(on: bool = True):
    _check(load().fb_profile_enable(1 if on else 0))


def fb_profile_report() -> list:
    """Per-kernel timing recorded since fb_profile_enable(True)."""
    import json
    cap = 1 << 16
    buf = ctypes.create_string_buffer(cap)
    _check(load().fb_profile_report(buf, cap))
    return json.loads(buf.value.decode())


def fb_spectral_evolve(plan: Plan, u, alpha: float, t: float, stream=None):
    plan.check_tensor(u, "u")
    _check(load().fb_spectral_evolve(plan.handle, _ptr(u), float(alpha), float(t), _stream(stream)))


def fb_checksum(plan: Plan, x, out2, stream=None):
    """out2: a float64 device tensor with at least 2 elements (or an address)."""
    plan.check_tensor(x, "x")
    _check_sums(out2, 2, "out2", allow_none=False)
    _check(load().fb_checksum(plan.handle, _ptr(x), _ptr(out2), _stream(stream)))


def fb_spectral_step(plan: Plan, uhat0, x_out, alpha: float, t: float, out2=None, stream=None):
    plan.check_tensor(uhat0, "uhat0")
    plan.check_tensor(x_out, "x_out")
    _check_sums(out2, 2, "out2", allow_none=True)
    _check(load().fb_spectral_step(plan.handle, _ptr(uhat0), _ptr(x_out), float(alpha), float(t),
                                   _ptr(out2), _stream(stream)))


def fb_lu_factor(a, ipiv, info, stream=None):
    """a: square float64 device tensor (row-major, factored in place); ipiv:
    int32 device tensor of n elements; info: int32 device tensor of at least
    one element."""
    import torch
    if not isinstance(a, int):
        if a.dim() != 2 or a.shape[0] != a.shape[1] or a.dtype != torch.float64 or not a.is_cuda:
            raise FbError(FB_ERR_INVALID_ARG, "a must be a square float64 device tensor")
        if a.stride(1) != 1:
            raise FbError(FB_ERR_INVALID_ARG, "a must have unit column stride (row-major)")
        n, lda = a.shape[0], a.stride(0)
    else:
        raise FbError(FB_ERR_INVALID_ARG, "pass a tensor")
    for t, name, need in ((ipiv, "ipiv", n), (info, "info", 1)):
        if t.dtype != torch.int32 or not t.is_cuda or t.numel() < need or not t.is_contiguous():
            raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a contiguous int32 device tensor of >= {need} elements")
    _check(load().fb_lu_factor(_ptr(a), n, lda, _ptr(ipiv), _ptr(info), _stream(stream)))


def fb_fft3d_exec_host(plan: Plan, x_in, x_out, direction: int = FB_FORWARD):
    """Host numpy arrays of the plan's shape and dtype (complex128 or
    complex64), C-contiguous; synchronous."""
    import numpy as np
    want = np.complex128 if plan.dtype == FB_C128 else np.complex64
    for a, name in ((x_in, "x_in"), (x_out, "x_out")):
        if a.shape != plan.shape or a.dtype != want or not a.flags["C_CONTIGUOUS"]:
            raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a C-contiguous {want.__name__} array of shape {plan.shape}")
    _check(load().fb_fft3d_exec_host(plan.handle, x_in.ctypes.data, x_out.ctypes.data, direction))


FB_STATIC_SCRATCH_BYTES = 64 << 20


def fb_fft3d_exec_host_noalloc(plan: Plan, x_in, x_out, direction: int = FB_FORWARD):
    """As fb_fft3d_exec_host, staged through the library's static device
    buffer (no device allocation; grids up to FB_STATIC_SCRATCH_BYTES)."""
    import numpy as np
    want = np.complex128 if plan.dtype == FB_C128 else np.complex64
    for a, name in ((x_in, "x_in"), (x_out, "x_out")):
        if a.shape != plan.shape or a.dtype != want or not a.flags["C_CONTIGUOUS"]:
            raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a C-contiguous {want.__name__} array of shape {plan.shape}")
    _check(load().fb_fft3d_exec_host_noalloc(plan.handle, x_in.ctypes.data, x_out.ctypes.data, direction))


def fb_spectral_steps(plan: Plan, uhat0, x_out, alpha: float, ts, sums=None, stream=None):
    """x_out: a device tensor of len(ts) grids (shape (len(ts), nx, ny, nz) or
    any contiguous tensor of that many elements); sums: float64 device tensor
    of at least 2 len(ts) elements or None."""
    plan.check_tensor(uhat0, "uhat0")
    ts = [float(v) for v in ts]
    n = plan.shape[0] * plan.shape[1] * plan.shape[2]
    if not isinstance(x_out, int) and (x_out.numel() != len(ts) * n or not x_out.is_contiguous()
                                       or x_out.dtype != plan.torch_dtype or not x_out.is_cuda):
        raise FbError(FB_ERR_INVALID_ARG, f"x_out must be a contiguous {plan.torch_dtype} device tensor of "
                                          f"{len(ts)} grids")
    _check_sums(sums, 2 * len(ts), "sums", allow_none=True)
    arr = (ctypes.c_double * max(1, len(ts)))(*ts)
    _check(load().fb_spectral_steps(plan.handle, _ptr(uhat0), _ptr(x_out), float(alpha), arr, len(ts), _ptr(sums),
                                    _stream(stream)))


def fb_fft3d_forward_uniform(plan: Plan, seed: int, out, stream=None):
    """Forward 3D FFT of the seeded uniform grid, generated inside the first pass."""
    plan.check_tensor(out, "out")
    _check(load().fb_fft3d_forward_uniform(plan.handle, int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out), _stream(stream)))


def fb_fill_uniform(plan: Plan, x, seed: int, stream=None):
    plan.check_tensor(x, "x")
    _check(load().fb_fill_uniform(plan.handle, _ptr(x), int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream)))


class Batch:
    """Owns an fb_batch*: n1d 1D transforms of the given lengths plus n2d 2D
    side x side transforms, packed back to back (complex64)."""

    def __init__(self, lens, n2d: int = 0, side2d: int = 0, dtype: int = FB_C64):
        self._lib = load()
        lens = [int(v) for v in lens]
        arr = (ctypes.c_int64 * max(1, len(lens)))(*lens)
        h = self._lib.fb_batch_plan(arr, len(lens), int(n2d), int(side2d), dtype)
        if not h:
            code, msg = fb_last_error()
            raise FbError(code, msg)
        self.handle = h
        self.lens = lens
        self.n2d = int(n2d)
        self.side2d = int(side2d)
        self.elements = int(self._lib.fb_batch_elements(h))
        off = (ctypes.c_int64 * (len(lens) + self.n2d))()
        _check(self._lib.fb_batch_offsets(h, off))
        self.offsets = list(off)
        self.launches = int(self._lib.fb_batch_launches(h))
        self.description = self._lib.fb_batch_describe(h).decode()

    def workspace_bytes(self, in_place: bool = False) -> int:
        return int(self._lib.fb_batch_workspace_bytes(self.handle, 1 if in_place else 0))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.fb_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fb_batch_plan(lens, n2d: int = 0, side2d: int = 0, dtype: int = FB_C64) -> Batch:
    return Batch(lens, n2d, side2d, dtype)


def fb_batch_exec(batch: Batch, x_in, x_out, workspace, direction: int = FB_FORWARD, persistent=True,
                  stream=None):
    """x_in/x_out: complex64 device tensors of batch.elements values; workspace:
    a device tensor (uint8) of at least batch.workspace_bytes(x_in is x_out).
    persistent: False/0 one launch per group, True/1 the whole batch in one
    launch, 2 one persistent launch per phase."""
    for t, name in ((x_in, "in"), (x_out, "out")):
        if not isinstance(t, int) and (t.numel() != batch.elements or not t.is_contiguous()):
            raise FbError(FB_ERR_INVALID_ARG, f"{name} must be a contiguous tensor of {batch.elements} elements")
    wbytes = workspace.numel() * workspace.element_size() if not isinstance(workspace, int) else 1 << 62
    _check(load().fb_batch_exec(batch.handle, _ptr(x_in), _ptr(x_out), _ptr(workspace), wbytes, direction,
                                int(persistent), _stream(stream)))




class Server:
    """Owns an fb_server*: the continuous-batching request loop."""

    def __init__(self, budget_bytes: int, n_streams: int = 8, policy: int = FB_SERVE_FIFO):
        self._lib = load()
        h = self._lib.fb_server_create(int(budget_bytes), int(n_streams))
        if not h:
            raise FbError(FB_ERR_INVALID_ARG, "fb_server_create failed (budget >= 1 MiB, 1..64 streams, a device)")
        self.handle = h
        if policy != FB_SERVE_FIFO:
            self.set_policy(policy)

    def set_policy(self, policy: int):
        """FB_SERVE_FIFO or FB_SERVE_DEADLINE (see include/fb.h)."""
        _check(self._lib.fb_server_set_policy(self.handle, int(policy)))

    def submit(self, nx, ny, nz, dtype, steps, alpha, seed, request_key, want_grid=False) -> int:
        r = FbRequest(nx, ny, nz, dtype, steps, alpha, seed & 0xFFFFFFFFFFFFFFFF, request_key, 1 if want_grid else 0)
        rid = self._lib.fb_server_submit(self.handle, ctypes.byref(r))
        if rid < 0:
            raise FbError(int(rid), "fb_server_submit rejected the request")
        return int(rid)

    def poll(self, grid_capacity: int = 0):
        """One finished request as a dict, or None."""
        res = FbResult()
        sums = (ctypes.c_double * (2 * FB_SERVE_MAX_STEPS))()
        grid = None
        if grid_capacity:
            if getattr(self, "_grid", None) is None or len(self._grid) < grid_capacity:
                self._grid = ctypes.create_string_buffer(grid_capacity)
            grid = self._grid
            grid_capacity = len(grid)
        got = self._lib.fb_server_poll(self.handle, ctypes.byref(res), sums, 2 * FB_SERVE_MAX_STEPS, grid,
                                       grid_capacity)
        if got <= 0:
            return None
        out = {k: getattr(res, k) for k, _ in FbResult._fields_}
        out["checksums"] = [complex(sums[2 * i], sums[2 * i + 1]) for i in range(res.steps)]
        out["grid"] = grid.raw[:res.grid_bytes] if (grid is not None and res.grid_bytes) else None
        return out

    def in_flight(self) -> int:
        return int(self._lib.fb_server_in_flight(self.handle))

    def stats(self) -> dict:
        info = FbServerInfo()
        _check(self._lib.fb_server_stats(self.handle, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in FbServerInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.fb_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fb_server_create(budget_bytes: int, n_streams: int = 8) -> Server:
    return Server(budget_bytes, n_streams)
