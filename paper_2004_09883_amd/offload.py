"""Offload-pattern verification for the spectral block (the paper's
verification step, section 3.4 and section 4: every candidate block is
measured on the CPU and on the accelerator one at a time, the faster
placement of each block is kept, the combination is measured as a whole and
the fastest pattern is reported).

The block is: forward 3D FFT, then for t = 1..steps: evolution, inverse 3D
FFT, checksum.  Its four function blocks each have two placements:

* "gpu": the libfb call on the device (fb_fft3d_exec, fb_spectral_evolve,
  fb_checksum), data in device memory;
* "cpu": the same operation written with numpy on the host (numpy.fft for
  the transforms).  These host versions exist only to be measured against the
  library, as the paper's original CPU code is; nothing in libfb or its
  binding calls them.

A pattern assigns a placement to each of the four blocks; data move between
host and device (pinned buffers, timed) wherever consecutive blocks are
placed on different sides.  The input starts on the host and the checksums
end there.
"""
from __future__ import annotations

import itertools
import math
import time

import numpy as np

BLOCKS = ("forward", "evolve", "inverse", "checksum")
FOUR_PI2 = 4.0 * math.pi * math.pi


def all_patterns():
    """Every placement of the four blocks, all-CPU first."""
    return [dict(zip(BLOCKS, p)) for p in itertools.product(("cpu", "gpu"), repeat=len(BLOCKS))]


def transfers(pattern) -> int:
    """Host/device crossings of the grid in one block with `steps` = 1 (the
    input starts on the host, checksums end on the host): forward -> evolve ->
    inverse -> checksum."""
    side = "cpu"
    n = 0
    for b in BLOCKS:
        if pattern[b] != side:
            n += 1
            side = pattern[b]
    return n


def greedy_pattern(block_times):
    """The per-block winners: block_times[b] = {"cpu": s, "gpu": s}."""
    return {b: min(("cpu", "gpu"), key=lambda p: block_times[b][p]) for b in BLOCKS}


# ---------------------------------------------------------------- host blocks

def _kgrid(shape):
    ks = [np.fft.fftfreq(n, 1.0 / n) for n in shape]   # signed integer wavenumbers
    k2 = ks[0][:, None, None] ** 2 + ks[1][None, :, None] ** 2 + ks[2][None, None, :] ** 2
    return k2


def cpu_forward(x):
    return np.fft.fftn(x)


def cpu_evolve(u0, alpha, t, k2):
    return u0 * np.exp(-(FOUR_PI2 * alpha * t) * k2)


def cpu_inverse(u):
    return np.fft.ifftn(u)


def cpu_checksum(x):
    flat = x.reshape(-1)
    return complex(np.sum(flat[(17 * np.arange(1024)) % flat.size]))


# ---------------------------------------------------------------- one pattern

class _Runner:
    """Runs the block under one pattern with host and device buffers."""

    def __init__(self, torch, fb, shape, alpha, steps, x_host):
        self.torch, self.fb = torch, fb
        self.shape, self.alpha, self.steps = shape, alpha, steps
        self.plan = fb.Plan(*shape, fb.FB_C128)
        self.x_host = x_host
        self.k2 = _kgrid(shape)
        self.pin = torch.empty(shape, dtype=torch.complex128).pin_memory()
        self.dev = [torch.empty(shape, dtype=torch.complex128, device="cuda") for _ in range(3)]
        self.sums = torch.zeros(2, dtype=torch.float64, device="cuda")

    def to_dev(self, a, d):
        self.torch.cuda.synchronize()   # the staging buffer is free again
        self.pin.copy_(self.torch.from_numpy(a))
        d.copy_(self.pin, non_blocking=True)

    def to_host(self, d):
        self.pin.copy_(d, non_blocking=True)
        self.torch.cuda.synchronize()
        return self.pin.numpy().copy()

    def run(self, pattern):
        """Returns (seconds, checksums) of the whole block under `pattern`."""
        torch, fb = self.torch, self.fb
        u0d, ud, xd = self.dev
        out = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # forward
        if pattern["forward"] == "gpu":
            self.to_dev(self.x_host, xd)
            fb.fb_fft3d_exec(self.plan, xd, u0d, fb.FB_FORWARD)
            u0h = None
        else:
            u0h = cpu_forward(self.x_host)
        for t in range(1, self.steps + 1):
            # evolve
            if pattern["evolve"] == "gpu":
                if u0h is not None:
                    self.to_dev(u0h, u0d)
                    u0h = None
                ud.copy_(u0d)
                fb.fb_spectral_evolve(self.plan, ud, self.alpha, float(t))
                uh = None
            else:
                if u0h is None:
                    u0h = self.to_host(u0d)
                uh = cpu_evolve(u0h, self.alpha, t, self.k2)
            # inverse
            if pattern["inverse"] == "gpu":
                if uh is not None:
                    self.to_dev(uh, ud)
                fb.fb_fft3d_exec(self.plan, ud, xd, fb.FB_INVERSE)
                xh = None
            else:
                if uh is None:
                    uh = self.to_host(ud)
                xh = cpu_inverse(uh)
            # checksum
            if pattern["checksum"] == "gpu":
                if xh is not None:
                    self.to_dev(xh, xd)
                fb.fb_checksum(self.plan, xd, self.sums)
                s = self.sums.cpu().numpy()
                out.append(complex(s[0], s[1]))
            else:
                if xh is None:
                    xh = self.to_host(xd)
                out.append(cpu_checksum(xh))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out


def time_blocks(runner, reps: int = 3):
    """Each block alone on each side (data already on that side), best of
    `reps`: the per-candidate measurement of the paper's verification step."""
    torch, fb = runner.torch, runner.fb
    u0h = cpu_forward(runner.x_host)
    uh = cpu_evolve(u0h, runner.alpha, 1.0, runner.k2)
    xh = cpu_inverse(uh)
    u0d, ud, xd = runner.dev
    runner.to_dev(runner.x_host, xd)
    fb.fb_fft3d_exec(runner.plan, xd, u0d, fb.FB_FORWARD)
    torch.cuda.synchronize()

    def best(fn, gpu):
        ts = []
        for _ in range(reps):
            if gpu:
                torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            if gpu:
                torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return min(ts)

    def gpu_evolve():
        ud.copy_(u0d)
        fb.fb_spectral_evolve(runner.plan, ud, runner.alpha, 1.0)

    return {
        "forward": {"cpu": best(lambda: cpu_forward(runner.x_host), False),
                    "gpu": best(lambda: fb.fb_fft3d_exec(runner.plan, xd, u0d, fb.FB_FORWARD), True)},
        "evolve": {"cpu": best(lambda: cpu_evolve(u0h, runner.alpha, 1.0, runner.k2), False),
                   "gpu": best(gpu_evolve, True)},
        "inverse": {"cpu": best(lambda: cpu_inverse(uh), False),
                    "gpu": best(lambda: fb.fb_fft3d_exec(runner.plan, ud, xd, fb.FB_INVERSE), True)},
        "checksum": {"cpu": best(lambda: cpu_checksum(xh), False),
                     "gpu": best(lambda: fb.fb_checksum(runner.plan, xd, runner.sums), True)},
    }


def search(torch, fb, shape=(64, 64, 64), alpha: float = 1e-6, steps: int = 6, seed: int = 1,
           exhaustive: bool = True) -> dict:
    """The verification search on one block: per-block timings, the greedy
    combination, and (exhaustive) every pattern measured end to end; every
    pattern's checksums must agree with the all-GPU pattern's."""
    from . import inputs

    x = inputs.uniform_grid(shape, seed)
    runner = _Runner(torch, fb, shape, alpha, steps, x)
    per_block = time_blocks(runner)
    chosen = greedy_pattern(per_block)
    patterns = all_patterns() if exhaustive else [chosen, {b: "cpu" for b in BLOCKS}]
    ref = None
    results = []
    for p in [{b: "gpu" for b in BLOCKS}] + patterns:
        runner.run(p)                       # warm-up (plans, caches, clocks)
        secs, sums = runner.run(p)
        if ref is None:
            ref = sums
            continue
        norm = max(1e-300, max(abs(v) for v in ref))
        err = max(abs(a - b) for a, b in zip(sums, ref)) / norm
        results.append({"pattern": "".join("G" if p[b] == "gpu" else "C" for b in BLOCKS), "seconds": secs,
                        "transfers_per_step": transfers(p), "checksum_rel_err_vs_all_gpu": err,
                        "checksums": [[v.real, v.imag] for v in sums]})
    best = min(results, key=lambda r: r["seconds"])
    cpu_only = next(r for r in results if r["pattern"] == "CCCC")
    greedy_name = "".join("G" if chosen[b] == "gpu" else "C" for b in BLOCKS)
    greedy = next(r for r in results if r["pattern"] == greedy_name)
    return {
        "workload": "%dx%dx%d complex128, forward + %d x (evolve alpha=%g + inverse + checksum)"
                    % (shape + (steps, alpha)),
        "blocks": list(BLOCKS),
        "pattern_code": "one letter per block in the order above: G device (libfb), C host (numpy)",
        "block_seconds": {b: {k: round(v, 6) for k, v in d.items()} for b, d in per_block.items()},
        "greedy_pattern": greedy_name,
        "greedy_seconds": round(greedy["seconds"], 6),
        "best_pattern": best["pattern"],
        "best_seconds": round(best["seconds"], 6),
        "all_cpu_seconds": round(cpu_only["seconds"], 6),
        "x_vs_all_cpu": round(cpu_only["seconds"] / best["seconds"], 1),
        "patterns": [{k: (round(v, 6) if isinstance(v, float) and k != "checksum_rel_err_vs_all_gpu" else v)
                      for k, v in r.items()} for r in results],
        "max_checksum_rel_err": max(r["checksum_rel_err_vs_all_gpu"] for r in results),
        "all_gpu_checksums": [[v.real, v.imag] for v in ref],
    }
