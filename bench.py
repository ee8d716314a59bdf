#!/usr/bin/env python3
"""Benchmark of the 3D FFT spectral block on one MI355X.

One step = one whole spectral block of the 256 x 256 x 128 complex128
workload: the forward 3D FFT of a seeded uniform grid, then for t = 1..20
the fused evolve (alpha = 1e-6) + inverse 3D FFT + checksum, all through the
C ABI (libfb.so).  Inputs are generated on the device before the timed
region and stay resident in HBM.

Prints one JSON line with the throughput (GFLOP/s, 5 N log2 N per transform),
the roofline of the dominant kernel (per-launch HIP events recorded by the
library on the stream the kernels run on), the CPU oracle timed on a bounded
sample of the same workload, and the forms of the 512 x 256 x 256 grid
(complex128 vs complex64 forward FFT).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FFT GFLOP/s (5NlogN) & %HBM roofline; served p50/p99 latency; FP32 vs FP64"
HBM_PEAK_GBS = 8000.0
SHAPE = (256, 256, 128)
ALPHA = 1e-6
T_STEPS = 20
SEED = 1
KERNEL_SOURCES = ["paper_2004_09883_amd/csrc/fb_pass.hpp", "paper_2004_09883_amd/csrc/fb_device.hpp",
                  "paper_2004_09883_amd/csrc/fb_plan_rules.hpp", "paper_2004_09883_amd/csrc/fb_pass_inst.hpp"]


def flops_fft(shape) -> float:
    n = math.prod(shape)
    return 5.0 * n * math.log2(n)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    rec = d.get("kernels", {}).get(kernel)
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def cpu_baseline(budget_steps: int = 10) -> dict:
    """The oracle (plain C, binary64) on the host cores: forward 3D FFT plus
    `budget_steps` of the 20 evolve/inverse/checksum steps of the same
    workload, scaled to GFLOP/s."""
    import numpy as np  # noqa: F401

    import oracle
    from paper_2004_09883_amd import inputs

    x0 = inputs.uniform_grid(SHAPE, SEED)
    t0 = time.perf_counter()
    X0 = oracle.fft3d(x0, -1)
    for t in range(1, budget_steps + 1):
        xt = oracle.fft3d(oracle.evolve(X0, ALPHA, t), +1)
        oracle.checksum(xt)
    dt = time.perf_counter() - t0
    return {"value": round((1 + budget_steps) * flops_fft(SHAPE) / dt / 1e9, 3), "unit": "GFLOP/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"forward FFT + {budget_steps} of the {T_STEPS} evolve/inverse/checksum steps of the "
                      f"{SHAPE[0]}x{SHAPE[1]}x{SHAPE[2]} complex128 block ({dt:.2f} s wall)"}


def forms_section(torch, fb, reps: int = 20) -> dict:
    """512 x 256 x 256 forward 3D FFT per form: time, GFLOP/s, %roofline."""
    shape = (512, 256, 256)
    n = math.prod(shape)
    out = {}
    for name, dt, esize in (("c128", fb.FB_C128, 16), ("c64", fb.FB_C64, 8),
                            ("c64_splitbf16", fb.FB_C64_SPLITBF16, 8)):
        plan = fb.Plan(*shape, dt)
        x = torch.empty(shape, dtype=plan.torch_dtype, device="cuda")
        y = torch.empty_like(x)
        fb.fb_fill_uniform(plan, x, 2)
        for _ in range(3):
            fb.fb_fft3d_exec(plan, x, y, fb.FB_FORWARD)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fb.fb_fft3d_exec(plan, x, y, fb.FB_FORWARD)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        b_alg = 3 * 2 * esize * n
        out[name] = {"forward_ms": round(ms, 4), "gflops": round(flops_fft(shape) / ms / 1e6, 1),
                     "hbm_roofline_frac": round(b_alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                     "model_bytes": b_alg}
        del x, y, plan
        torch.cuda.empty_cache()
    out["c64_speedup_vs_c128"] = round(out["c128"]["forward_ms"] / out["c64"]["forward_ms"], 3)
    out["c64_splitbf16_speedup_vs_c128"] = round(out["c128"]["forward_ms"] / out["c64_splitbf16"]["forward_ms"], 3)
    out["workload"] = "forward 3D FFT of a 512x256x256 grid, 3 pencil passes"
    return out


def copy_reference(torch, nbytes: int = 1 << 29, reps: int = 20) -> dict:
    """A plain device-to-device copy (torch's copy kernel) of a grid-sized
    buffer: the practical bandwidth ceiling a streaming pass is compared with."""
    n = nbytes // 16
    a = torch.empty(n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    a.zero_()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * nbytes, "ms": round(ms, 4), "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain 512 MiB copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the spectral block runs on a single MI355X here; "
              "run it with --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_2004_09883_amd import fb

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    fb.load()
    if args.copy_only:
        print(json.dumps({"copy_reference": copy_reference(torch)}), flush=True)
        return 0

    plan = fb.Plan(*SHAPE, fb.FB_C128)
    x0 = torch.empty(SHAPE, dtype=torch.complex128, device="cuda")
    u0 = torch.empty_like(x0)
    xt = torch.empty_like(x0)
    sums = torch.zeros((T_STEPS, 2), dtype=torch.float64, device="cuda")
    fb.fb_fill_uniform(plan, x0, SEED)

    def step():
        fb.fb_fft3d_exec(plan, x0, u0, fb.FB_FORWARD)
        for t in range(1, T_STEPS + 1):
            fb.fb_spectral_step(plan, u0, xt, ALPHA, float(t), sums[t - 1])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    fb.fb_profile_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    prof = fb.fb_profile_report()
    fb.fb_profile_enable(False)

    ms = start.elapsed_time(stop) / args.steps
    flops_step = (1 + T_STEPS) * flops_fft(SHAPE)
    value = flops_step / (ms * 1e-3) / 1e9
    c = sums.cpu().numpy()
    if not all(map(math.isfinite, c.reshape(-1))):
        print("non-finite checksum", file=sys.stderr)
        return 1

    passes = [k for k in prof if k["kernel"].startswith("fft_pass")]
    dom = max(passes, key=lambda k: k["total_ms"])
    achieved = dom["bytes_per_launch"] / (dom["avg_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom["kernel"]),
                "kernel": dom["kernel"], "avg_launch_ms": round(dom["avg_ms"], 5),
                "bytes_per_launch": dom["bytes_per_launch"]}

    rec = {"metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (SplitMix64 uniform [-1,1), seed 1)",
           "config": {"workload": "spectral block 256x256x128 complex128: forward 3D FFT + 20 x (evolve "
                                  "alpha=1e-6 + inverse 3D FFT + stride-17 checksum)",
                      "shape": list(SHAPE), "steps_per_block": T_STEPS, "alpha": ALPHA,
                      "transforms_per_step": 1 + T_STEPS, "wall_s": round(wall, 3)},
           "roofline": roofline,
           "kernels": [{k: v for k, v in p.items()} for p in prof]}
    if not args.no_forms:
        rec["forms_512x256x256"] = forms_section(torch, fb)
        rec["copy_reference"] = copy_reference(torch)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
