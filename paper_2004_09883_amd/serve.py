"""Serving driver: replays a seeded Poisson stream of spectral-block requests
against the continuous-batching request loop of libfb (fb_server_*) and
reports throughput and end-to-end latency percentiles.

Latency of a request = completion (checksums on the host, stamped by the
server) - its scheduled arrival in the Poisson stream (start of the replay +
the arrival offset), both on the host's monotonic clock; so a submit loop
that falls behind the schedule shows up in the latency instead of hiding it
(coordinated omission).  The part before the server's own arrival stamp is
reported as submit lateness; the rest splits into queue wait (arrival stamp
-> admission) and service (admission -> completion).  Requests arriving
during the warm-up are served but not counted.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import fb, inputs

HBM_PEAK_GBS = 8000.0


def request_model_bytes(shape, is_c64: bool, steps: int) -> float:
    """Bytes a request moves under the pencil-pass model: every pass reads
    and writes the grid once; the forward transform's first pass generates
    its input (writes only); the steps share their first inverse pass (with
    the evolution fused in) in chunks of up to 8, which read the spectrum
    once and write one grid per step."""
    n = math.prod(shape)
    e = 8 if is_c64 else 16
    chunks = (steps + 7) // 8
    return e * n * (5 + chunks + steps * 5)


def request_flops(shape, steps: int) -> float:
    n = math.prod(shape)
    return (1 + steps) * 5.0 * n * math.log2(n)


def run_serving(rate: float = 2000.0, duration: float = 10.0, warmup: float = 1.0, budget_bytes: float = 200e9,
                n_streams: int = 8, seed_arrivals: int = 5, seed_payload: int = 4, alpha: float = 1e-6,
                poll_every: int = 4, policy: int = fb.FB_SERVE_FIFO, copy_gbs: float | None = None) -> dict:
    """Replays the seeded stream once.  copy_gbs: a measured plain-copy
    bandwidth of the same GPU; the offered load is then also reported
    against it (rho against the practical ceiling as well as against the
    8 TB/s peak)."""
    count = int(math.ceil((warmup + duration) * rate * 1.2)) + 16
    w = inputs.serving_workload(count, rate, seed_arrivals)
    keep = w["arrival"] < warmup + duration
    arrival = w["arrival"][keep]
    n_req = len(arrival)
    server = fb.Server(int(budget_bytes), n_streams, policy)
    results = {}
    meta = {}

    def drain():
        while True:
            r = server.poll()
            if r is None:
                return
            results[r["id"]] = r

    # time.monotonic() and the server's std::chrono::steady_clock are both
    # CLOCK_MONOTONIC on Linux, so scheduled arrivals and server stamps compare
    t0 = time.monotonic()
    for j in range(n_req):
        target = t0 + arrival[j]
        while True:
            now = time.monotonic()
            if now >= target:
                break
            if target - now > 5e-4:
                time.sleep(min(target - now - 4e-4, 2e-3))
        shape = inputs.SERVING_SHAPES[int(w["shape"][j])]
        is_c64 = bool(w["is_c64"][j])
        steps = int(w["steps"][j])
        rid = server.submit(*shape, fb.FB_C64 if is_c64 else fb.FB_C128, steps, alpha, seed_payload, j)
        meta[rid] = (j, shape, is_c64, steps, arrival[j])
        if j % poll_every == 0:
            drain()
    while server.in_flight() > 0:
        drain()
        time.sleep(2e-4)
    drain()
    stats = server.stats()
    server.close()

    measured = [rid for rid, m in meta.items() if m[4] >= warmup]
    bad = [rid for rid in meta if results[rid]["status"] != 0]
    sched = {r: t0 + meta[r][4] for r in measured}
    late = np.array([results[r]["t_arrival"] - sched[r] for r in measured])
    lat = np.array([results[r]["t_done"] - sched[r] for r in measured])
    wait = np.array([results[r]["t_admit"] - results[r]["t_arrival"] for r in measured])
    svc = np.array([results[r]["t_done"] - results[r]["t_admit"] for r in measured])
    t_first = min(sched[r] for r in measured)
    t_last = max(results[r]["t_done"] for r in measured)
    span = t_last - t_first
    model_bytes = sum(request_model_bytes(meta[r][1], meta[r][2], meta[r][3]) for r in measured)
    flops = sum(request_flops(meta[r][1], meta[r][3]) for r in measured)
    offered_bps = model_bytes / duration
    return {
        "rate_req_s": rate,
        "duration_s": duration,
        "warmup_s": warmup,
        "requests": len(measured),
        "failed": len(bad),
        "throughput_req_s": round(len(measured) / span, 1),
        "model_gbs": round(model_bytes / span / 1e9, 1),
        "gflops": round(flops / span / 1e9, 1),
        "offered_load_rho": round(offered_bps / (HBM_PEAK_GBS * 1e9), 3),
        "offered_model_gbs": round(offered_bps / 1e9, 1),
        "offered_load_rho_vs_copy": None if not copy_gbs else round(offered_bps / (copy_gbs * 1e9), 3),
        "copy_gbs": copy_gbs,
        # served slower than requests arrived: the queue grows for the whole
        # run and the latency percentiles grow with its duration
        "saturated": bool(len(measured) / span < 0.97 * rate),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "mean_ms": round(float(lat.mean()) * 1e3, 3),
        "latency_from": "scheduled arrival (start of replay + Poisson offset)",
        "submit_lateness_p50_ms": round(float(np.percentile(late, 50)) * 1e3, 3),
        "submit_lateness_p99_ms": round(float(np.percentile(late, 99)) * 1e3, 3),
        "submit_lateness_max_ms": round(float(late.max()) * 1e3, 3),
        "submit_lateness_min_ms": round(float(late.min()) * 1e3, 3),
        "queue_wait_p50_ms": round(float(np.percentile(wait, 50)) * 1e3, 3),
        "queue_wait_p99_ms": round(float(np.percentile(wait, 99)) * 1e3, 3),
        "service_p50_ms": round(float(np.percentile(svc, 50)) * 1e3, 3),
        "service_p99_ms": round(float(np.percentile(svc, 99)) * 1e3, 3),
        "streams": n_streams,
        "policy": "deadline" if policy == fb.FB_SERVE_DEADLINE else "fifo",
        "budget_bytes": int(budget_bytes),
        "peak_device_bytes": int(stats["peak_allocated"]),
        "max_concurrent": int(stats["max_concurrent"]),
        "plans_cached": int(stats["plans_cached"]),
        "workload": "Poisson arrivals (seed 5), shapes uniform over 32^3/64^3/128^3/256^3/128x256x512, "
                    "70% complex64 / 30% complex128, 1-10 steps, alpha=1e-6, inputs from (seed 4, request)",
    }
