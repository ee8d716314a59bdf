"""Builds and runs a C host program before and after library-call
substitution (the paper's flow: detect, replace, compile, measure in the
verification environment) and compares what the two print."""
from __future__ import annotations

import os
import subprocess
import tempfile

from . import substitute

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)


def build_pair(source: str, cpu_library_sources, include_dirs, workdir: str):
    """Compiles the original program (with the CPU library's sources) and the
    rewritten one (linked with libfb); returns (original exe, rewritten exe,
    substitution report)."""
    with open(source) as f:
        src = f.read()
    out, calls = substitute.rewrite(src, substitute.load_patterns())
    rewritten = os.path.join(workdir, "rewritten.c")
    with open(rewritten, "w") as f:
        f.write(out)
    incs = [a for d in include_dirs for a in ("-I", d)]
    common = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L"]
    orig_exe = os.path.join(workdir, "original")
    subprocess.run(common + incs + [source] + list(cpu_library_sources) + ["-lm", "-o", orig_exe], check=True)
    new_exe = os.path.join(workdir, "rewritten")
    subprocess.run(common + incs + ["-I", os.path.join(ROOT, "include"), rewritten, "-L", PKG]
                   + substitute.link_flags(calls) + ["-Wl,-rpath," + PKG, "-lm", "-o", new_exe], check=True)
    return orig_exe, new_exe, calls


def run(exe: str, args):
    """(per-step checksums, elapsed seconds the program reports, wall seconds)."""
    import time
    t0 = time.perf_counter()
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, check=True)
    wall = time.perf_counter() - t0
    sums = [complex(float(a), float(b)) for _, a, b in (ln.split() for ln in r.stdout.strip().splitlines())]
    elapsed = float(r.stderr.split("elapsed_s")[1].split()[0])
    return sums, elapsed, wall


def heat3d_experiment(shape=(128, 128, 128), steps: int = 6, alpha: float = 1e-6) -> dict:
    """The sample heat-equation application, original (CPU library) and
    rewritten (libfb), on the same grid: agreement and speed."""
    apps = os.path.join(ROOT, "tests", "apps")
    with tempfile.TemporaryDirectory() as d:
        orig, new, calls = build_pair(os.path.join(apps, "heat3d.c"), [os.path.join(apps, "cpufft.c")], [apps], d)
        args = list(shape) + [steps, alpha]
        s0, e0, w0 = run(orig, args)
        s1, e1, w1 = run(new, args)
    err = max(abs(a - b) for a, b in zip(s0, s1))
    return {"workload": "heat3d.c (tests/apps), %dx%dx%d complex128, %d steps, alpha=%g: forward + per step evolve, "
                        "inverse, checksum; every transform a call of the CPU library cpufft" % (shape + (steps, alpha)),
            "calls_replaced": sum(1 for c in calls if c["action"].startswith("replaced")),
            "cpu_library_s": round(e0, 4), "libfb_s": round(e1, 4),
            "x_vs_cpu_library": round(e0 / e1, 1),
            "wall_s": {"original": round(w0, 3), "rewritten": round(w1, 3)},
            "note": "program-reported time from the first transform to the last checksum; the rewritten program's "
                    "includes device initialisation, plan creation and the host-device copies of every call",
            "max_abs_checksum_diff": err}
