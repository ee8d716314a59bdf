"""Library-call substitution (the paper's steps A-1, B-1, C-1, C-2) on C
sources, on the CPU: detection, the interface check, the rewrite, and the
sample application it is demonstrated on (its checksums pinned to the
oracle)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2004_09883_amd import inputs, substitute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
APPS = os.path.join(ROOT, "tests", "apps")
TABLE = substitute.load_patterns()


def read(name):
    with open(os.path.join(APPS, name)) as f:
        return f.read()


def test_table_has_the_cpu_fft_record():
    rec = TABLE["cfft3d"]
    assert rec["library"] == "cpufft" and rec["replacement"]["library"] == "libfb"
    assert len(rec["params"]) == 5
    assert any("fb_fft3d_exec_host" in ln for ln in rec["replacement"]["usage"])


def test_detects_both_calls_of_the_sample_application():
    src = read("heat3d.c")
    calls = substitute.detect(src, TABLE)
    lines = [i + 1 for i, ln in enumerate(src.splitlines()) if "cfft3d(" in ln and "usage" not in ln]
    assert [c["line"] for c in calls] == lines and len(calls) == 2
    assert all(c["interface_ok"] and c["name"] == "cfft3d" for c in calls)
    assert [c["args"][-1] for c in calls] == ["-1", "+1"]


def test_comments_literals_declarations_and_definitions_are_not_calls():
    src = ('#include "cpufft.h"\n'
           "/* cfft3d(1, 2, 3, p, -1) in a comment */\n"
           "// cfft3d(1, 2, 3, p, -1)\n"
           "int cfft3d(int64_t nx, int64_t ny, int64_t nz, double *data, int sign);\n"
           'const char *s = "cfft3d(1, 2, 3, p, -1)";\n'
           "char c = '(';\n"
           "int f(double *p) { return cfft3d(4, 4, 4, p, -1); }\n")
    calls = substitute.detect(src, TABLE)
    assert len(calls) == 1 and calls[0]["line"] == 7
    defined = "int cfft3d(int64_t a, int64_t b, int64_t c, double *d, int s) { return 0; }\nint g(double *p) { return cfft3d(1, 1, 1, p, 1); }\n"
    assert substitute.detect(defined, TABLE) == []   # the file defines it: not an external call


def test_interface_mismatch_is_reported_not_rewritten(tmp_path):
    src = '#include "cpufft.h"\nint f(double *p) { return cfft3d(4, 4, p, -1) + cfft3d(4, 4, 4, p, (1 > 0) ? 1 : -1); }\n'
    out, calls = substitute.rewrite(src, TABLE)
    assert [c["interface_ok"] for c in calls] == [False, True]
    assert "cfft3d(4, 4, p, -1)" in out and "fbsub_cfft3d(4, 4, 4, p, (1 > 0) ? 1 : -1)" in out
    assert "ask the user" in calls[0]["action"]
    a = tmp_path / "a.c"
    a.write_text(src)
    assert substitute.main([str(a), "-o", str(tmp_path / "b.c")]) == 3


def test_rewritten_application_compiles_against_the_header(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    out, calls = substitute.rewrite(read("heat3d.c"), TABLE)
    assert out.count("fbsub_cfft3d(nx, ny, nz") == 2 and '#include "fb.h"' in out
    p = tmp_path / "heat3d_fb.c"
    p.write_text(out)
    r = subprocess.run(["gcc", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-Wall", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), "-I", APPS, str(p)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert substitute.link_flags(calls) == ["-lfb"]


def test_sample_application_matches_the_oracle(tmp_path):
    """The CPU program the substitution starts from computes the spectral
    block: its checksums equal the oracle's on a 16^3 grid."""
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = tmp_path / "heat3d"
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", os.path.join(APPS, "heat3d.c"),
                    os.path.join(APPS, "cpufft.c"), "-lm", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe), "16", "16", "16", "3", "1e-3"], capture_output=True, text=True, check=True)
    got = [complex(float(a), float(b)) for _, a, b in (ln.split() for ln in r.stdout.strip().splitlines())]
    ref, _ = oracle.spectral_block(inputs.uniform_grid((16, 16, 16), 1), 1e-3, 3)
    assert np.max(np.abs(np.array(got) - ref)) < 1e-12 * 1024
