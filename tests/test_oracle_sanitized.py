"""The oracle's C code runs clean under AddressSanitizer and UBSan.

`oracle_sanitize.c` drives the transpose, O1 and O3 over small random
hypergraphs (including empty rows and one-vertex universes), several s,
thread counts and row selections, and the refused-argument paths; it is
built here with gcc and the sanitizers, and any report fails the run.
"""

from __future__ import annotations

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_under_sanitizers(tmp_path):
    exe = os.path.join(str(tmp_path), "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitize.c"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("gcc here has no sanitizer runtime: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert run.stdout.startswith("ok "), run.stdout
