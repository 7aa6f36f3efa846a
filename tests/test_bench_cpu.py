"""bench.py pieces that need no GPU: the one-GPU refusal and the rule that a
committed counter summary is used only for the kernel source it was taken on."""

from __future__ import annotations

import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_follows_the_kernel_source(tmp_path):
    b = _bench()
    rec = b.committed_traffic("plain")
    if rec is not None:
        assert rec["kernel_sha"] == b.kernel_sha() and rec["bytes_per_launch"] > 0
    assert b.committed_traffic("no such form") is None
    # a summary taken on other kernel source is not used
    text = open(b.TRAFFIC_FILE).read()
    stale = tmp_path / "traffic.md"
    stale.write_text(text.replace(b.kernel_sha(), "0" * len(b.kernel_sha())))
    b.TRAFFIC_FILE = str(stale)
    assert b.committed_traffic("plain") is None
