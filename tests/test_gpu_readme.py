"""The Python example in README.md runs as printed and gives the oracle's answers."""

from __future__ import annotations

import contextlib
import io
import os
import re

import numpy as np
import pytest

import oracle

from helpers import assert_same

pytestmark = pytest.mark.gpu

README = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "README.md")


def test_readme_example():
    text = open(README).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert len(blocks) == 1
    ns: dict = {}
    buf = io.StringIO()
    print("case: README example", flush=True)
    with contextlib.redirect_stdout(buf):
        exec(compile(blocks[0], "README.md", "exec"), ns)
    assert buf.getvalue().strip() == "[0, 0] [1, 2] [2, 2]"
    rp = ns["row_ptr"].cpu().numpy()
    col = ns["col"].cpu().numpy()
    ref, _ = oracle.naive(rp, col, len(rp) - 1, 5, 2, dual=1)
    assert_same(ns["D"], ref, "README dual s=2")
    for got, plan_got, s in zip(ns["outs"], ns["P"], (1, 2)):
        ref, _ = oracle.naive(rp, col, len(rp) - 1, 5, s)
        assert_same(got, ref, f"README batch s={s}")
        assert_same(plan_got, ref, f"README plan s={s}")
    assert np.array_equal(ns["L"].w.cpu().numpy(), [2, 2])
