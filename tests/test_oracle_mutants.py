"""The oracle's pins have teeth: each planted mistake in the oracle fails one.

Every case below copies ``oracle/sline_oracle.c``, plants one plausible
mistake by an exact text substitution (a threshold off by one, a dropped or
extra pair, a wrong pointer step, a missing reset, a wrong id in the
transpose, a swapped output column, a wrong statistic), builds the copy with
gcc into a temporary folder, points the ``oracle`` wrapper at it and runs the
pins of ``test_oracle_pins`` against it.  The unmodified copy must pass them
all; every mutant must fail at least one.  Each substitution keeps every
memory access in bounds, so a mutant can only give wrong answers.
"""

from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_pins_stages as stages

SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "sline_oracle.c")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("o1 threshold off by one",
     "if (w >= J->s) record(J, ri, a, b, w);", "if (w > J->s) record(J, ri, a, b, w);"),
    ("o1 skips the next item",
     "for (int32_t b = a + 1; b < J->N; ++b)", "for (int32_t b = a + 2; b < J->N; ++b)"),
    ("merge advances the wrong list",
     "if (x[i] < y[j]) ++i;\n        else if (y[j] < x[i]) ++j;\n        else { ++c;",
     "if (x[i] < y[j]) ++j;\n        else if (y[j] < x[i]) ++j;\n        else { ++c;"),
    ("short-circuit merge advances the wrong list",
     "if (x[i] < y[j]) ++i;\n        else if (y[j] < x[i]) ++j;\n        else {\n",
     "if (x[i] < y[j]) ++j;\n        else if (y[j] < x[i]) ++j;\n        else {\n"),
    ("o3 counts the item with itself",
     "if (b <= a) continue;", "if (b < a) continue;"),
    ("o3 prunes items of size s",
     "if (J->rp[b + 1] - J->rp[b] < J->s) continue;",
     "if (J->rp[b + 1] - J->rp[b] <= J->s) continue;"),
    ("o3 threshold off by one",
     "if (cnt[b] >= J->s) record(J, ri, a, b, cnt[b]);",
     "if (cnt[b] > J->s) record(J, ri, a, b, cnt[b]);"),
    ("o3 never clears its counters",
     "cnt[b] = 0;", ";"),
    ("transpose writes reversed item ids",
     "colT[fill[col[k]]++] = i;", "colT[fill[col[k]]++] = m - 1 - i;"),
    ("gather swaps the item and weight columns",
     "out->w[o] = Jt->out.w[base + q];", "out->w[o] = Jt->out.b[base + q];"),
    ("weight sum counts pairs",
     "J->st.sum_w += w;", "J->st.sum_w += 1;"),
    ("o2 prunes items of size s",
     "if (prune && ni < J->s) continue;", "if (prune && ni <= J->s) continue;"),
    ("o2 never resets its visited flags",
     "for (int64_t t = 0; t < nt; ++t) visited[touched[t]] = 0;", ";"),
    ("o2 short-circuits one member early",
     "if (++c >= s) return 1;", "if (++c >= s - 1) return 1;"),
    ("o2 keeps the diagonal",
     "if (i >= j) continue;                  /* strictly upper triangle */",
     "if (i > j) continue;"),
    ("o2 counts an intersection per accepted pair only",
     "J->st.intersections++;\n                const int ok",
     "const int ok"),
    ("components link the smaller root under the larger",
     "if (ra < rb) comp[rb] = ra;", "if (ra < rb) comp[ra] = rb;"),
]


def _dense_cases():
    rng = np.random.default_rng(2024)
    for m, n, p in ((12, 9, 0.4), (20, 15, 0.25), (7, 30, 0.3)):
        B = (rng.random((m, n)) < p).astype(np.int64)
        g = pins.csr_from_dense(B)
        for s in (1, 2, 3):
            for dual in (0, 1):
                pins.check_against_dense(g, s, dual)


BATTERY = [
    ("dense product", _dense_cases),
    ("structure families", pins.test_structure_families),
    ("worked example", pins.test_worked_example_text_facts),
    ("pruning and bounds", pins.test_pruning_and_bounds),
    ("brute force", pins.test_symmetric_by_brute_force),
    ("dual is the transpose", pins.test_dual_is_the_transposed_hypergraph),
    ("o3 equals o1", pins.test_o3_equals_o1_on_planted_and_random),
    ("weight sum closed form", pins.test_weight_sum_closed_form),
    ("naive intersection count", pins.test_naive_makes_all_pairs_intersections),
    ("digest", pins.test_digest_terms_and_sum),
    ("o2 variants equal the dense product",
     lambda: [stages.test_o2_variants_return_the_dense_product_result(v)
              for v in sorted(oracle.VARIANTS)]),
    ("o2 intersection closed forms",
     lambda: [stages.test_o2_intersection_counts_match_closed_forms(v)
              for v in sorted(oracle.VARIANTS)]),
    ("components match scipy", stages.test_components_match_scipy),
    ("components closed forms", stages.test_components_closed_forms),
]


def _build(text: str, folder, name: str) -> str:
    src = os.path.join(str(folder), name + ".c")
    lib = os.path.join(str(folder), name + ".so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", src,
                           "-o", lib])
    return lib


def _first_failure(lib: str, monkeypatch) -> str | None:
    """Name of the first pin that fails with the oracle built as ``lib``."""
    monkeypatch.setattr(oracle, "_LIB", lib)
    monkeypatch.setattr(oracle, "_lib", None)
    try:
        for name, pin in BATTERY:
            try:
                pin()
            except (AssertionError, KeyError, RuntimeError, ValueError):
                return name
        return None
    finally:
        monkeypatch.undo()


def test_unmodified_copy_passes_every_pin(tmp_path, monkeypatch):
    text = open(SRC).read()
    assert _first_failure(_build(text, tmp_path, "control"), monkeypatch) is None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(name, old, new, tmp_path, monkeypatch):
    text = open(SRC).read()
    old, new = old.replace("\\n", "\n"), new.replace("\\n", "\n")
    assert text.count(old) == 1, f"mutation site for '{name}' not found once in the oracle"
    lib = _build(text.replace(old, new), tmp_path, "mutant")
    caught = _first_failure(lib, monkeypatch)
    assert caught is not None, f"no pin fails when the oracle has: {name}"
