"""The C-ABI library loads on the CPU host and exports every declared symbol."""

from __future__ import annotations

import ctypes
import os
import re

from paper_2010_11448_amd import sline

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions() -> list[str]:
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(sline_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("sline_create", "sline_destroy", "sline_build", "sline_edges_free",
                 "sline_status_str", "sline_last_error", "sline_last_stats"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sline.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_names_match_header():
    names = set(declared_functions())
    assert set(sline.SIGNATURES) <= names


def test_status_strings_without_gpu():
    assert sline.status_str(sline.SLINE_OK) == "ok"
    assert sline.status_str(sline.SLINE_ECAPACITY) == "output capacity too small"
    assert sline.status_str(12345) == "unknown status"


def test_null_arguments_rejected_without_gpu():
    lib = sline.load()
    assert lib.sline_create(None, 0, None, None) == sline.SLINE_EINVAL
    out = sline.sline_edges()
    assert lib.sline_build(None, sline.sline_csr(), 1, 0, 0, ctypes.byref(out)) == sline.SLINE_EINVAL
    assert lib.sline_last_stats(None, None) == sline.SLINE_EINVAL
    assert lib.sline_last_error(None) == b"no context"
    lib.sline_destroy(None)


def test_every_entry_point_rejects_a_null_handle_without_gpu():
    """Each declared call checks its handle and sizes before any device work."""
    lib = sline.load()
    E = sline.SLINE_EINVAL
    out = sline.sline_edges()
    csr = sline.sline_csr()
    i32, i64 = ctypes.c_int32(0), ctypes.c_int64(0)
    graph = sline.sline_graph()
    srv = ctypes.c_void_p()
    calls = {
        "sline_create": lambda: lib.sline_create(None, 0, None, None),
        "sline_build": lambda: lib.sline_build(None, csr, 1, 0, 0, ctypes.byref(out)),
        "sline_build_noalloc": lambda: lib.sline_build_noalloc(None, csr, 1, 0, 0,
                                                               ctypes.byref(out)),
        "sline_build_batch": lambda: lib.sline_build_batch(None, 1, None, None, None, 0, None),
        "sline_build_spgemm": lambda: lib.sline_build_spgemm(None, csr, 1, 0, 0,
                                                             ctypes.byref(out)),
        "sline_batch_plan_create": lambda: lib.sline_batch_plan_create(None, 1, None, None, None, 0,
                                                                       ctypes.byref(srv)),
        "sline_batch_plan_run": lambda: lib.sline_batch_plan_run(None, None, None),
        "sline_batch_plan_info": lambda: lib.sline_batch_plan_info(None, None, None, None),
        "sline_edges_free": lambda: lib.sline_edges_free(None, ctypes.byref(out)),
        "sline_filter": lambda: lib.sline_filter(None, ctypes.byref(out), 1, 0, ctypes.byref(out)),
        "sline_build_sweep": lambda: lib.sline_build_sweep(None, csr, 0, None, 0, 0, None),
        "sline_squeeze": lambda: lib.sline_squeeze(None, 0, ctypes.byref(out), 0,
                                                   ctypes.byref(graph)),
        "sline_graph_free": lambda: lib.sline_graph_free(None, ctypes.byref(graph)),
        "sline_components": lambda: lib.sline_components(None, 0, ctypes.byref(out), None, None),
        "sline_last_stats": lambda: lib.sline_last_stats(None, None),
        "sline_get_tuning": lambda: lib.sline_get_tuning(None, None),
        "sline_set_tuning": lambda: lib.sline_set_tuning(None, None),
        "sline_server_create": lambda: lib.sline_server_create(None, 0, 1 << 30, 8, 1),
        "sline_server_register": lambda: lib.sline_server_register(None, csr, ctypes.byref(i32)),
        "sline_server_submit": lambda: lib.sline_server_submit(None, 0, 1, 0, ctypes.byref(i64)),
        "sline_server_poll": lambda: lib.sline_server_poll(None, 0, ctypes.byref(out), None),
        "sline_server_release": lambda: lib.sline_server_release(None, ctypes.byref(out)),
        "sline_server_pending": lambda: lib.sline_server_pending(None, None, None),
        "sline_server_set_reuse": lambda: lib.sline_server_set_reuse(None, 0, 0, 0),
        "sline_server_reuse_stats": lambda: lib.sline_server_reuse_stats(None, None, None, None),
    }
    for name, call in calls.items():
        assert call() == E, name
    # sizes a server cannot have are refused before it touches a device
    for budget, batch, workers in ((0, 8, 1), (1 << 30, 0, 1), (1 << 30, 8, 0), (1 << 30, 8, 17)):
        assert lib.sline_server_create(ctypes.byref(srv), 0, budget, batch, workers) == E
    assert lib.sline_server_last_error(None) == b"no server"
    lib.sline_server_destroy(None)
    lib.sline_destroy(None)
    # every declared call is covered here or by a test above
    lib.sline_batch_plan_destroy(None)
    covered = set(calls) | {"sline_server_last_error", "sline_server_destroy", "sline_destroy",
                            "sline_last_error", "sline_status_str", "sline_batch_plan_destroy"}
    assert set(declared_functions()) <= covered


def test_struct_layouts_match_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets: a C program built against include/sline.h prints them."""
    import shutil
    import subprocess

    import pytest

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [sline.sline_csr, sline.sline_edges, sline.sline_stats, sline.sline_tuning,
               sline.sline_graph, sline.sline_query_info, sline.sline_allocator]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sline.h"',
             "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'    printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    c_side = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        name, field, value = line.split()
        c_side[(name, field)] = int(value)
    for st in structs:
        name = st.__name__
        assert c_side[(name, "sizeof")] == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert c_side[(name, field)] == getattr(st, field).offset, f"{name}.{field}"
    # the same fields, in the same order (a field missing at the end can hide
    # in the struct's padding)
    fields = header_struct_fields()
    for st in structs:
        assert [f for f, _ in st._fields_] == fields[st.__name__], st.__name__


def header_struct_fields() -> dict[str, list[str]]:
    """Field names, in order, of every `typedef struct { ... } name;` in the
    public header."""
    text = open(os.path.join(ROOT, "include", "sline.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            fp = re.search(r"\(\s*\*\s*(\w+)\s*\)", decl)  # function pointer
            names.append(fp.group(1) if fp else re.findall(r"\w+", decl)[-1])
        out[name] = names
    return out
