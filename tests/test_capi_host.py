"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/ms.h declares, rejects invalid arguments before
touching the device, and the Python binding mirrors the header's structs."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2009_12638_amd import ms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "ms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ms.LIB_PATH):
        from paper_2009_12638_amd import build
        build.build()
    return ms.lib()


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert "ms_solve" in names and "ms_create" in names and "ms_residual" in names
    for n in names:
        assert hasattr(L, n), f"libms.so does not export {n}"


STRUCTS = ["ms_grid", "ms_blocks", "ms_bc", "ms_opts", "ms_stats"]


def c_layout(tmp_path):
    """sizeof and offsetof of every member of the header's structs, as gcc
    lays them out (a small C program that includes ms.h)."""
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ms.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(ms, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for ln in out.splitlines():
        sname, field, val = ln.split()
        table[(sname, field)] = int(val)
    return table


def test_struct_layouts_match_gcc(tmp_path):
    # the binding's ctypes structs name every header member, in order, at
    # gcc's offsets and with gcc's sizes
    table = c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(ms, name)
        assert C.sizeof(cls) == table[(name, "size")], name
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == table[(name, fname)], f"{name}.{fname}"
    # and no header member is missing from the binding
    text = open(os.path.join(ROOT, "include", "ms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    for name in STRUCTS:
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text, flags=re.S)
        assert body, name
        decl = re.sub(r"\[[^\]]*\]", "", body.group(1))
        members = re.findall(r"\*?\s*([a-z_][a-z0-9_]*)\s*(?=[,;])", decl)
        assert sorted(members) == sorted(f for f, _ in getattr(ms, name)._fields_), name


def test_status_strings(L):
    assert ms.ms_status_string(0) == "MS_OK"
    assert ms.ms_status_string(4) == "MS_ERR_NOT_CONVERGED"
    assert "libms" in ms.ms_version()


def test_default_opts(L):
    o = ms.ms_default_opts()
    assert o.max_sweeps == 100000 and o.staleness == 2 and o.precision == 0
    assert o.use_graph == 1 and o.inner_solver == ms.MS_INNER_CG


@pytest.mark.parametrize("shape,blocks,cuts,why", [
    ((0, 4, 4), (1, 1, 1), None, "sizes"),
    ((8, 8, 8), (3, 1, 1), None, "uniform split"),
    ((8, 8, 8), (0, 1, 1), None, "block counts"),
    ((8, 8, 8), None, ([0, 4, 8], [0, 8], [0, 5, 5, 8]), "cuts"),
    ((8, 8, 8), None, ([0, 4, 9], [0, 8], [0, 8]), "cuts"),
    ((8, 8, 8), (9, 1, 1), None, "more blocks"),
])
def test_create_rejects_bad_arguments(L, shape, blocks, cuts, why):
    with pytest.raises(ms.MsError) as e:
        ms.ms_create(shape, blocks=blocks, cuts=cuts)
    assert e.value.status == ms.MS_ERR_ARG
    assert why.split()[0] in ms.ms_last_error(None)


def test_null_handle_is_an_argument_error(L):
    st = L.ms_solve(None, None, None, 1e-8, 10, 0, None, None)
    assert st == ms.MS_ERR_ARG
    L.ms_destroy(None)  # ignored
