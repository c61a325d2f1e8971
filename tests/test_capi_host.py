"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/ms.h declares, rejects invalid arguments before
touching the device, and the Python binding mirrors the header's structs."""
import ctypes as C
import os
import re

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


def test_struct_sizes_match_c_layout():
    # sizes fixed by the C rules for the header's member lists
    assert C.sizeof(ms.ms_grid) == 24
    assert C.sizeof(ms.ms_blocks) == 12 + 4 + 24
    assert C.sizeof(ms.ms_bc) == 48
    # max_sweeps, pad, inner_tol, staleness, precision, stream, five int32
    # options, rows, workers, inner_solver, z_vector, tail padding to 8
    assert C.sizeof(ms.ms_opts) == 4 + 4 + 8 + 4 + 4 + 8 + 4 * 5 + 4 + 4 + 4 + 4 + 4
    assert C.sizeof(ms.ms_stats) == 4 + 4 + 8 + 8 + 8 + 4 + 4 + 4 + 4 + 8 + 4 + 4 + 64 + 64


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
