"""The byte model behind the benchmark's GB/s and roofline figures, checked
against closed forms and hand counts (no GPU needed)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("m", [1, 2, 5, 10, 30])
@pytest.mark.parametrize("T", [4, 8])
def test_cg_sweep_bytes_closed_form(bench, m, T):
    """Per unknown and sweep: residual 16 + T; iteration 0 moves 2T
    (stencil) + 4T (update); later iterations 3T + 5T; the last update is
    replaced by the outer update (16 + 2T, or 16 + T when m = 1)."""
    if m == 1:
        want = (16 + T) + 2 * T + (16 + T)
    else:
        want = (16 + T) + 2 * T + 4 * T + (m - 1) * 3 * T + (m - 2) * 5 * T + (16 + 2 * T)
    assert bench.sweep_bytes(m, T) == want
    kinds = [k for k, _ in bench.kernel_bytes(m, T)]
    assert kinds.count("stencil") == m and kinds.count("update") == m - 1
    assert kinds[0] == "resid" and kinds[-1] == "final"


def test_documented_sweep_bytes(bench):
    # m = 10: 336 B mixed, 640 B FP64 (CG); 636 / 1240 B (GMRES)
    assert bench.sweep_bytes(10, 4) == 336 and bench.sweep_bytes(10, 8) == 640
    assert bench.sweep_bytes(10, 4, gmres=True) == 636
    assert bench.sweep_bytes(10, 8, gmres=True) == 1240
    # the method's own model: 10 words per CG iteration plus the outer step
    assert bench.model_sweep_bytes(10, True) == 440 and bench.model_sweep_bytes(10, False) == 848


@pytest.mark.parametrize("m", [1, 4, 10, 20])
@pytest.mark.parametrize("T", [4, 8])
def test_gmres_sweep_bytes_closed_form(bench, m, T):
    """Classical Gram-Schmidt reads every earlier basis vector twice per
    step: 32 + T (m^2 + 5m + 1) bytes per unknown and sweep."""
    assert bench.sweep_bytes(m, T, gmres=True) == 32 + T * (m * m + 5 * m + 1)


def test_region_cells(bench):
    # no overlap: the grid
    assert bench.region_cells((48, 40, 36), ([0, 16, 48], [0, 40], [0, 12, 36]), 0) == 48 * 40 * 36
    # 8^3 in 2^3 blocks of 4^3, overlap 1: x and y extents 4 + 1 (one
    # neighbour per block), z grown by 1 rounded up to 4 cells: 4 + 4
    assert bench.region_cells((8, 8, 8), [[0, 4, 8]] * 3, 1) == (5 + 5) * (5 + 5) * (8 + 8)
    # three blocks along x (middle block grown on both sides), z cuts not
    # multiples of 2 (z grows by exactly the overlap)
    shape, cuts = (12, 4, 5), ([0, 4, 8, 12], [0, 4], [0, 2, 5])
    x = [4 + 2, 4 + 2 + 2, 4 + 2]
    z = [2 + 2, 3 + 2]
    assert bench.region_cells(shape, cuts, 2) == sum(x) * 4 * sum(z)
