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


def test_team_byte_counts(bench):
    """Resident-team sweeps: x and b read, x written through HBM; per inner
    iteration two stencil applies from LDS (5 z vectors and 2 single cells
    per vector of 4 FP32 or 2 FP64 cells) and one read and write of p."""
    assert bench.TEAM_HBM_BYTES == 24
    assert bench.team_lds_bytes(4) == 2 * (5 * 4 + 2) * 4 / 4 + 8 == 52
    assert bench.team_lds_bytes(8) == 2 * (5 * 2 + 2) * 8 / 2 + 16 == 112
    assert abs(bench.LDS_PEAK_GBPS - 78643.2) < 1e-6


def test_counter_summary(tmp_path):
    """The rocprofv3 counter summary: kernel classes from demangled names,
    calibration on the 1 GiB copies, bytes per launch with the launch sizes
    from the bench line."""
    import json
    from paper_2009_12638_amd import pmc
    assert pmc.kernel_class("ms::k_update<float, 4, 1, true, false>") == ("final", "mixed")
    assert pmc.kernel_class("ms::k_update<double, 2, 1, false, false>") == ("update", "fp64")
    assert pmc.kernel_class("ms::k_resid<float, 4, 1, false, false>") is None
    assert pmc.kernel_class("ms::k_team<double, 2, 8, false, false>") == ("team", "fp64")
    assert pmc.short_name("void ms::k_stencil<float, 4, 1>(ms::Geom, int)") == \
        "ms::k_stencil<float, 4, 1>"
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    for counter, copy_kib, team_kib in (("FETCH_SIZE", 524288.0, 1000.0),
                                        ("WRITE_SIZE", 1048576.0, 3000.0)):
        d = tmp_path / counter
        d.mkdir()
        rows = [f"1,void __amd_rocclr_copyBuffer(),{counter},{copy_kib}",
                f"2,void __amd_rocclr_copyBuffer(),{counter},{copy_kib / 64}",
                f"3,\"void ms::k_team<float, 4, 8, false, false>(ms::Geom, int)\",{counter},"
                f"{team_kib}"]
        (d / "run_counter_collection.csv").write_text(hdr + "\n".join(rows) + "\n")
    line = {"config": {"workload": "w"},
            "modes": {"sync-mixed": {"kernels": {"team": {"unknowns_per_launch": 1024}}}}}
    bj = tmp_path / "bench.json"
    bj.write_text("[bench] log\n" + json.dumps(line) + "\n")
    out = tmp_path / "t.json"
    pmc.traffic(str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"), str(bj), str(out),
                str(tmp_path / "t.md"), "cmd")
    data = json.loads(out.read_text())
    assert abs(data["fetch_scale"] - 2.0) < 1e-12 and data["write_scale"] == 1.0
    k = data["kernels"]["team:mixed"]
    assert k["fetch_bytes_per_launch"] == 2 * 1000.0 * 1024
    assert k["write_bytes_per_launch"] == 3000.0 * 1024
    assert k["unknowns_per_launch"] == 1024
    assert data["kernel_source_sha1"] == pmc.source_sha1()
