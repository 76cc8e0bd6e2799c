"""The C-ABI library loads and exports every symbol include/rbdi.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rbdi.h")).read()
    return sorted(set(re.findall(r"RBDI_API\s+[\w\s\*]+?\b(rbdi_\w+)\s*\(", txt)))


def test_header_declares_the_api():
    syms = declared_symbols()
    for s in ("rbdi_create", "rbdi_step", "rbdi_set_rigid_sdf", "rbdi_rigid_force", "rbdi_set_material"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2111_11806_amd import build, rbdi
    if not os.path.exists(build.LIB):
        build.build(force=False)
    lib = rbdi.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    out = subprocess.run(["nm", "-D", "--defined-only", build.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (rbdi_\w+)", out))
    assert set(declared_symbols()) <= exported
    assert set(rbdi.EXPORTS) == set(declared_symbols())


def test_bad_arguments_fail_without_gpu_work():
    from paper_2111_11806_amd import rbdi
    lib = rbdi.load()
    h = ctypes.c_void_p()
    d = rbdi.Desc()
    d.dim = 4
    assert lib.rbdi_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"dim" in lib.rbdi_last_error()
    assert lib.rbdi_create(None, ctypes.byref(h)) == -1


def test_elvira_outside_2d_is_rejected():
    """ELVIRA normals exist in 2D only; other dimensions fail at create,
    before any device work."""
    from paper_2111_11806_amd import rbdi
    lib = rbdi.load()
    h = ctypes.c_void_p()
    d = rbdi.Desc()
    d.dim = 3
    for a in range(3):
        d.n[a] = 8
        d.dx[a] = 0.125
    d.nmat = 1
    d.thinc_beta = 1.6
    d.lm_mach = 0.1
    d.normal = 1
    assert lib.rbdi_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"ELVIRA" in lib.rbdi_last_error()
    d.normal = 2
    assert lib.rbdi_create(ctypes.byref(d), ctypes.byref(h)) == -1


def _desc2d(rbdi, nx, ny):
    d = rbdi.Desc()
    d.dim = 2
    d.n[0], d.n[1], d.n[2] = nx, ny, 1
    d.dx[0] = d.dx[1] = d.dx[2] = 0.01
    d.nmat = 1
    d.thinc_beta = 1.6
    d.lm_mach = 0.1
    return d


def test_empty_and_oversized_grids_are_rejected():
    """Degenerate sizes fail at create, before any device work: an empty grid,
    2^31 cells (band indices are 32-bit), a reflective face on fewer cells
    than the 3-cell halo."""
    from paper_2111_11806_amd import rbdi
    lib = rbdi.load()
    h = ctypes.c_void_p()
    for nx, ny in ((0, 8), (8, 0), (-1, 8)):
        assert lib.rbdi_create(ctypes.byref(_desc2d(rbdi, nx, ny)), ctypes.byref(h)) == -1
        assert b"grid size" in lib.rbdi_last_error()
    assert lib.rbdi_create(ctypes.byref(_desc2d(rbdi, 1 << 16, 1 << 15)), ctypes.byref(h)) == -1
    assert b"too many cells" in lib.rbdi_last_error()
    d = _desc2d(rbdi, 8, 2)
    d.bc[2] = d.bc[3] = 1  # reflective y faces on 2 rows
    assert lib.rbdi_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"reflective" in lib.rbdi_last_error()
    d = _desc2d(rbdi, 8, 8)
    d.n[2] = 2  # unused dimension must be 1
    assert lib.rbdi_create(ctypes.byref(d), ctypes.byref(h)) == -1


def test_bench_traffic_needs_matching_sources(tmp_path):
    """The benchmark reports measured HBM traffic only from a counter summary
    taken on the current kernel sources and grid."""
    import bench
    sweeps = ("sweep_z", "sweep_y", "sweep_x")
    good = bench.measured_traffic(bench.TRAFFIC_COPPER, 256 ** 3, sweeps)
    if good is not None:
        assert bench.measured_traffic(bench.TRAFFIC_COPPER, 128 ** 3, sweeps) is None
    fake = tmp_path / "traffic.txt"
    keys = ["cells: 524288", "copy_bytes_read: 1", "copy_bytes_written: 1", "copy_fetch_kib: 1",
            "copy_write_kib: 1", "sweep_y_fetch_kib: 1", "sweep_y_write_kib: 1", "sweep_x_fetch_kib: 1",
            "sweep_x_write_kib: 1"]
    fake.write_text("\n".join(["source_sha1: 0000"] + keys) + "\n")
    assert bench.measured_traffic(str(fake), 524288, ("sweep_y", "sweep_x")) is None  # other sources
    fake.write_text("\n".join(["source_sha1: " + bench.kernel_source_hash()] + keys) + "\n")
    # 2 + 2 KiB counted, each KiB worth 1 byte by the copy scale: 4 bytes
    assert bench.measured_traffic(str(fake), 524288, ("sweep_y", "sweep_x")) == 4
    assert bench.measured_traffic(str(fake), 1000, ("sweep_y", "sweep_x")) is None    # other grid
    assert bench.measured_traffic(str(fake), 524288, sweeps) is None                  # a sweep missing
