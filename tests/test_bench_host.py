"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the counter
calibration that turns rocprofv3 FETCH_SIZE / WRITE_SIZE into HBM bytes per
pixel, and the staleness rule that drops those bytes once the sweep kernels'
sources change."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def _csv(path, counter, rows):
    with open(path, "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (name, val) in enumerate(rows):
            fh.write(f'{i},"{name}",{counter},{val}\n')


def test_counter_calibration_and_staleness(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h1")
    px = 32 * 1024 * 1024
    copy_kib = bench.COPY_BYTES / 1024.0
    s11 = "void pwf::col_sweep<1024, 8, 6>(pwf::Sweep)"
    # FETCH_SIZE reads half of the copy's bytes, WRITE_SIZE all of them (as measured on the MI355X)
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy_kib / 2), (s11, 32.0 * px / 1024 / 2),
                                            (s11, 32.0 * px / 1024 / 2)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy_kib), (s11, 24.0 * px / 1024),
                                            (s11, 24.0 * px / 1024)])
    assert bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 32) == 0
    rec = json.load(open(tmp_path / "profiles" / "traffic_counters.json"))
    assert abs(rec["sweeps"]["11:8"]["hbm_bytes_per_px"] - 56.0) < 1e-9   # 32 B read + 24 B written per pixel
    assert abs(bench.measured_traffic(11, px, 8) - 56.0 * px) < 1e-3
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h2")      # the sweep sources changed
    assert bench.measured_traffic(11, px, 8) is None


def test_counter_ingest_at_another_side(tmp_path, monkeypatch):
    """A --side 2048 counter run goes to its own file, keyed by the 2048 kernels, and
    leaves the 1024^2 record (the bench's roofline.traffic) alone."""
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h1")
    px = 4 * 2048 * 2048
    copy_kib = bench.COPY_BYTES / 1024.0
    chirp = "void pwf::col_sweep<2048, 8, 0>(pwf::Sweep)"
    other = "void pwf::col_sweep<1024, 8, 0>(pwf::Sweep)"
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy_kib / 2), (chirp, 8.0 * px / 1024 / 2),
                                            (other, 1.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy_kib), (chirp, 8.5 * px / 1024),
                                            (other, 1.0)])
    assert bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 4, side=2048) == 0
    assert not os.path.exists(tmp_path / "profiles" / "traffic_counters.json")
    rec = json.load(open(tmp_path / "profiles" / "traffic_counters_2048.json"))
    assert rec["side"] == 2048 and set(rec["sweeps"]) == {"1:8"}
    assert abs(rec["sweeps"]["1:8"]["hbm_bytes_per_px"] - 16.5) < 1e-9
    assert bench.measured_traffic(1, px, 8) is None


def test_compiled_widths_from_the_library():
    """The counter runs launch every compiled column-tile width, asked of the library (host
    calls only), the default first; the settings are left at the defaults."""
    from paper_2503_20146_amd import _lib
    lib = _lib.load()
    assert bench.compiled_widths(lib, 1024) == [16, 8]
    assert bench.compiled_widths(lib, 2048) == [8, 16]
    assert bench.compiled_widths(lib, 512) == [16, 32]
    assert lib.pwf_column_tile(1024, 11) == 16 and lib.pwf_column_tile(2048, 11) == 8
