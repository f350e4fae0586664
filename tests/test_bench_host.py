"""Host logic of bench.py (no GPU): counter readings are used only for the
kernel source and launch shape they were taken on, the full-storage run
reads its own entry, and the multi-GPU request is refused."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    """bench.py with its root moved to a scratch tree holding a stand-in
    kernel source and a counter summary taken on it."""
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    src = tmp_path / "paper_2008_11778_amd" / "csrc" / "wave_kernels.hip"
    src.parent.mkdir(parents=True)
    src.write_bytes(b"// stand-in kernel source\n")
    (tmp_path / "profiles").mkdir()
    summary = {
        "source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(), "fetch_factor": 2.0, "write_factor": 1.0,
        "kernels": {
            "fwd_step": {"fetch_kib": 100.0, "write_kib": 50.0, "steps_per_launch": 1, "rows": 8, "order": 0},
            "rec_step": {"fetch_kib": 110.0, "write_kib": 90.0, "steps_per_launch": 1, "rows": 64, "order": 0},
            "kept_forward": {"fetch_kib": 120.0, "write_kib": 95.0, "steps_per_launch": 1, "rows": 64, "order": 0},
            "adj_step": {"fetch_kib": 300.0, "write_kib": 150.0, "steps_per_launch": 2, "rows": 20, "order": 1}},
        "large_kernels": {
            "fwd_step": {"fetch_kib": 400.0, "write_kib": 300.0, "steps_per_launch": 2, "rows": 48, "order": 0}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(summary))
    monkeypatch.setattr(mod, "ROOT", str(tmp_path))
    mod._summary = summary
    mod._src = src
    return mod


def shape_of(entry, kid):
    return {kid: entry["rows"], f"order{kid}": entry["order"]}


def calibrated(e):
    return round((e["fetch_kib"] * 2.0 + e["write_kib"] * 1.0) * 1024.0)


def test_lookup_by_kernel_and_launch_shape(bench):
    ks = bench._summary["kernels"]
    for name, kid in (("fwd_step", 0), ("rec_step", 1), ("adj_step", 2)):
        e = ks[name]
        assert bench.measured_traffic(name, e["steps_per_launch"], shape_of(e, kid)) == calibrated(e)
        other = shape_of(e, kid)
        other[kid] += 4
        assert bench.measured_traffic(name, e["steps_per_launch"], other) is None
        other = shape_of(e, kid)
        other[f"order{kid}"] ^= 1
        assert bench.measured_traffic(name, e["steps_per_launch"], other) is None
        assert bench.measured_traffic(name, 3 - e["steps_per_launch"], shape_of(e, kid)) is None


def test_full_storage_reads_the_kept_forward_entry(bench):
    ks = bench._summary["kernels"]
    e = ks["kept_forward"]
    assert bench.measured_traffic("rec_step", 1, shape_of(e, 1), full=True) == calibrated(e)
    assert bench.measured_traffic("rec_step", 1, shape_of(e, 1)) == calibrated(ks["rec_step"])


def test_large_grid_section(bench):
    e = bench._summary["large_kernels"]["fwd_step"]
    assert bench.measured_traffic("fwd_step", 2, shape_of(e, 0), "large_kernels") == calibrated(e)
    assert bench.measured_traffic("adj_step", 2, {2: 20, "order2": 1}, "large_kernels") is None


def test_other_kernel_source_gives_no_reading(bench):
    e = bench._summary["kernels"]["fwd_step"]
    bench._src.write_bytes(b"// changed kernel source\n")
    assert bench.measured_traffic("fwd_step", 1, shape_of(e, 0)) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU only" in p.stderr
