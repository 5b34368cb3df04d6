"""CPU checks of bench.py's contract pieces that need no GPU: the one-GPU guard, the profile
summarisers, and the rule that counter traffic is reported only for the kernel source it was
measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_summarize_trace(tmp_path):
    (tmp_path / "run_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        '"k_a",3,3000,1000.0,75.0,900,1100,50\n"k_b",1,1000,1000.0,25.0,1000,1000,0\n')
    md = bench.summarize_trace(str(tmp_path))
    assert "| `k_a` | 3 | 1.0 | 0.9 | 1.1 | 75.00 |" in md


def test_summarize_pmc_calibrates(tmp_path):
    def write(d, counter, kernel, vals):
        d.mkdir()
        rows = ['"Kernel_Name","Counter_Name","Counter_Value"']
        rows += [f'"{kernel}","{counter}",{v}' for v in vals]
        (d / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    write(tmp_path / "f", "FETCH_SIZE", "k_ttmc3_lds<float>(args)", [100.0, 300.0])
    write(tmp_path / "w", "WRITE_SIZE", "k_ttmc3_lds<float>(args)", [50.0])
    write(tmp_path / "cf", "FETCH_SIZE", "__amd_rocclr_copyBuffer", [262144.0])
    write(tmp_path / "cw", "WRITE_SIZE", "__amd_rocclr_copyBuffer", [524288.0])
    text = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                               kernel="k_ttmc3_lds<float>")
    # fetch 200 KiB x 2 (copy reads count half) + write 50 KiB x 1
    assert "traffic bytes per launch: %d" % ((200 * 2 + 50) * 1024) in text


def test_traffic_needs_matching_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "p.md"
    prof.write_text("traffic bytes per launch: 1234\nttmc.hip sha256: %s\n" % bench._sha256(bench.TTMC_SOURCE))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.measured_traffic() == 1234.0
    prof.write_text("traffic bytes per launch: 1234\nttmc.hip sha256: 00\n")
    assert bench.measured_traffic() is None


def test_committed_profile_is_well_formed():
    """The committed counter summary of the default workload names its traffic and the hash of
    the kernel source it was taken on (bench.py reports the traffic only while that hash matches)."""
    text = open(bench.TRAFFIC_PROFILE).read()
    assert "traffic bytes per launch:" in text and "ttmc.hip sha256:" in text
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text


def test_oracle_fit_lookup():
    """The stored oracle fit sequences are found by workload name, whatever the TTMc type."""
    fits = bench.oracle_fits("zipf_500000x100000x365_nnz50000000_r10_f32")
    assert fits is not None and len(fits) == 5
    assert bench.oracle_fits("zipf_500000x100000x365_nnz50000000_r10_bf16") == fits
    assert len(bench.oracle_fits("lowrank_10000x10000x10000_nnz10000000_r16_f32")) == 10
    assert bench.oracle_fits("no_such_workload") is None


def test_host_info():
    model, avail, threads = bench.host_info()
    assert isinstance(model, str) and model
    assert 1 <= threads <= avail
