"""Host logic of bench.py (no GPU): the one-GPU guard, the choice of the dominant
kernel, the roofline arithmetic and the lookup of the measured HBM traffic."""
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
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _prof(**ms):
    return {k: {"launches": 10, "total_ms": v, "bytes": 1e9 * 10, "flops": 1e12 * 10} for k, v in ms.items()}


def test_dominant_class_is_the_largest_single_kernel_class():
    p = _prof(bj_apply=5.0, jvp=2.0, mdot=9.0)   # mdot spans several kernels: not a candidate
    assert bench.dominant_class(p) == "bj_apply"


def test_roofline_arithmetic():
    p = _prof(bj_apply=2.5)                      # 1 GB per launch in 0.25 ms -> 4000 GB/s
    r = bench.roofline_of(p, "no_such_workload", "mixed")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert r["traffic"] is None                  # no counter record for this workload
    p = _prof(bj_invert=5.0)                     # 1 TFLOP per launch in 0.5 ms -> 2000 TFLOP/s
    r32 = bench.roofline_of(p, "w", "mixed")
    r64 = bench.roofline_of(p, "w", "fp64")
    assert r32["bound"] == "alu" and r32["peak"] == bench.FP32_PEAK_TFLOPS and r64["peak"] == bench.FP64_PEAK_TFLOPS
    assert abs(r32["achieved"] - 2000.0) < 1e-9


def test_measured_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "kernel.hip"
    src.write_text("// a kernel\n")
    import hashlib
    rec = {"kernel": "bj_apply", "workload": "wl", "bytes_per_launch": 123456789, "source": "kernel.hip",
           "sha256": hashlib.sha256(src.read_bytes()).hexdigest()}
    (tmp_path / "profiles" / "bj_apply_wl_traffic.md").write_text("text\n<!-- traffic %s -->\n" % json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("bj_apply", "wl") == 123456789.0
    assert bench.measured_traffic("bj_apply", "other") is None
    src.write_text("// the kernel changed\n")
    assert bench.measured_traffic("bj_apply", "wl") is None


def test_committed_traffic_records_are_current():
    """Every committed counter record that bench.py reads names a kernel source whose SHA-256 it
    recorded; a kernel changed since its counters were taken would make the bench report no
    measured traffic."""
    import glob
    import hashlib
    import re
    recs = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        m = re.search(r"<!-- traffic (\{.*\}) -->", open(path).read())
        if m:
            recs.append((path, json.loads(m.group(1))))
    assert recs
    for path, rec in recs:
        src = os.path.join(ROOT, rec["source"])
        assert hashlib.sha256(open(src, "rb").read()).hexdigest() == rec["sha256"], os.path.basename(path)
        assert bench.measured_traffic(rec["kernel"], rec["workload"]) == float(rec["bytes_per_launch"])


def test_form_settings():
    """Each benchmark form maps to the precision, preconditioner and block storage it names."""
    assert bench.form_settings("fp64") == ("fp64", "bjext", 0)
    assert bench.form_settings("mixed") == ("mixed", "bjext", 0)
    assert bench.form_settings("mixed16") == ("mixed", "bjext", 1)
    assert bench.form_settings("fp64_h") == ("fp64", "bjext_h", 0)
    assert bench.form_settings("mixed_h") == ("mixed", "bjext_h", 0)
    for f in ("learned", "learned_first", "learned_guess"):
        assert bench.form_settings(f) == ("mixed", f, 0)
    with pytest.raises(ValueError):
        bench.form_settings("fp16")
    assert bench.STUDY_PC == ("none", "bjext", "bjext_h")


def test_profile_commands_run_committed_files():
    """Every profile summary gives the command that made it, and the scripts that command runs
    are files of this repository (no working files)."""
    import glob
    import re
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert paths
    for path in paths:
        text = open(path).read()
        blocks = re.findall(r"```\n(.*?)```", text, re.S)
        assert blocks, os.path.basename(path)
        cmd = " ".join(blocks)
        assert "rocprofv3" in cmd, os.path.basename(path)
        assert "_work" not in cmd, os.path.basename(path)
        for script in re.findall(r"(?:python3?|--)\s+(\S+\.py)", cmd):
            assert os.path.exists(os.path.join(ROOT, script)), (os.path.basename(path), script)
