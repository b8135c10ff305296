"""Host-side pieces of bench.py: the profile lookups behind the roofline
line and the one-GPU guard (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_traffic_profile_lookup(fake_root):
    sha = bench.kernel_sha()
    p = fake_root / "profiles" / "traffic_stepk_kernel_k3_c3_f32.md"
    p.write_text(f"text\n\nkernel_sha: {sha}\nhbm_bytes_per_launch: 1.8798e+10\n")
    assert bench.traffic_from_profile(sha, "c3", "f32", 9, 3) == pytest.approx(1.8798e10)
    # another kernel source, another launch shape, or no profile: no figure
    assert bench.traffic_from_profile("0" * 16, "c3", "f32", 9, 3) is None
    assert bench.traffic_from_profile(sha, "c3", "f32", 9, 1) is None
    assert bench.traffic_from_profile(sha, "c3", "f32", 5, 3) is None


def test_valu_profile_lookup(fake_root):
    sha = bench.kernel_sha()
    p = fake_root / "profiles" / "valu_step_kernels_c3_f32.md"
    p.write_text(f"table\n\nkernel_sha: {sha}\nvalu_per_node_step_k1: 463.34\nvalu_per_node_step_k3: 597.56\n")
    assert bench.valu_from_profile(sha, "c3", "f32", 9, 3) == pytest.approx(597.56)
    assert bench.valu_from_profile(sha, "c3", "f32", 9, 1) == pytest.approx(463.34)
    assert bench.valu_from_profile(sha, "c3", "f32", 9, 2) is None
    assert bench.valu_from_profile(sha, "c4", "f32", 9, 3) is None
    assert bench.valu_from_profile("0" * 16, "c3", "f32", 9, 3) is None


def test_issue_rate_and_bytes_per_node():
    # one 64-lane wave instruction per CU and clock: 256 CUs at 2.4 GHz
    assert bench.PEAK_VALU_GIPS == pytest.approx(256 * 64 * 2.4)
    # 27 populations read and written, Sr_prev read, Sr written
    assert bench.bytes_per_node("f32") == 27 * 4 * 2 + 8
    assert bench.bytes_per_node("f64") == 2 * 224
    assert bench.bytes_per_node("f32", 5) == 19 * 4 * 2 + 8


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_errors_against_fp64():
    import numpy as np
    ny, nx = 6, 7
    rf = {k: np.zeros((ny, nx)) for k in ("T_pcm", "T_mf", "f_l", "ux", "uy", "rho")}
    rf["ux"][2, 3] = 2.0
    f = {k: v.copy() for k, v in rf.items()}
    f["T_pcm"][0, 0] = 5.0          # a wall node: not counted
    f["T_pcm"][3, 3] = 0.25
    f["f_l"][1, 1] = 0.5
    f["uy"][4, 4] = 0.1
    rd = {"liquid_fraction": 0.2, "x_front_mid": 0.3, "Nu_hot": 4.0}
    d = {"liquid_fraction": 0.25, "x_front_mid": 0.35, "Nu_hot": 5.0}
    e = bench.errors_vs_f64(f, d, rf, rd, 0.5)
    assert e["T_pcm"] == pytest.approx(0.5) and e["T_mf"] == 0.0 and e["f_l"] == pytest.approx(0.5)
    assert e["u"] == pytest.approx(0.05) and e["Nu_hot_rel"] == pytest.approx(0.25)
    assert e["liquid_fraction"] == pytest.approx(0.05) and e["x_front_mid"] == pytest.approx(0.05)
