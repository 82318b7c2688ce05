"""Host-side pieces of bench.py (CPU): the one-GPU guard, the algorithmic byte counts behind the
roofline, and the rule that measured traffic is used only for the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2506_19742_amd import nic, synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("precision", [0, 1])
def test_algorithmic_bytes_ct256(precision):
    w = synth.WORKLOADS["ct256"]
    cfg = nic.config_for(w, precision=precision)
    lay = nic.nic_describe(cfg)
    P = w.rays * w.samples
    ab = bench.algorithmic_bytes(cfg, lay, P, fused_adam=True)
    # 16 levels x 8 corners x 2 features, 4-byte gradients; gathers of 4 (FP32) or 2 (FP16) bytes
    assert ab["per_point"] == 16 * 8 * 2 * 4 == 1024
    assert ab["backward"] == 393216 * 1024 == 402653184
    assert ab["forward"] == 393216 * 16 * 8 * 2 * (2 if precision else 4)
    # the fused bin reduction also reads and writes each table parameter and its two moments
    n_table = lay["n_table"]
    assert ab["bin_reduce"] == 402653184 + n_table * (24 + (2 if precision else 0))
    assert ab["adam"] == lay["n_params_padded"] * 32


def test_mlp_flops_per_point_4x32():
    cfg = nic.config_for(synth.WORKLOADS["ct256"])
    fwd, bwd = bench.mlp_flops_per_point(cfg)
    macs = 32 * 32 + 3 * 32 * 32 + 32          # layer 0 (C = 32), three hidden 32 x 32, head
    assert fwd == 2 * macs and bwd == 3 * fwd


def test_measured_traffic_needs_matching_sources(tmp_path, monkeypatch):
    rec = {"source_sha": bench.kernel_source_sha(), "copy_scale": {},
           "workloads": {"ct256:p0": {"backward": {"bytes_per_launch": 123.0}}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(f))
    assert bench.measured_traffic("backward", "ct256", 0) == 123.0
    assert bench.measured_traffic("backward", "ct256", 1) is None
    rec["source_sha"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic("backward", "ct256", 0) is None

