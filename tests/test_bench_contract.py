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
    assert ab["encode"] == 393216 * 16 * 8 * 2 * (2 if precision else 4)
    assert ab["forward"] == 393216 * 16 * 2 * 4          # the stored encoding, read back
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



def _write_counter_csv(d, rows):
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    import csv
    with open(os.path.join(d, "host", "run_counter_collection.csv"), "w", newline="") as f:
        wr = csv.writer(f, quoting=csv.QUOTE_ALL)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writerows(rows)


def test_pmc_summary_scales_counters_by_the_copy(tmp_path, capsys):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of each kernel, scaled so that the plain copy of
    COPY_BYTES reads and writes COPY_BYTES; k_bin_reduce and k_bin_combine add up to one kind."""
    kib = bench.COPY_BYTES / 1024.0
    _write_counter_csv(tmp_path / "cf", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2)])
    _write_counter_csv(tmp_path / "cw", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", kib)])
    _write_counter_csv(tmp_path / "f", [(1, "k_fwd<16, 32, 4, 0>", "FETCH_SIZE", 1000.0),
                                        (2, "k_fwd<16, 32, 4, 0>", "FETCH_SIZE", 3000.0),
                                        (3, "k_bin_reduce<true>", "FETCH_SIZE", 100.0),
                                        (4, "k_bin_combine", "FETCH_SIZE", 50.0),
                                        (5, "k_rays", "FETCH_SIZE", 7.0),
                                        (6, "k_enc<16, 0>", "FETCH_SIZE", 400.0)])
    _write_counter_csv(tmp_path / "w", [(1, "void nic::k_fwd<16, 32, 4, 0>(nic::FwdArgs)", "WRITE_SIZE", 10.0),
                                        (3, "k_bin_reduce<true>", "WRITE_SIZE", 20.0)])
    out = tmp_path / "traffic.json"
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                      "ct256", 0, out_json=str(out))
    t = json.load(open(out))
    assert t["source_sha"] == bench.kernel_source_sha()
    assert t["copy_scale"]["fetch"] == pytest.approx(2.0) and t["copy_scale"]["write"] == pytest.approx(1.0)
    k = t["workloads"]["ct256:p0"]
    assert k["forward"]["read"] == pytest.approx(2000.0 * 1024 * 2)     # mean of two dispatches x 2
    assert k["forward"]["write"] == pytest.approx(10.0 * 1024)
    assert k["bin_reduce"]["read"] == pytest.approx(150.0 * 1024 * 2)
    assert k["bin_reduce"]["bytes_per_launch"] == pytest.approx(150.0 * 1024 * 2 + 20.0 * 1024)
    assert "rays" not in k
    assert k["encode"]["read"] == pytest.approx(400.0 * 1024 * 2)
    assert "| `k_fwd<16, 32, 4, 0>` |" in capsys.readouterr().out


def test_achievable_fractions():
    kt = {"encode": (2.0, 10), "forward": (0.5, 10), "backward": (3.0, 10), "bin_reduce": (2.0, 10),
          "adam": (0.0, 0)}
    ab = {"encode": 4e8, "forward": 5e7, "backward": 4e8, "bin_reduce": 7e8}
    ceil = {"encode_fp32": {"value": 100.0, "unit": "us"}, "stream_copy": {"value": 5000.0, "unit": "GB/s"}}
    a = bench.achievable(kt, ab, ceil, {"backward": None, "bin_reduce": None}, 0, "ct256")
    assert a["encode"]["frac"] == pytest.approx(100.0 / 200.0)
    t = 0.3e-3 + 0.2e-3
    assert a["scatter"]["frac"] == pytest.approx(1.1e9 / t / 1e9 / 5000.0)
    assert "measured_frac" not in a["scatter"]
    assert "encode" not in bench.achievable(kt, ab, ceil, {}, 0, "tiny64")
