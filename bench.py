"""Throughput of the training step on one MI355X.

A step is one pass of the whole hot path over one batch: rays of one view -> samples -> hash encode
-> LayerNorm -> MLP -> ray sums (Eq. 1) -> L1 loss (Eq. 3) -> backward with table scatter-add ->
Adam on every parameter.  Workload: the 256^3 synthetic phantom (20 random ellipsoids), 50 cone-beam
views on a 256 x 256 detector with Poisson noise at I0 = 1e5, 16 levels x 2 features, T = 2^19,
base resolution 16 (max 2048), MLP 4 x 32, 192 samples per ray, 2048 rays per step, FP32.
Projections are resident in HBM before the timed region; every draw (view order, pixels, jitter)
happens on the device.

Prints one JSON line: value = sample points per second of full steps (rays * samples * steps /
seconds), roofline of the dominant kernel from HIP events on the library's stream, and the FP64
oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
TIMING_EVERY = 10   # timed steps per step whose kernels are bracketed by HIP events
sys.path.insert(0, ROOT)

METRIC = "train pts/s (fwd+bwd); secs to 30 dB PSNR, BF16+MCI vs plain FP32"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {0: 157.3, 1: 2500.0}   # dense FP32 / BF16 matrix cores, MI355X published figures
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
COPY_BYTES = 256 << 20


def kernel_source_sha() -> str:
    """Hash of the HIP sources of libnic (its .hip files and the headers): measured traffic is used
    only for the kernels it was taken on."""
    import hashlib
    from paper_2506_19742_amd import build as _build
    h = hashlib.sha256()
    for f in sorted(os.listdir(_build.CSRC)):
        if f.endswith(".h") or f in _build.SOURCES:
            h.update(open(os.path.join(_build.CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, precision: int):
    """HBM bytes per launch of `kernel` from profiles/traffic.json (rocprofv3 FETCH_SIZE and
    WRITE_SIZE passes scaled by the same counters on a plain copy of known size), or None when the
    file is absent, covers another workload, or was taken on other kernel sources."""
    try:
        import json as _json
        t = _json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    rec = t.get("workloads", {}).get(f"{workload}:p{precision}", {}).get(kernel)
    return None if rec is None else rec.get("bytes_per_launch")


def algorithmic_bytes(cfg, lay, n_points, fused_adam=False):
    """Bytes the method itself moves per launch (independent of this implementation), for the
    roofline: the encode gathers 8 corners x F features per level and point (4 B each, 2 B from the
    FP16 table of the precision form; forward); the scatter-add carries 8 x F FP32 gradients per
    level and point back (backward writes them as records, the bin reduction folds them into the
    table gradient); dense Adam reads p, g, m, v and writes p, m, v, g (32 B per parameter).  When the
    training step runs Adam inside the bin reduction (fused_adam), that kernel also reads and writes
    each table parameter with its two moments (24 B, plus 2 B for the FP16 copy)."""
    L, F = cfg.n_levels, cfg.feats_per_level
    payload = L * 8 * F * 4
    gather = L * 8 * F * (2 if cfg.precision else 4)
    table_adam = lay["n_table"] * (24 + (2 if cfg.precision else 0)) if fused_adam else 0
    return {
        "forward": n_points * gather,
        "backward": n_points * payload,
        "bin_reduce": n_points * payload + table_adam,
        "adam": lay["n_params_padded"] * 32,
        "per_point": payload,
    }


def mlp_flops_per_point(cfg):
    """Multiply-adds x 2 of LayerNorm-free network work per sample point: the forward pass
    (layer 0: C x W, hidden: (D-1) W x W, head W) and, in the backward kernel, its recomputation
    plus the data gradients (every layer's transposed product, layer 0 included for LayerNorm) and
    the weight gradients (one outer product per layer)."""
    C, W, D = 2 * cfg.n_levels, cfg.mlp_width, cfg.mlp_depth
    fwd = 2 * (C * W + (D - 1) * W * W + W)
    bwd = fwd + 2 * (C * W + (D - 1) * W * W + W) + 2 * (C * W + (D - 1) * W * W + W)
    return fwd, bwd


def cpu_baseline(w, g, A, n_rays_sample=1024):
    """FP64 oracle (single thread) on a bounded sample: n_rays_sample rays of one view forward +
    backward, plus one dense Adam over all parameters; scaled to the full step of R rays."""
    import oracle as ora
    ora.build(force=False)
    from paper_2506_19742_amd import synth
    oc = ora.Config(w.n_levels, w.feats, w.log2_table, w.base_res, w.max_res, w.depth, w.width)
    tot, nt, nd = ora.n_params(oc)
    p = ora.init_params(oc, 1)
    pix, jit = synth.ray_batch(3, g.n_pix, n_rays_sample, w.samples)
    t0 = time.perf_counter()
    _, _, grad = ora.ray_batch(oc, g, p, float(g.angles[0]), A[0], pix, jit)
    t_rays = time.perf_counter() - t0
    m, v = np.zeros(tot), np.zeros(tot)
    t0 = time.perf_counter()
    ora.adam(p, grad, m, v, 1)
    t_adam = time.perf_counter() - t0
    step_s = t_rays * (w.rays / n_rays_sample) + t_adam
    return {"value": w.rays * w.samples / step_s, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_rays_sample} rays x {w.samples} samples fwd+bwd ({t_rays:.1f} s) + one "
                      f"Adam over {tot} params ({t_adam:.2f} s), scaled to {w.rays} rays/step",
            "fwd_bwd_pts_per_s": n_rays_sample * w.samples / t_rays}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ct256")
    ap.add_argument("--precision", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--render", type=int, default=0,
                    help="also time forward-only inference of the full n^3 volume (voxel centres)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (counter calibration) and exit")
    ap.add_argument("--ubench", action="store_true",
                    help="only run the memory-ceiling microbenchmark (nic_ubench, built by build()) and exit")
    args = ap.parse_args()
    if args.ubench:
        import subprocess
        exe = os.path.join(ROOT, "paper_2506_19742_amd", "nic_ubench")
        if not os.path.exists(exe):
            sys.exit(f"{exe} is missing: run __graft_entry__.build() first")
        sys.exit(subprocess.run([exe]).returncode)
    if args.copy_calibration:
        import torch
        x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): it measures the "
              "training step on one GPU; sharding over several GPUs is a design, not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_19742_amd import nic, synth

    w = synth.WORKLOADS[args.workload]
    over = {} if args.precision is None else {"precision": args.precision}
    cfg = nic.config_for(w, seed=2024, **over)
    print(f"[bench] workload {w.name}: generating scan", file=sys.stderr, flush=True)
    ph, g, A = synth.scan(w)
    dev = torch.device("cuda:0")
    proj = torch.tensor(A, device=dev)
    model = nic.Model(cfg, g)
    model.set_projections(proj)
    lay = model.layout
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    model.train(args.warmup, want_loss=False)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        # HIP events around every kernel of every TIMING_EVERY-th step: each event costs a few us of
        # stream time, so bracketing every step would slow the step it measures by about 4 %
        model.set_timing(i % TIMING_EVERY == 0)
        model.train(1, want_loss=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = model.kernel_times()
    model.set_timing(False)
    losses = model.train(1)

    P = w.rays * w.samples
    value = P * args.steps / dt
    fused = kt["adam"][1] == 0
    ab = algorithmic_bytes(cfg, lay, P, fused_adam=fused)
    per_kernel = {k: {"avg_ms": (ms / n if n else None), "launches": n} for k, (ms, n) in kt.items()}
    dom = max((k for k in ("forward", "backward", "bin_reduce", "adam") if kt[k][1]), key=lambda k: kt[k][0])
    avg_s = kt[dom][0] / kt[dom][1] / 1e3
    achieved = ab[dom] / avg_s / 1e9
    n_timed = len(range(0, args.steps, TIMING_EVERY))
    kernel_ms = sum(kt[k][0] for k in kt) / n_timed
    ffwd, fbwd = mlp_flops_per_point(cfg)
    kernel_rooflines = {}
    for k in ("forward", "backward", "bin_reduce", "adam"):
        if not kt[k][1]:
            continue
        t = kt[k][0] / kt[k][1] / 1e3
        r = {"avg_ms": t * 1e3, "hbm_GBs": ab[k] / t / 1e9, "hbm_frac": ab[k] / t / 1e9 / HBM_PEAK_GBS,
             "measured_traffic_bytes": measured_traffic(k, w.name, cfg.precision)}
        if k in ("forward", "backward"):
            fl = P * (ffwd if k == "forward" else fbwd)
            r["mfma_TFLOPs"] = fl / t / 1e12
            r["mfma_frac"] = fl / t / 1e12 / MFMA_PEAK_TFLOPS[cfg.precision]
        kernel_rooflines[k] = r

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg.precision == 0 else "bf16/f16+f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.grid}^3 phantom of {w.n_ellipsoids} ellipsoids, "
                               f"{w.n_views} views on {w.n_det}x{w.n_det} detector, "
                               f"{'Poisson I0=%g' % w.noise_i0 if w.noise_i0 else 'noiseless'}",
                   "levels": w.n_levels, "feats": w.feats, "log2_table": w.log2_table,
                   "base_res": w.base_res, "max_res": w.max_res, "mlp": f"{w.depth}x{w.width}",
                   "samples_per_ray": w.samples, "rays_per_step": w.rays,
                   "points_per_step": P, "n_params": lay["n_table"] + lay["n_dense"],
                   "precision": cfg.precision},
        "adam": "fused into the reductions" if fused else "separate pass",
        "kernel_pts_per_s": P / (kernel_ms / 1e3),
        "kernels": per_kernel,
        "kernel_timing": f"HIP events around each kernel of every {TIMING_EVERY}th timed step",
        "final_loss": float(losses[-1]),
        "kernel_rooflines": kernel_rooflines,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, w.name, cfg.precision),
                     "algorithmic_bytes_per_launch": ab[dom]},
    }
    if args.render:
        n = args.render
        vol = model.render_volume(n, n, n)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            vol = model.render_volume(n, n, n)
        torch.cuda.synchronize()
        rs = (time.perf_counter() - t0) / reps
        out["render"] = {"n": n, "points": n ** 3, "seconds": rs, "pts_per_s": n ** 3 / rs}
        del vol
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, g, A)
    model.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
