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
    FP16 table of the precision form; the level-major encoder kernel); the forward kernel then reads
    the encoding (L x F x 4 B per point: the network's input, not bytes of the method, which would
    keep it in registers); the scatter-add carries 8 x F FP32 gradients per level and point back
    (backward writes them as records, the bin reduction folds them into the table gradient); dense
    Adam reads p, g, m, v and writes p, m, v, g (32 B per parameter).  When the training step runs
    Adam inside the bin reduction (fused_adam), that kernel also reads and writes each table
    parameter with its two moments (24 B, plus 2 B for the FP16 copy)."""
    L, F = cfg.n_levels, cfg.feats_per_level
    payload = L * 8 * F * 4
    gather = L * 8 * F * (2 if cfg.precision else 4)
    table_adam = lay["n_table"] * (24 + (2 if cfg.precision else 0)) if fused_adam else 0
    return {
        "encode": n_points * gather,
        "forward": n_points * L * F * 4,
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


def ceilings(quick: bool = True) -> dict:
    """Memory ceilings measured now by nic_ubench (a child process, run before this process touches
    the GPU): stream copy / read / write in GB/s and the encode-pattern gathers of the 256^3
    workload in microseconds per step ({} when the program is missing or fails)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2506_19742_amd", "nic_ubench")
    if not os.path.exists(exe):
        return {}
    r = subprocess.run([exe, "--quick"] if quick else [exe], capture_output=True, text=True, timeout=120)
    out = {}
    for line in r.stdout.splitlines():
        f = line.split()
        if len(f) == 4 and f[0] == "ceiling":
            out[f[1]] = {"value": float(f[2]), "unit": f[3]}
    return out if r.returncode == 0 else {}


def achievable(kt, ab, ceil, traffic, precision, workload):
    """The encode and scatter sides against ceilings measured on this GPU: the level-major encoder
    kernel against its gathers and encoding store alone (encode-pattern microbenchmark, same
    placement of levels on XCDs, table and rays; only for the 256^3 workload it reproduces), and the
    scatter side (backward kernel's records + the bin reduction with the fused table Adam) against
    the stream-copy rate, by algorithmic bytes and, where the counters match these kernel sources,
    by measured traffic."""
    res = {"bar": 0.5}
    if not ceil:
        return res
    enc = ceil.get("encode_fp16" if precision else "encode_fp32")
    if enc and workload == "ct256" and kt["encode"][1]:
        t_enc = kt["encode"][0] / kt["encode"][1] * 1e3
        res["encode"] = {"kernel": "encode", "avg_us": t_enc, "gathers_alone_us": enc["value"],
                         "frac": enc["value"] / t_enc}
    copy = ceil.get("stream_copy")
    if copy and kt["backward"][1] and kt["bin_reduce"][1]:
        t = (kt["backward"][0] / kt["backward"][1] + kt["bin_reduce"][0] / kt["bin_reduce"][1]) / 1e3
        algo = ab["backward"] + ab["bin_reduce"]
        r = {"kernels": "backward + bin_reduce", "avg_us": t * 1e6, "stream_copy_GBs": copy["value"],
             "algorithmic_bytes": algo, "algorithmic_GBs": algo / t / 1e9,
             "frac": algo / t / 1e9 / copy["value"]}
        if traffic.get("backward") and traffic.get("bin_reduce"):
            mt = traffic["backward"] + traffic["bin_reduce"]
            r.update({"measured_bytes": mt, "measured_GBs": mt / t / 1e9,
                      "measured_frac": mt / t / 1e9 / copy["value"]})
        res["scatter"] = r
    return res


def timed_steps(model, steps: int) -> None:
    """steps training steps with HIP events around every kernel of every TIMING_EVERY-th step: each
    event costs a few us of stream time, so bracketing every step would slow the step it measures by
    about 4 %.  The steps in between run as one training call, as a caller training for many steps
    would (within a call each step's combine kernel draws the next step's rays)."""
    i = 0
    while i < steps:
        model.set_timing(True)
        model.train(1, want_loss=False)
        i += 1
        n = min(TIMING_EVERY - 1, steps - i)
        if n > 0:
            model.set_timing(False)
            model.train(n, want_loss=False)
            i += n


KERNEL_KIND = (("k_enc", "encode"), ("k_fwd", "forward"), ("k_bwd", "backward"), ("k_bin_reduce", "bin_reduce"),
               ("k_bin_combine", "bin_reduce"), ("k_adam", "adam"))


def _short(name: str) -> str:
    """Kernel name without return type, namespace and parameter list: k_bwd<16, 32, 4, 0>."""
    import re
    name = re.sub(r"^void\s+", "", name.strip())
    name = re.sub(r"^nic::", "", name)
    depth, out = 0, []
    for ch in name:                      # cut at the parameter list (outside template brackets)
        if ch == "(" and depth == 0:
            break
        depth += (ch == "<") - (ch == ">")
        out.append(ch)
    return "".join(out)


def _csv_rows(d: str, suffix: str):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        sys.exit(f"no *{suffix} under {d}")
    for f in files:
        yield from csv.DictReader(open(f, newline=""))


def _per_kernel_counter(d: str, counter: str) -> dict:
    """Mean of a rocprofv3 counter (summed over the rows of one dispatch) per kernel name."""
    per_dispatch = {}
    for row in _csv_rows(d, "counter_collection.csv"):
        if row.get("Counter_Name") != counter:
            continue
        key = (row.get("Dispatch_Id"), _short(row.get("Kernel_Name", "")))
        per_dispatch[key] = per_dispatch.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (_, name), v in per_dispatch.items():
        out.setdefault(name, []).append(v)
    return {k: sum(v) / len(v) for k, v in out.items()}


def pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, precision,
                out_json=TRAFFIC_JSON):
    """HBM bytes per launch from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per
    dispatch), each scaled by what the same counter reads for the plain copy of COPY_BYTES that
    --copy-calibration launches; per kernel kind (k_bin_reduce + k_bin_combine = bin_reduce) into
    profiles/traffic.json under the current kernel-source hash, and a Markdown table on stdout."""
    f, wr = _per_kernel_counter(fetch_dir, "FETCH_SIZE"), _per_kernel_counter(write_dir, "WRITE_SIZE")
    cf, cw = _per_kernel_counter(copy_fetch_dir, "FETCH_SIZE"), _per_kernel_counter(copy_write_dir, "WRITE_SIZE")
    ck = next(k for k in cf if "copyBuffer" in k)
    sf, sw = COPY_BYTES / (cf[ck] * 1024.0), COPY_BYTES / (cw[ck] * 1024.0)
    sha = kernel_source_sha()
    try:
        t = json.load(open(out_json))
    except (OSError, ValueError):
        t = {}
    if t.get("source_sha") != sha:
        t = {"source_sha": sha, "workloads": {}}
    t["copy_scale"] = {"fetch": sf, "write": sw, "copy_kernel": ck}
    kinds = {}
    for name in sorted(set(f) | set(wr)):
        kind = next((k for p, k in KERNEL_KIND if name.startswith(p)), None)
        if kind is None:
            continue
        r, w_ = f.get(name, 0.0) * 1024.0 * sf, wr.get(name, 0.0) * 1024.0 * sw
        e = kinds.setdefault(kind, {"bytes_per_launch": 0.0, "read": 0.0, "write": 0.0})
        e["read"] += r
        e["write"] += w_
        e["bytes_per_launch"] += r + w_
    t["workloads"][f"{workload}:p{precision}"] = kinds
    json.dump(t, open(out_json, "w"), indent=1)
    print(f"Counter scale from a plain copy of {COPY_BYTES >> 20} MiB (`{ck}`): FETCH_SIZE x {sf:.3f}, "
          f"WRITE_SIZE x {sw:.3f} (KiB -> bytes included).\n")
    print("| kernel | read MB/launch | write MB/launch |\n|---|---|---|")
    for name in sorted(set(f) | set(wr)):
        print(f"| `{name}` | {f.get(name, 0.0) * 1.024e-3 * sf:.1f} | {wr.get(name, 0.0) * 1.024e-3 * sw:.1f} |")
    print(f"\nKernel sources sha256[:16] at measurement: `{sha}`.")


SQ_PASSES = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY "
             "SQ_ACTIVE_INST_VALU SQ_VALU_MFMA_BUSY_CYCLES",
             "SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAIT_INST_LDS SQ_LDS_BANK_CONFLICT "
             "SQ_INSTS_SALU SQ_ACTIVE_INST_LDS")


def sq_summary(dir_a: str, dir_b: str, stats_dir: str, n_cu: int = 256, clock_ghz: float = 2.4):
    """Markdown tables of two rocprofv3 --pmc passes of SQ counters (SQ_PASSES), averaged per kernel
    launch: instructions per wave, the share of the waves' lifetime spent issuing, in s_waitcnt and
    waiting for an issue slot or a dependency, and the matrix cores' busy share (MFMA busy cycles
    over 4 SIMDs x n_cu x the kernel's average duration from the --stats run in stats_dir)."""
    names = [c for p in SQ_PASSES for c in p.split()]
    per = {}
    for d, p in ((dir_a, SQ_PASSES[0]), (dir_b, SQ_PASSES[1])):
        for c in p.split():
            for k, v in _per_kernel_counter(d, c).items():
                per.setdefault(k, {})[c] = v
    dur = {_short(r["Name"]): float(r["AverageNs"]) for r in _csv_rows(stats_dir, "kernel_stats.csv")}
    keep = [k for k in per if k.startswith(("k_enc", "k_fwd", "k_bwd", "k_bin_reduce", "k_bin_combine", "k_adam"))]
    print("| kernel | waves | VALU instr / wave | LDS instr / wave | VMEM rd / wr per wave | issuing | s_waitcnt | "
          "waiting to issue | matrix cores busy |\n|---|---|---|---|---|---|---|---|---|")
    for k in sorted(keep):
        c = per[k]
        w, cyc = c.get("SQ_WAVES", 0.0) or 1.0, c.get("SQ_WAVE_CYCLES", 0.0) or 1.0
        mf = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (4 * n_cu * dur.get(k, float("nan")) * clock_ghz)
        print(f"| `{k}` | {w:.0f} | {c.get('SQ_INSTS_VALU', 0) / w:.0f} | {c.get('SQ_INSTS_LDS', 0) / w:.0f} | "
              f"{c.get('SQ_INSTS_VMEM_RD', 0) / w:.0f} / {c.get('SQ_INSTS_VMEM_WR', 0) / w:.0f} | "
              f"{100 * c.get('SQ_ACTIVE_INST_ANY', 0) / cyc:.0f}% | {100 * c.get('SQ_WAIT_ANY', 0) / cyc:.0f}% | "
              f"{100 * c.get('SQ_WAIT_INST_ANY', 0) / cyc:.0f}% | {100 * mf:.0f}% |")
    print("\nRaw averages:\n\n| kernel | counter | value |\n|---|---|---|")
    for k in sorted(keep):
        for c in names:
            if c in per[k]:
                print(f"| `{k}` | {c} | {per[k][c]:.4g} |")
    print(f"\nKernel sources sha256[:16] at measurement: `{kernel_source_sha()}`.")


def stats_summary(d: str):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    rows = list(_csv_rows(d, "kernel_stats.csv"))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | avg µs | % of GPU time |\n|---|---|---|---|")
    for r in rows:
        print(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    print(f"\nKernel sources sha256[:16] at measurement: `{kernel_source_sha()}`.")


def converge(n_pre: int = 16, n_heldout: int = 8, cap: int = 3000, eval_every: int = 50, target: float = 30.0,
             log=None) -> dict:
    """Seconds (and steps) to 30 dB PSNR on held-out 256^3 phantoms, BF16 form + Mapping Consistency
    Initialization against plain FP32 with random initialisation (Sec. 2.4, Eq. 2; Sec. 3.1), every
    compute step in libnic's kernels: (1) the method's own FP32 reconstructions of n_pre 128^3
    phantoms (seeds 1000 + i, 20 ellipsoids, 50 views on a 128 x 128 detector, Poisson I0 = 1e5,
    3000 steps each); (2) voxel-loss pre-training of one LayerNorm + MLP 4 x 64 over their n_pre
    tables (2000 steps x 2^18 points); (3) held-out phantoms 2000 + i (the 256^3 benchmark scan
    recipe), MLP 4 x 64 in both arms, PSNR of the full 256^3 render every eval_every steps; the
    clock is cumulative training-step time (evaluation excluded); an arm stops at the first check at
    or above the target, or at cap steps."""
    import torch
    from paper_2506_19742_amd import mci, nic, synth
    base = synth.WORKLOADS["ct256"]

    def cfg_for(prec, seed):
        return nic.config_for(base, mlp_width=64, mlp_depth=4, precision=prec, seed=seed)

    t0 = time.perf_counter()
    vols, t_rec = [], 0.0
    for i in range(n_pre):
        _, g, A, gt = mci.scan_workload(128, 20, 1000 + i, 50, 128, 1e5)
        r = mci.reconstruct(cfg_for(0, 1000 + i), g, A, gt, 3000, 3000, target)
        t_rec += r["curve"][-1][1]
        vols.append(r["model"].render_volume(128, 128, 128).cpu().numpy())
        r["model"].close()
        if log:
            log(f"[bench] converge: pre-training reconstruction {i + 1}/{n_pre}, PSNR {r['curve'][-1][2]:.2f} dB")
    blob, info = mci.pretrain(cfg_for(0, 99), np.stack(vols).astype(np.float32), 2000, 1 << 18)
    del vols
    torch.cuda.empty_cache()
    arms = {"fp32_random": (0, None), "bf16_mci": (1, blob)}
    per = {}
    for i in range(n_heldout):
        seed = 2000 + i
        _, g, A, gt = mci.scan_workload(256, 20, seed, 50, 256, 1e5)
        for arm, (prec, b) in arms.items():
            r = mci.reconstruct(cfg_for(prec, 3000 + i), g, A, gt, cap, eval_every, target, blob=b,
                                stop_at_target=True)
            r["model"].close()
            best = max(p for _, _, p in r["curve"])
            per.setdefault(str(seed), {})[arm] = {
                "steps": r["hit"][0] if r["hit"] else None, "seconds": r["hit"][1] if r["hit"] else None,
                "best_psnr_db": best, "steps_run": r["curve"][-1][0]}
            if log:
                log(f"[bench] converge: phantom {seed} {arm}: {per[str(seed)][arm]}")
    summary = {}
    for arm in arms:
        hits = [per[s][arm] for s in per if per[s][arm]["seconds"] is not None]
        summary[arm] = {"reached": f"{len(hits)}/{len(per)}",
                        "median_steps": float(np.median([h["steps"] for h in hits])) if hits else None,
                        "median_seconds": float(np.median([h["seconds"] for h in hits])) if hits else None,
                        "mean_seconds": float(np.mean([h["seconds"] for h in hits])) if hits else None}
    a, b_ = summary["fp32_random"]["median_seconds"], summary["bf16_mci"]["median_seconds"]
    return {"target_db": target, "metric": "seconds of training steps to reach the target PSNR (full 256^3 render)",
            "arms": summary, "speedup_bf16_mci_vs_fp32": (a / b_) if a and b_ else None, "per_phantom": per,
            "protocol": f"MCI pre-trained on the method's own 128^3 reconstructions of {n_pre} phantoms "
                        f"(seeds 1000-{999 + n_pre}, 3000 steps each, {t_rec:.1f} s) + 2000 voxel-loss steps x 2^18 "
                        f"points ({info['seconds']:.1f} s); held-out phantoms 2000-{1999 + n_heldout} at 256^3, "
                        f"MLP 4x64, PSNR every {eval_every} steps, cap {cap} steps",
            "pretraining_seconds": t_rec + info["seconds"], "wall_seconds": time.perf_counter() - t0}


def small(steps: int = 200, warmup: int = 20) -> dict:
    """The 64^3 workload (6 ellipsoids, 50 views on a 64 x 64 detector, 8 levels, T = 2^14, MLP 3 x 32,
    1024 rays x 64 samples; its table is L2-resident), FP32 and precision form: full-step pts/s."""
    import torch
    from paper_2506_19742_amd import nic, synth
    w = synth.WORKLOADS["tiny64"]
    _, g, A = synth.scan(w)
    out = {"workload": f"{w.name}: {w.grid}^3 phantom of {w.n_ellipsoids} ellipsoids, {w.n_views} views on "
                       f"{w.n_det}x{w.n_det} detector, L={w.n_levels}, T=2^{w.log2_table}, MLP {w.depth}x{w.width}, "
                       f"{w.rays} rays x {w.samples} samples"}
    for prec in (0, 1):
        model = nic.Model(nic.config_for(w, seed=2024, precision=prec), g)
        model.set_projections(torch.tensor(A, device="cuda:0"))
        model.train(warmup, want_loss=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model.train(steps, want_loss=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        model.close()
        out["fp32" if prec == 0 else "precision_form"] = {"ms_per_step": dt * 1e3 / steps,
                                                          "train_pts_per_s": w.rays * w.samples * steps / dt}
    return out


def large(steps: int = 50, warmup: int = 10, log=None) -> dict:
    """The largest workload on one GPU: 512^3 phantom of 40 ellipsoids, 100 views on a 512 x 512
    detector (Poisson I0 = 1e5), 16 levels x 2 features, T = 2^21, MLP 4 x 32, 320 samples per ray,
    8192 rays per step, precision form (BF16 MLP, FP16 table, FP32 master weights and Adam):
    training pts/s over `steps` full steps, and forward-only inference of the full 512^3 volume."""
    import torch
    from paper_2506_19742_amd import nic, synth
    w = synth.WORKLOADS["ct512"]
    cfg = nic.config_for(w, seed=2024)
    if log:
        log("[bench] large: generating the 512^3 scan")
    _, g, A = synth.scan(w)
    model = nic.Model(cfg, g)
    model.set_projections(torch.tensor(A, device="cuda:0"))
    del A
    model.train(warmup, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed_steps(model, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = model.kernel_times()
    model.set_timing(False)
    loss = float(model.train(1)[-1])
    n = w.grid
    vol = model.render_volume(n, n, n)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        vol = model.render_volume(n, n, n)
    torch.cuda.synchronize()
    rs = (time.perf_counter() - t1) / 3
    finite = bool(torch.isfinite(vol).all())
    del vol
    model.close()
    P = w.rays * w.samples
    return {"workload": f"{w.name}: {n}^3 phantom of {w.n_ellipsoids} ellipsoids, {w.n_views} views on "
                        f"{w.n_det}x{w.n_det} detector, Poisson I0={w.noise_i0:g}, T=2^{w.log2_table}, "
                        f"{w.samples} samples x {w.rays} rays, precision form",
            "train_pts_per_s": P * steps / dt, "ms_per_step": dt * 1e3 / steps, "steps": steps,
            "points_per_step": P, "final_loss": loss,
            "kernels_avg_ms": {k: (ms / c if c else None) for k, (ms, c) in kt.items()},
            "render": {"n": n, "points": n ** 3, "seconds": rs, "pts_per_s": n ** 3 / rs, "finite": finite}}


def cpu_info() -> dict:
    """CPU model and core counts of this host (threads the oracle may use: the affinity set, at
    most 16, the CPU share of one GPU on a shared box)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": aff, "threads": max(1, min(16, aff))}


def cpu_baseline(w, g, A, n_rays_one_core=512):
    """FP64 oracle as it stands, on the host cores: (1) all cores (the oracle splits the rays over
    threads with per-thread gradient buffers): one full step of R rays forward + backward plus one
    dense Adam over all parameters; (2) one core on a bounded sample of n_rays_one_core rays, scaled
    to the step.  value = the all-cores rate."""
    import oracle as ora
    ora.build(force=False)
    from paper_2506_19742_amd import synth
    info = cpu_info()
    oc = ora.Config(w.n_levels, w.feats, w.log2_table, w.base_res, w.max_res, w.depth, w.width)
    tot, nt, nd = ora.n_params(oc)
    p = ora.init_params(oc, 1)
    pix, jit = synth.ray_batch(3, g.n_pix, w.rays, w.samples)
    m, v = np.zeros(tot), np.zeros(tot)
    t0 = time.perf_counter()
    ora.adam(p.copy(), np.zeros(tot), m, v, 1)
    t_adam = time.perf_counter() - t0
    legs = {}
    for leg, threads, R in (("all", info["threads"], w.rays), ("one", 1, n_rays_one_core)):
        ora.set_threads(threads)
        try:
            t0 = time.perf_counter()
            ora.ray_batch(oc, g, p, float(g.angles[0]), A[0], pix[:R], jit[:R])
            t_rays = time.perf_counter() - t0
        finally:
            ora.set_threads(1)
        step_s = t_rays * (w.rays / R) + t_adam
        legs[leg] = {"value": w.rays * w.samples / step_s, "cores": threads, "rays": R, "t_rays": t_rays,
                         "fwd_bwd_pts_per_s": R * w.samples / t_rays}
    allc, one = legs["all"], legs["one"]
    return {"value": allc["value"], "unit": "pts/s", "cores": allc["cores"], "kind": "oracle",
            "sample": f"{allc['cores']} threads: one full step, {w.rays} rays x {w.samples} samples fwd+bwd "
                      f"({allc['t_rays']:.1f} s) + one Adam over {tot} params ({t_adam:.2f} s); one core: "
                      f"{one['rays']} rays x {w.samples} samples ({one['t_rays']:.1f} s) scaled to {w.rays} rays/step",
            "fwd_bwd_pts_per_s": allc["fwd_bwd_pts_per_s"],
            "one_core": {"value": one["value"], "unit": "pts/s", "cores": 1,
                         "fwd_bwd_pts_per_s": one["fwd_bwd_pts_per_s"]},
            **info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ct256")
    ap.add_argument("--precision", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the seconds-to-30-dB comparison (BF16 + MCI against plain FP32)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of --steps steps each (no kernel events), reported beside the value")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 64^3 workload (FP32 and precision form)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the largest workload (512^3, precision form: training and full-volume inference)")
    ap.add_argument("--converge-pre", type=int, default=16, help="MCI pre-training phantoms")
    ap.add_argument("--converge-heldout", type=int, default=8, help="held-out phantoms per arm")
    ap.add_argument("--render", type=int, default=0,
                    help="also time forward-only inference of the full n^3 volume (voxel centres)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (counter calibration) and exit")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the live memory-ceiling measurement (nic_ubench --quick)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="summarise rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this workload and of "
                         "--copy-calibration into profiles/traffic.json (no GPU use) and exit")
    ap.add_argument("--sq-summary", nargs=3, metavar=("PASS_A_DIR", "PASS_B_DIR", "STATS_DIR"),
                    help="print the SQ counter tables of the two SQ_PASSES runs (kernel times from a --stats "
                         "run) and exit")
    ap.add_argument("--stats-summary", metavar="DIR",
                    help="print a Markdown table of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--ubench", action="store_true",
                    help="only run the memory-ceiling microbenchmark (nic_ubench, built by build()) and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.workload, 0 if args.precision is None else args.precision)
        return
    if args.stats_summary:
        stats_summary(args.stats_summary)
        return
    if args.sq_summary:
        sq_summary(*args.sq_summary)
        return
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

    ceil = {}
    if not args.no_ceilings:
        print("[bench] measuring memory ceilings (nic_ubench --quick)", file=sys.stderr, flush=True)
        ceil = ceilings()

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
    timed_steps(model, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = model.kernel_times()
    model.set_timing(False)
    repeats = []
    for _ in range(args.repeats):           # the same K steps again, no kernel events
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        model.train(args.steps, want_loss=False)
        torch.cuda.synchronize()
        repeats.append((time.perf_counter() - t1) * 1e3 / args.steps)
    losses = model.train(1)

    P = w.rays * w.samples
    value = P * args.steps / dt
    fused = kt["adam"][1] == 0
    ab = algorithmic_bytes(cfg, lay, P, fused_adam=fused)
    per_kernel = {k: {"avg_ms": (ms / n if n else None), "launches": n} for k, (ms, n) in kt.items()}
    dom = max((k for k in ("encode", "forward", "backward", "bin_reduce", "adam") if kt[k][1]),
              key=lambda k: kt[k][0])
    avg_s = kt[dom][0] / kt[dom][1] / 1e3
    achieved = ab[dom] / avg_s / 1e9
    n_timed = len(range(0, args.steps, TIMING_EVERY))
    kernel_ms = sum(kt[k][0] for k in kt) / n_timed
    ffwd, fbwd = mlp_flops_per_point(cfg)
    kernel_rooflines = {}
    for k in ("encode", "forward", "backward", "bin_reduce", "adam"):
        if not kt[k][1]:
            continue
        t = kt[k][0] / kt[k][1] / 1e3
        r = {"avg_ms": t * 1e3, "hbm_GBs": ab[k] / t / 1e9, "hbm_frac": ab[k] / t / 1e9 / HBM_PEAK_GBS,
             "measured_traffic_bytes": measured_traffic(k, w.name, cfg.precision)}
        if k in ("forward", "backward"):
            fl = P * (ffwd if k == "forward" else fbwd)
            r["mfma_TFLOPs"] = fl / t / 1e12
            r["mfma_frac"] = fl / t / 1e12 / MFMA_PEAK_TFLOPS[cfg.precision]
        # against the ceiling measured for the kernel's own access pattern on this GPU
        enc = ceil.get("encode_fp16" if cfg.precision else "encode_fp32")
        if k == "encode" and enc and w.name == "ct256":
            r["achievable_frac"] = enc["value"] / (t * 1e6)
            r["achievable_ceiling"] = "the same gathers and encoding store alone (encode microbenchmark), us per step"
        elif k == "backward" and "stream_write" in ceil:
            r["achievable_frac"] = ab[k] / t / 1e9 / ceil["stream_write"]["value"]
            r["achievable_ceiling"] = "stream write GB/s (the kernel writes the corner gradients)"
        elif k in ("bin_reduce", "adam") and "stream_copy" in ceil:
            r["achievable_frac"] = ab[k] / t / 1e9 / ceil["stream_copy"]["value"]
            r["achievable_ceiling"] = "stream copy GB/s (read + write)"
        kernel_rooflines[k] = r
    traffic = {k: measured_traffic(k, w.name, cfg.precision) for k in ("encode", "forward", "backward", "bin_reduce")}

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
        "repeats": {"ms_per_step": repeats, "median_ms": float(np.median(repeats)) if repeats else None,
                    "note": f"{len(repeats)} further runs of {args.steps} steps, no kernel events"},
        "kernel_rooflines": kernel_rooflines,
        "ceilings": ceil,
        "achievable": achievable(kt, ab, ceil, traffic, cfg.precision, w.name),
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
    model.close()
    if not args.no_small and w.name == "ct256":
        out["small"] = small()
    if not args.no_large and w.name == "ct256":
        out["large"] = large(log=lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_converge and w.name == "ct256":
        print("[bench] seconds to 30 dB: MCI pre-training, then held-out phantoms", file=sys.stderr, flush=True)
        out["converge"] = converge(args.converge_pre, args.converge_heldout,
                                   log=lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, g, A)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
