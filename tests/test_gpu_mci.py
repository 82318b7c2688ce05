"""Mapping Consistency Initialization on the GPU: the voxel-loss pre-training step (Eq. 2) over
several hash tables with one shared LayerNorm + MLP, the LN + MLP blob transfer, and PSNR, against the
FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_19742_amd import nic, synth  # noqa: E402

pytestmark = pytest.mark.gpu

FWD_TOL = 1e-5
GRAD_TOL = 1e-4


def rel(gpu, ora):
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    s = np.abs(ora).max()
    return float(np.abs(gpu - ora).max() / (s if s > 0 else 1.0))


def _model(ora, K, seed=5, **over):
    w = synth.WORKLOADS["tiny64"]
    cfg = nic.config_for(w, n_tables=K, seed=seed, **over)
    g = synth.cone_geometry(64, 50)
    oc = ora.Config(n_levels=cfg.n_levels, feats=2, log2_table=cfg.log2_table, base_res=cfg.base_res,
                    max_res=cfg.max_res, depth=cfg.mlp_depth, width=cfg.mlp_width)
    print(f"[case] K={K} {over} creating model", flush=True)
    return cfg, oc, nic.Model(cfg, g)


def _smooth_volumes(K, n, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*(np.linspace(0, 1, n),) * 3, indexing="ij")
    vols = []
    for _ in range(K):
        a = rng.uniform(0.5, 2.0, 3)
        vols.append(0.02 + 0.015 * np.sin(a[0] * 3 * x) * np.cos(a[1] * 3 * y) + 0.01 * z * a[2])
    return np.stack(vols).astype(np.float32)


def _flat(m, K, nt1):
    """[K tables | dense] float64 from the model's params-shaped tensor."""
    return m.flat(m.tensors()[0])


def test_voxel_step_matches_oracle(ora):
    K = 3
    cfg, oc, m = _model(ora, K)
    tot, nt1, nd = ora.n_params(oc)
    lay = m.layout
    assert lay["n_table"] == K * nt1
    rng = np.random.default_rng(60)
    table = rng.standard_normal(K * nt1) * 0.05
    dense = ora.init_params(oc, 61)[nt1:]
    p = np.concatenate([table, dense]).astype(np.float32).astype(np.float64)
    m.load_params(p)
    vols = _smooth_volumes(K, 24, 62)
    m.set_volumes(torch.tensor(vols, device="cuda"))
    B = 32 * K * 20
    x = rng.random((B, 3)).astype(np.float32)
    tid = np.arange(B) // (B // K)
    loss = torch.zeros(1, device="cuda")
    for t in m.tensors()[1:4]:
        t.zero_()
    t0 = m.get_step()
    m.voxel_step(B, torch.tensor(x, device="cuda"), loss)
    ol, _, og = ora.voxel_batch(oc, p, vols, x, tid)
    op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
    ora.adam(op, og, om, ov, t0 + 1)
    assert abs(loss.item() - ol) <= FWD_TOL * ol
    got = m.flat(m.tensors()[0])
    assert rel(got[:K * nt1], op[:K * nt1]) <= GRAD_TOL
    assert rel(got[K * nt1:], op[K * nt1:]) <= GRAD_TOL
    m.close()


def test_voxel_step_wide_bins_matches_oracle(ora):
    """256^3-workload tables at width 64, as many as it takes (the fewest of 4, 8, 12, 16) for the
    per-bin counts to need bins wider than the bin reduction's 2^13-entry LDS tile, so each bin is
    reduced tile by tile."""
    w = synth.WORKLOADS["ct256"]
    for K in (4, 8, 12, 16):
        cfg = nic.config_for(w, n_tables=K, mlp_width=64, seed=11)
        lay = nic.nic_describe(cfg)
        if lay["bin_shift"] > 13:
            break
    assert lay["bin_shift"] > 13
    oc = ora.Config(n_levels=cfg.n_levels, feats=2, log2_table=cfg.log2_table, base_res=cfg.base_res,
                    max_res=cfg.max_res, depth=cfg.mlp_depth, width=cfg.mlp_width)
    print(f"[case] K={K} W=64 bin_shift={lay['bin_shift']} creating model", flush=True)
    m = nic.Model(cfg, synth.cone_geometry(64, 4))
    tot, nt1, nd = ora.n_params(oc)
    rng = np.random.default_rng(70)
    table = (rng.standard_normal(K * nt1) * 0.05).astype(np.float32).astype(np.float64)
    dense = ora.init_params(oc, 71)[nt1:].astype(np.float32).astype(np.float64)
    p = np.concatenate([table, dense])
    m.load_params(p)
    vols = _smooth_volumes(K, 24, 72)
    m.set_volumes(torch.tensor(vols, device="cuda"))
    B = 32 * K * 16
    x = rng.random((B, 3)).astype(np.float32)
    tid = np.arange(B) // (B // K)
    loss = torch.zeros(1, device="cuda")
    for t in m.tensors()[1:4]:
        t.zero_()
    m.voxel_step(B, torch.tensor(x, device="cuda"), loss)
    ol, _, og = ora.voxel_batch(oc, p, vols, x, tid)
    op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
    ora.adam(op, og, om, ov, 1)
    assert abs(loss.item() - ol) <= FWD_TOL * ol
    got = m.flat(m.tensors()[0])
    assert rel(got[:K * nt1], op[:K * nt1]) <= GRAD_TOL
    assert rel(got[K * nt1:], op[K * nt1:]) <= GRAD_TOL
    # every touched entry moved, every untouched entry stayed
    touched = og[:K * nt1] != 0
    assert np.array_equal(got[:K * nt1][~touched], p[:K * nt1][~touched])
    assert np.mean(got[:K * nt1][touched] != p[:K * nt1][touched]) > 0.999
    m.close()


def test_voxel_train_with_device_points_matches_oracle(ora):
    """Points drawn on the device from Philox against the oracle's own draw."""
    K = 2
    cfg, oc, m = _model(ora, K, seed=9)
    tot, nt1, nd = ora.n_params(oc)
    vols = _smooth_volumes(K, 16, 63)
    m.set_volumes(torch.tensor(vols, device="cuda"))
    p = m.flat(m.tensors()[0])
    B = 32 * K * 8
    losses = m.voxel_train(3, B)
    op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
    tid = np.arange(B) // (B // K)
    for t in range(3):
        x = ora.voxel_points(cfg.seed, t, B)
        ol, _, og = ora.voxel_batch(oc, op, vols, x, tid)
        assert abs(losses[t] - ol) <= FWD_TOL * ol
        ora.adam(op, og, om, ov, t + 1)
    assert rel(m.flat(m.tensors()[0]), op) <= GRAD_TOL
    m.close()


def test_mlp_blob_roundtrip_and_transfer(ora):
    cfg, oc, a = _model(ora, 1, seed=1)
    _, _, b = _model(ora, 1, seed=2)
    blob = a.export_mlp()
    nt, nd, do = a.n_params()
    assert len(blob) >= 4 * nd
    b.tensors()[2].fill_(1.0)
    b.tensors()[3].fill_(1.0)
    b.import_mlp(blob)
    pa, pb = a.tensors()[0], b.tensors()[0]
    assert torch.equal(pa[do:do + nd], pb[do:do + nd])          # bitwise
    assert not torch.equal(pa[:nt], pb[:nt])                    # the table is not transferred
    assert float(b.tensors()[2][do:do + nd].abs().max()) == 0.0  # Adam state of LN + MLP reset
    assert float(b.tensors()[2][:nt].min()) == 1.0               # table moments untouched
    assert b.export_mlp() == blob
    # same table + imported network -> same field, bit for bit
    pb[:nt].copy_(pa[:nt])
    x = torch.rand(1000, 3, device="cuda")
    assert torch.equal(a.query(x), b.query(x))
    # a network of another shape is refused
    _, _, c = _model(ora, 1, seed=3, mlp_depth=2)
    with pytest.raises(nic.NicError) as ei:
        c.import_mlp(blob)
    assert ei.value.status == nic.NIC_EVERSION
    with pytest.raises(nic.NicError):
        c.import_mlp(b"NICX" + blob[4:])
    for mm in (a, b, c):
        mm.close()


def test_ssim_matches_oracle(ora):
    cfg, oc, m = _model(ora, 1)
    rng = np.random.default_rng(65)
    z, y, x = np.meshgrid(np.arange(21), np.arange(18), np.arange(25), indexing="ij")
    gt = (0.02 + 0.01 * np.sin(x / 3.0) * np.cos(y / 5.0) + 0.004 * z / 21).astype(np.float32)
    pred = (gt + 2e-3 * rng.standard_normal(gt.shape)).astype(np.float32)
    tg, tp = torch.tensor(gt, device="cuda"), torch.tensor(pred, device="cuda")
    v = m.ssim(tg, tp)
    assert abs(v - ora.ssim(gt, pred)) <= 1e-12
    assert abs(m.ssim(tg, tg) - 1.0) <= 1e-12
    with pytest.raises(nic.NicError):
        m.ssim(tg[:, :8].contiguous(), tp[:, :8].contiguous())
    m.close()


def test_psnr_matches_oracle(ora):
    cfg, oc, m = _model(ora, 1)
    rng = np.random.default_rng(64)
    gt = (rng.random((33, 20, 17)) * 0.05).astype(np.float32)
    pred = (gt + rng.standard_normal(gt.shape) * 1e-3).astype(np.float32)
    v = m.psnr(torch.tensor(gt, device="cuda"), torch.tensor(pred, device="cuda"))
    assert abs(v - ora.psnr(gt, pred)) <= 1e-9 * abs(v)
    assert m.psnr(torch.tensor(gt, device="cuda"), torch.tensor(gt, device="cuda")) == float("inf")
    m.close()


def test_mci_initialisation_speeds_convergence():
    """What the pre-trained network gains: LN + MLP pre-trained (Eq. 2) on the method's own
    reconstructions of four phantoms, then loaded into reconstructions of three other phantoms, reach a
    higher PSNR over the first 400 steps than the same reconstructions from random initialisation."""
    from paper_2506_19742_amd import mci
    base = synth.WORKLOADS["ct256"]

    def cfg(seed):
        return nic.config_for(base, mlp_width=64, mlp_depth=4, precision=0, seed=seed)

    vols = []
    for s in range(1000, 1004):
        ph, g, A, gt = mci.scan_workload(128, 20, s, 50, 128, 1e5)
        print(f"[case] pre-training reconstruction, phantom {s}", flush=True)
        r = mci.reconstruct(cfg(s), g, A, gt, 1500, 1500)
        vols.append(r["model"].render_volume(128, 128, 128).cpu().numpy())
        r["model"].close()
    blob, info = mci.pretrain(cfg(99), np.stack(vols).astype(np.float32), 1000, 1 << 18)
    assert info["loss_last"] < info["loss_first"]
    gains = []
    for s in range(2000, 2003):
        ph, g, A, gt = mci.scan_workload(128, 20, s, 50, 128, 1e5)
        print(f"[case] held-out phantom {s}", flush=True)
        curves = {}
        for arm, b in (("random", None), ("mci", blob)):
            r = mci.reconstruct(cfg(3000 + s), g, A, gt, 400, 100, blob=b)
            r["model"].close()
            curves[arm] = [p for _, _, p in r["curve"]]
        print(f"  random {np.round(curves['random'], 2)}  mci {np.round(curves['mci'], 2)}", flush=True)
        gains.append(np.mean(curves["mci"]) - np.mean(curves["random"]))
    print(f"mean PSNR gain over the first 400 steps: {np.round(gains, 2)} dB", flush=True)
    assert np.mean(gains) >= 1.0
