"""The ray training step's level-major encoder against the forward kernel's own gathers.

A training step on rays computes the hash encoding (Sec. 2.2) in a kernel of its own, one level
per block with the blocks placed so that each XCD works on one level at a time, and counts the
table-gradient records there; the forward kernel then reads the stored encoding.  It runs the same
arithmetic in the same order as the forward kernel gathering every level itself, so the two
placements must give bitwise identical training: the losses of every step and, after the steps,
the parameters, gradient, both Adam moments and the FP16 table copy.  A record counted for the
wrong bin or block would move records between bins or leave slots stale, and show here.  Both
placements are forced here; the default picks the level-major one where it pays (the table larger
than an XCD's L2, each level's table at most twice it), which the last test checks for the three
workloads.

Cases: the three workloads at both precisions (8 levels: a single phase of levels; 16: two), small
tables whose gradient bins each hold eight levels, the 64-wide network, a
small batch whose last chunk is partial (97 rays x 32 samples over 25 backward blocks), a channel
mask that turns off a level pair and one level of another pair (the second level of that pair is
still gathered and scattered), and a detector shifted so that some rays miss the volume.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_19742_amd import nic, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _train_both(cfg, g, proj, steps, mask=None):
    """Losses of `steps` training steps, after checking both placements agree bit for bit."""
    runs = []
    for placement in ("level_major", "in_forward"):
        m = nic.Model(cfg, g)
        m.set_encoder_placement(placement)
        assert m.encoder_level_major() == (placement == "level_major")
        m.set_projections(proj)
        if mask is not None:
            m.set_channel_mask(mask)
        loss = m.train(steps)
        runs.append((loss, [None if t is None else t.clone() for t in m.tensors()]))
        m.close()
    (la, ta), (lb, tb) = runs
    assert np.array_equal(la, lb), (la, lb)
    for k, (x, y) in enumerate(zip(ta, tb)):
        assert (x is None) == (y is None), k
        if x is not None:
            assert torch.equal(x, y), k
    return la


@pytest.mark.parametrize("workload,precision", [("tiny64", 0), ("tiny64", 1), ("ct256", 0), ("ct256", 1),
                                                ("ct512", 0), ("ct512", 1)])
def test_level_major_encoder_is_bitwise_identical(workload, precision):
    print(f"[case] encoder placement {workload} precision {precision}", flush=True)
    w = synth.WORKLOADS[workload]
    if workload == "ct512":   # zero projections: generating the 100 views would take most of the test
        g = synth.cone_geometry(w.n_det, w.n_views)
        A = np.zeros((w.n_views, g.nv, g.nu), np.float32)
    else:
        _, g, A = synth.scan(w)
    loss = _train_both(nic.config_for(w, seed=51, precision=precision), g, torch.tensor(A, device="cuda"), 3)
    assert np.all(np.isfinite(loss))


@pytest.mark.parametrize("workload", ["tiny64", "ct256"])
def test_level_major_encoder_partial_chunk(workload):
    """97 rays x 32 samples = 3104 points: 24 full chunks of 128 and one of 32, 25 backward blocks."""
    print(f"[case] encoder placement {workload} partial chunk", flush=True)
    w = synth.WORKLOADS[workload]
    g = synth.cone_geometry(64, 8)
    ph = synth.make_phantom(2, 5)
    A = synth.project(ph, g).astype(np.float32)
    cfg = nic.config_for(w, seed=52, rays_per_step=97, samples_per_ray=32)
    _train_both(cfg, g, torch.tensor(A, device="cuda"), 4)


def test_level_major_encoder_channel_mask():
    print("[case] encoder placement tiny64 channel mask", flush=True)
    w = synth.WORKLOADS["tiny64"]
    _, g, A = synth.scan(w)
    C_ = 2 * w.n_levels
    mask = [1.0] * C_
    # levels 1 and 3 (a pair) off entirely; level 4 off, its pair partner level 6 on; one scaled channel
    for ch in (2, 3, 6, 7, 8, 9):
        mask[ch] = 0.0
    mask[C_ - 1] = 0.5
    _train_both(nic.config_for(w, seed=53), g, torch.tensor(A, device="cuda"), 3, mask=mask)


def test_level_major_encoder_rays_missing_the_box():
    print("[case] encoder placement tiny64 rays missing the box", flush=True)
    w = synth.WORKLOADS["tiny64"]
    g = synth.cone_geometry(64, 8)
    g.off_u = 150.0
    ph = synth.make_phantom(3, 5)
    A = synth.project(ph, g).astype(np.float32)
    _train_both(nic.config_for(w, seed=54, rays_per_step=256), g, torch.tensor(A, device="cuda"), 3)


def test_default_placement_follows_the_l2_size():
    """tiny64 (0.94 MB table: fits in L2) and ct512 FP32 (16 MB per level) encode in the forward
    kernel; ct256 (4 MB / 2 MB per level) and ct512 FP16 (8 MB per level) level-major."""
    l2 = torch.cuda.get_device_properties(0).L2_cache_size
    print(f"[case] default encoder placement, L2 {l2} bytes", flush=True)
    assert l2 == 4 << 20            # one XCD's L2 on this GPU: the rule's unit
    want = {("tiny64", 0): False, ("tiny64", 1): False, ("ct256", 0): True, ("ct256", 1): True,
            ("ct512", 0): False, ("ct512", 1): True}
    for (wl, prec), lm in want.items():
        w = synth.WORKLOADS[wl]
        m = nic.Model(nic.config_for(w, seed=55, precision=prec), synth.cone_geometry(w.n_det, 4))
        assert m.encoder_level_major() == lm, (wl, prec)
        m.set_encoder_placement("in_forward")
        assert not m.encoder_level_major()
        m.set_encoder_placement("auto")
        assert m.encoder_level_major() == lm
        assert nic.lib().nic_set_encoder_placement(m.h, 3) == nic.NIC_EINVAL
        assert m.encoder_level_major() == lm
        m.close()


@pytest.mark.parametrize("workload,log2_table,width", [("tiny64", 10, 32), ("ct256", 10, 32), ("tiny64", 14, 64)])
def test_level_major_encoder_shared_bins_and_wide_mlp(workload, log2_table, width):
    """T = 2^10: every level is a hashed table of 1024 entries, so one 8192-entry gradient bin holds
    the entries of eight levels (tiny64: all 8 levels in a single bin; ct256: 16 levels in two bins)
    and each such bin's count is the sum of eight levels' edge rows.  Width 64: the 8-level, 64-wide
    kernel set."""
    print(f"[case] encoder placement {workload} T=2^{log2_table} W={width}", flush=True)
    w = synth.WORKLOADS[workload]
    _, g, A = synth.scan(w)
    over = dict(seed=56, log2_table=log2_table, mlp_width=width)
    if width == 64:
        over["mlp_depth"] = 4
    cfg = nic.config_for(w, **over)
    lay = nic.nic_describe(cfg)
    if log2_table == 10:
        assert lay["n_bins"] == (1 if workload == "tiny64" else 2)
    _train_both(cfg, g, torch.tensor(A, device="cuda"), 3)
