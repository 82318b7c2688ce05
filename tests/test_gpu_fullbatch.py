"""The benchmarked step at full size against the oracle, every ray and every parameter.

ct256 (256^3 phantom of 20 ellipsoids, 50 views on a 256 x 256 detector with Poisson noise, 16
levels x 2 features, T = 2^19, MLP 4 x 32, 2048 rays x 192 samples = 393,216 points per step): one
fused training step, FP32, through nic_step in the launch configuration the benchmark times, compared
with the oracle's Eq. (3) batch (Sec. 2.5) and Adam (Sec. 3.1) on the same pixels and jitter.  The
oracle splits the rays over the host's cores.  Checked: the loss, all 2048 ray sums of Eq. (1)
(nic_forward, same parameters), and every parameter and both Adam moments after the step.  The Adam
state before the step is a mid-training one (moments away from zero), so each parameter's update
is a smooth function of its gradient; the first moment after the step carries the gradient itself
(m = beta1 m0 + (1 - beta1) g), so its bar is a bar on the table scatter-add and the network
gradients of every parameter.  Also: mu of a 256^3 render at sampled voxel centres.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_19742_amd import nic, synth  # noqa: E402
from test_gpu_parity import FWD_TOL, GRAD_TOL, ocfg, random_params, rel  # noqa: E402

pytestmark = pytest.mark.gpu


def _threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


@pytest.fixture(scope="module")
def ct256(ora):
    w = synth.WORKLOADS["ct256"]
    print("[case] ct256 full batch: scan", flush=True)
    _, g, A = synth.scan(w)
    cfg = nic.config_for(w, seed=3)
    m = nic.Model(cfg, g)
    m.set_projections(torch.tensor(A, device="cuda"))
    yield w, g, A, cfg, m
    m.close()


def test_full_ct256_step_matches_oracle(ora, ct256):
    w, g, A, cfg, m = ct256
    oc = ocfg(ora, cfg)
    p = random_params(ora, oc, 81, 0.05)
    rng = np.random.default_rng(82)
    m0 = (rng.standard_normal(p.size) * 1e-5).astype(np.float32).astype(np.float64)
    v0 = rng.uniform(1e-10, 1e-9, p.size).astype(np.float32).astype(np.float64)
    m.load_params(p)
    tp_, tg_, tm_, tv_ = m.tensors()[:4]
    nt, nd, do = m.n_params()
    for dst, src in ((tm_, m0), (tv_, v0)):
        dst.zero_()
        dst[:nt].copy_(torch.tensor(src[:nt], dtype=torch.float32))
        dst[do:do + nd].copy_(torch.tensor(src[nt:], dtype=torch.float32))
    m.zero_grad()
    t = m.get_step() + 1
    pix, jit = synth.ray_batch(83, g.n_pix, w.rays, w.samples)
    tp, tj = torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")
    v = 17
    a = m.forward(v, tp, tj).cpu().numpy()
    loss = torch.zeros(1, device="cuda")
    m.step(v, tp, tj, loss)
    m.sync()
    print(f"[case] ct256 full batch: oracle on {_threads()} threads", flush=True)
    ora.set_threads(_threads())
    try:
        ol, oa, og = ora.ray_batch(oc, g, p, float(g.angles[v]), A[v], pix, jit)
    finally:
        ora.set_threads(1)
    op, om, ov = p.copy(), m0.copy(), v0.copy()
    ora.adam(op, og, om, ov, t)
    assert rel(a, oa) <= FWD_TOL
    assert abs(loss.item() - ol) <= FWD_TOL * abs(ol)
    # the step moved most of the table: no vacuous comparison
    touched = np.count_nonzero(og[:nt])
    assert touched > 0.5 * nt, touched
    got_p, got_m, got_v = (m.flat(x) for x in (tp_, tm_, tv_))
    assert rel(got_p, op) <= GRAD_TOL
    assert rel(got_m[:nt], om[:nt]) <= GRAD_TOL          # table gradient (scatter-add)
    assert rel(got_m[nt:], om[nt:]) <= GRAD_TOL          # LayerNorm + MLP gradients
    assert rel(got_v, ov) <= GRAD_TOL
    dp_gpu, dp_ora = got_p - p, op - p                   # the update itself, not only the sum
    assert rel(dp_gpu, dp_ora) <= 1e-3
    assert float(tg_.abs().max()) == 0.0                 # the fused step stores no gradient


def test_render_256_sampled_voxels_match_oracle(ora, ct256):
    """Forward-only inference of the full 256^3 grid (voxel centres): mu at 4096 sampled voxels,
    the eight corners and a full row, against the oracle."""
    w, g, A, cfg, m = ct256
    oc = ocfg(ora, cfg)
    p = random_params(ora, oc, 84, 0.05)
    m.load_params(p)
    n = 256
    vol = m.render_volume(n, n, n)
    rng = np.random.default_rng(85)
    ijk = rng.integers(0, n, (4096, 3))
    corners = np.array([[i, j, k] for i in (0, n - 1) for j in (0, n - 1) for k in (0, n - 1)])
    row = np.stack([np.arange(n), np.full(n, 100), np.full(n, 37)], 1)
    ijk = np.concatenate([ijk, corners, row])
    got = vol[torch.tensor(ijk[:, 2]), torch.tensor(ijk[:, 1]), torch.tensor(ijk[:, 0])].cpu().numpy()
    xn = ((ijk.astype(np.float64) + 0.5) / n).astype(np.float32)
    assert rel(got, ora.field(oc, p, xn)) <= FWD_TOL
    assert bool(torch.isfinite(vol).all())
