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

ReLU gates that FP32 cannot decide.  A step evaluates 393,216 x 4 x 32 = 50 M hidden
pre-activations; a few hundred of them lie within 1e-6 of zero, where the FP32 kernel and the FP64
oracle may take the ReLU derivative (0 at and below zero) differently.  A flipped gate changes that
one point's gradient through the whole network, and at the fine levels an entry's gradient is made
of one or two points, so those entries differ by a large fraction of their value: both results are
correct for their precision.  The tests therefore compare at the bar everything no such gate
decides: every parameter, the dense gradient, the table gradient over all rays free of such gates
(nic_backward with the oracle's upstream gradient, zero on the other rays), and the table moments of
the fused step outside the corner entries of the points that carry such a gate.
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


GATE_TAU = 1e-6   # |hidden pre-activation| below which FP32 and FP64 may take the ReLU gate apart


def _gate_margins(ora, oc, g, p, angle, pix, jit):
    """Sample positions [R*N][3] (FP32, as both sides compute them) and the smallest |hidden
    pre-activation| of every point [R][N] in FP64 (inf on rays that miss the box)."""
    R, N = jit.shape
    xs, hit = [], np.zeros(R, bool)
    for r in range(R):
        h, xn, _ = ora.ray_samples(g, angle, int(pix[r]), N, jit[r])
        hit[r] = h
        xs.append(xn if h else np.full((N, 3), 0.5, np.float32))
    xn = np.concatenate(xs)
    _, _, h = ora.field(oc, p, xn, want=True)
    _, nt, _ = ora.n_params(oc)
    lay, dense = ora.dense_layout(oc), p[nt:]
    marg = np.full(xn.shape[0], np.inf)
    for k in range(oc.depth):
        o, n = lay[f"W{k}"]
        Wk = dense[o:o + n].reshape(oc.width, -1)
        o, n = lay[f"b{k}"]
        a = h @ Wk.T + dense[o:o + n]
        marg = np.minimum(marg, np.abs(a).min(1))
        h = np.maximum(a, 0.0)
    marg[~np.repeat(hit, N)] = np.inf
    return xn, marg.reshape(R, N)


def _batch(g, w):
    pix, jit = synth.ray_batch(83, g.n_pix, w.rays, w.samples)
    return pix, jit, torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda"), 17


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
    pix, jit, tp, tj, v = _batch(g, w)
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
    assert rel(got_p, op) <= GRAD_TOL                    # every parameter
    assert rel(got_m[nt:], om[nt:]) <= GRAD_TOL          # LayerNorm + MLP gradients
    assert rel(got_v[nt:], ov[nt:]) <= GRAD_TOL
    assert rel(got_v, ov) <= GRAD_TOL
    # table moments (the scatter-add) outside the corner entries of points with an undecided gate
    xn, marg = _gate_margins(ora, oc, g, p, float(g.angles[v]), pix, jit)
    amb = marg.reshape(-1) < GATE_TAU
    _, idx, _ = ora.encode(oc, p[:nt], xn[amb], want_idx=True)
    keep = np.ones(nt, bool)
    keep[2 * idx.reshape(-1).astype(np.int64)] = False
    keep[2 * idx.reshape(-1).astype(np.int64) + 1] = False
    print(f"[case] ct256 full batch: {int(amb.sum())} points with an undecided gate, "
          f"{int((~keep).sum())} table parameters set aside", flush=True)
    assert (~keep).sum() < 0.01 * touched
    assert rel(got_m[:nt][keep], om[:nt][keep]) <= GRAD_TOL
    dp_gpu, dp_ora = got_p - p, op - p                   # the update itself, not only the sum
    assert rel(np.concatenate([dp_gpu[:nt][keep], dp_gpu[nt:]]),
               np.concatenate([dp_ora[:nt][keep], dp_ora[nt:]])) <= 1e-3
    assert float(tg_.abs().max()) == 0.0                 # the fused step stores no gradient


def test_full_ct256_backward_matches_oracle(ora, ct256):
    """The scatter-add of the whole batch: nic_backward with the oracle's Eq. (3) upstream gradient
    sign(A - A_gt) / R, set to zero on the rays that hold a point with an undecided ReLU gate; the
    whole table gradient and the network gradients against the oracle's on the same dA."""
    w, g, A, cfg, m = ct256
    oc = ocfg(ora, cfg)
    p = random_params(ora, oc, 81, 0.05)
    m.load_params(p)
    m.zero_grad()
    nt, nd, do = m.n_params()
    pix, jit, tp, tj, v = _batch(g, w)
    ang = float(g.angles[v])
    ora.set_threads(_threads())
    try:
        _, oa, _ = ora.ray_batch(oc, g, p, ang, A[v], pix, jit, grad=False)
        res = oa - np.asarray(A[v], np.float64).reshape(-1)[pix]
        assert np.abs(res).min() > 1e-3          # every residual's sign is decided
        dA = (np.sign(res) / w.rays).astype(np.float32).astype(np.float64)
        _, marg = _gate_margins(ora, oc, g, p, ang, pix, jit)
        free = marg.min(1) >= GATE_TAU
        print(f"[case] ct256 full backward: {int(free.sum())} of {w.rays} rays free of undecided gates",
              flush=True)
        assert free.sum() >= 0.75 * w.rays
        dA[~free] = 0.0
        m.backward(v, tp, tj, torch.tensor(dA, dtype=torch.float32, device="cuda"))
        gg = m.flat(m.tensors()[1])
        _, _, og = ora.ray_batch(oc, g, p, ang, A[v], pix, jit, dA=dA)
    finally:
        ora.set_threads(1)
        m.zero_grad()
    assert np.count_nonzero(og[:nt]) > 0.5 * nt
    assert rel(gg[:nt], og[:nt]) <= GRAD_TOL
    assert rel(gg[nt:], og[nt:]) <= GRAD_TOL


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
