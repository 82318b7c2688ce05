"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Bars: corner entries bit-exact; forward values (encoding, mu, ray sums, loss) within 1e-5 and
gradients / post-Adam parameters within 1e-4, both as max|gpu - oracle| / max|oracle| per tensor
(entries near zero make an elementwise relative error meaningless).  Random draws (pixels, jitter)
are either given to both sides as data or drawn by both from Philox and compared bit for bit.
"""
import math

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
    scale = np.abs(ora).max()
    return float(np.abs(gpu - ora).max() / (scale if scale > 0 else 1.0))


def ocfg(ora, cfg: nic.Config):
    return ora.Config(n_levels=cfg.n_levels, feats=cfg.feats_per_level, log2_table=cfg.log2_table,
                      base_res=cfg.base_res, max_res=cfg.max_res, depth=cfg.mlp_depth,
                      width=cfg.mlp_width, out_act=cfg.out_act, layernorm=cfg.layernorm,
                      mu_max=cfg.mu_max, ln_eps=cfg.ln_eps)


def random_params(ora, oc, seed, table_scale):
    """Flat [table | dense] parameters: table N(0, table_scale), LN gain near 1, MLP uniform."""
    tot, nt, nd = ora.n_params(oc)
    lay = ora.dense_layout(oc)
    rng = np.random.default_rng(seed)
    p = synth.init_params(nt // 2, 2, lay, oc.depth, seed).astype(np.float64)
    p[:nt] = rng.standard_normal(nt) * table_scale
    o, n = lay["ln_g"]
    p[nt + o:nt + o + n] = 1.0 + 0.1 * rng.standard_normal(n)
    o, n = lay["ln_b"]
    p[nt + o:nt + o + n] = 0.05 * rng.standard_normal(n)
    return p.astype(np.float32).astype(np.float64)


class Case:
    """A model on the GPU plus the same scan on the host."""

    def __init__(self, ora, wname, seed=11, **over):
        w = synth.WORKLOADS[wname]
        self.w = w
        self.cfg = nic.config_for(w, seed=seed, **over)
        self.ph, self.g, self.A = synth.scan(w)
        self.oc = ocfg(ora, self.cfg)
        print(f"[case] {wname} {over} creating model", flush=True)
        self.model = nic.Model(self.cfg, self.g)
        self.proj = torch.tensor(self.A, device="cuda")
        self.model.set_projections(self.proj)

    def set_params(self, p):
        self.model.load_params(p)

    def params(self):
        return self.model.flat(self.model.tensors()[0])

    def grads(self):
        return self.model.flat(self.model.tensors()[1])


@pytest.fixture(scope="module")
def tiny(ora):
    return Case(ora, "tiny64")


def _pts(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)).astype(np.float32)
    # faces, edges and corners of the unit cube and exact grid vertices of a power-of-two level
    x[:8] = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [0.5, 1, 0.25],
                      [0.0, 0.5, 1.0]], np.float32)
    x[8:40] = (rng.integers(0, 17, (32, 3)) / 16).astype(np.float32)
    return x


def test_encode_indices_bit_exact_and_values(ora, tiny):
    c = tiny
    p = random_params(ora, c.oc, 1, 0.1)
    c.set_params(p)
    x = _pts(5000, 2)
    print("[gpu] nic_encode 5000 points", flush=True)
    enc, idx = c.model.encode(torch.tensor(x, device="cuda"), want_idx=True)
    oenc, oidx, _ = ora.encode(c.oc, p[:ora.n_params(c.oc)[1]], x, want_idx=True)
    assert np.array_equal(idx.cpu().numpy().astype(np.uint32), oidx)
    assert rel(enc.cpu().numpy(), oenc) <= FWD_TOL


def test_encode_all_collision_table(ora):
    """T = 32 entries per hashed level: every hashed level collides heavily."""
    c = Case(ora, "tiny64", log2_table=5, base_res=2, max_res=64)
    lay = c.model.layout
    assert sum(lay["dense"]) >= 1 and not all(lay["dense"])
    p = random_params(ora, c.oc, 3, 0.1)
    c.set_params(p)
    x = _pts(3000, 4)
    enc, idx = c.model.encode(torch.tensor(x, device="cuda"), want_idx=True)
    oenc, oidx, _ = ora.encode(c.oc, p[:ora.n_params(c.oc)[1]], x, want_idx=True)
    assert np.array_equal(idx.cpu().numpy().astype(np.uint32), oidx)
    assert rel(enc.cpu().numpy(), oenc) <= FWD_TOL
    c.model.close()


@pytest.mark.parametrize("scale", [1e-4, 0.1])
def test_query_matches_oracle(ora, tiny, scale):
    c = tiny
    p = random_params(ora, c.oc, 5, scale)
    c.set_params(p)
    x = _pts(3001, 6)                       # not a multiple of the 32-point wave tile
    mu = c.model.query(torch.tensor(x, device="cuda")).cpu().numpy()
    assert rel(mu, ora.field(c.oc, p, x)) <= FWD_TOL


def test_channel_mask_matches_oracle(ora):
    """Channel mask before LayerNorm (Sec. 2.3): forward, backward and a training step with some
    channels off (a pair of levels entirely, so neither is gathered nor scattered) and one scaled, against
    the oracle with the same mask; then the mask removed.  A model of its own: the step moves it."""
    import dataclasses
    c = Case(ora, "tiny64", seed=12)
    p = random_params(ora, c.oc, 35, 0.05)
    c.set_params(p)
    C_ = 2 * c.cfg.n_levels
    mask = [1.0] * C_
    # levels 1 and 3 (a pair handled together, channels 2, 3, 6, 7) fully off: skipped
    mask[1], mask[2], mask[3], mask[6], mask[7], mask[C_ - 1], mask[4] = 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.5
    oc = dataclasses.replace(c.oc, mask=tuple(mask))
    c.model.set_channel_mask(mask)
    try:
        x = _pts(777, 36)
        mu = c.model.query(torch.tensor(x, device="cuda")).cpu().numpy()
        assert rel(mu, ora.field(oc, p, x)) <= FWD_TOL
        pix, jit, tp, tj = _rays(c, 300, 37)
        a = c.model.forward(8, tp, tj).cpu().numpy()
        dA = np.random.default_rng(38).standard_normal(300).astype(np.float32)
        c.model.zero_grad()
        c.model.backward(8, tp, tj, torch.tensor(dA, device="cuda"))
        _, oa, og = ora.ray_batch(oc, c.g, p, float(c.g.angles[8]), c.A[8], pix, jit, dA=dA)
        assert rel(a, oa) <= FWD_TOL
        g = c.grads()
        nt = ora.n_params(oc)[1]
        assert rel(g[:nt], og[:nt]) <= GRAD_TOL
        assert rel(g[nt:], og[nt:]) <= GRAD_TOL
        # a training step with the level skipped (no gathers, no records) against the oracle step
        c.model.zero_grad()
        c.model.tensors()[2].zero_()
        c.model.tensors()[3].zero_()
        t0 = c.model.get_step()
        loss = torch.zeros(1, device="cuda")
        pix2, jit2, tp2, tj2 = _rays(c, 1024, 40)
        c.model.step(21, tp2, tj2, loss)
        ol, _, og2 = ora.ray_batch(oc, c.g, p, float(c.g.angles[21]), c.A[21], pix2, jit2)
        op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
        ora.adam(op, og2, om, ov, t0 + 1)
        assert abs(loss.item() - ol) <= FWD_TOL * abs(ol)
        assert rel(c.params(), op) <= GRAD_TOL
        c.set_params(p)
        with pytest.raises(nic.NicError):
            c.model.set_channel_mask([1.0] * (C_ - 1))
    finally:
        c.model.set_channel_mask(None)
    mu2 = c.model.query(torch.tensor(x, device="cuda")).cpu().numpy()
    assert rel(mu2, ora.field(c.oc, p, x)) <= FWD_TOL
    c.model.close()


def test_channel_spectrum_matches_oracle(ora, tiny):
    """FFT noise measure of every encoder channel (DFT on the GPU in FP64) against numpy's FFT on the
    oracle's encoding of the same probe points."""
    c = tiny
    p = random_params(ora, c.oc, 39, 0.05)
    c.set_params(p)
    nt = ora.n_params(c.oc)[1]
    for g_max in (32, 13):
        hf = c.model.channel_spectrum(g_max)
        ohf = ora.channel_hf_fraction(c.oc, p[:nt], g_max)
        assert np.abs(hf - ohf).max() <= 1e-5, (g_max, hf, ohf)
    with pytest.raises(nic.NicError):
        c.model.channel_spectrum(65)


def test_field_from_features_matches_oracle(ora, tiny):
    """LayerNorm + MLP + activation on given encoder outputs (the mapping Fig. 3 tracks), fed with the
    GPU's own encoding of 1001 points and with arbitrary feature vectors."""
    c = tiny
    p = random_params(ora, c.oc, 8, 0.1)
    c.set_params(p)
    x = _pts(1001, 9)
    tx = torch.tensor(x, device="cuda")
    enc = c.model.encode(tx)
    mu = c.model.field_from_features(enc).cpu().numpy()
    assert rel(mu, ora.field_from_features(c.oc, p, enc.cpu().numpy().astype(np.float64))) <= FWD_TOL
    assert rel(mu, c.model.query(tx).cpu().numpy()) <= 1e-6
    f = (np.random.default_rng(10).standard_normal((77, 2 * c.cfg.n_levels)) * 0.3).astype(np.float32)
    mu2 = c.model.field_from_features(torch.tensor(f, device="cuda")).cpu().numpy()
    assert rel(mu2, ora.field_from_features(c.oc, p, f.astype(np.float64))) <= FWD_TOL
    with pytest.raises(ValueError):
        c.model.field_from_features(torch.zeros((3, 5), device="cuda"))


def test_render_volume_matches_oracle(ora, tiny):
    c = tiny
    p = random_params(ora, c.oc, 7, 0.1)
    c.set_params(p)
    vol = c.model.render_volume(9, 7, 5).cpu().numpy()
    assert rel(vol, ora.render_volume(c.oc, p, 9, 7, 5)) <= FWD_TOL


def _rays(c, R, seed):
    pix, jit = synth.ray_batch(seed, c.g.n_pix, R, c.cfg.samples_per_ray)
    return pix, jit, torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")


@pytest.mark.parametrize("R", [1, 37, 1024])
def test_forward_ray_sums_match_oracle(ora, tiny, R):
    c = tiny
    p = random_params(ora, c.oc, 9, 0.1)
    c.set_params(p)
    pix, jit, tp, tj = _rays(c, R, 10 + R)
    v = 17
    a = c.model.forward(v, tp, tj).cpu().numpy()
    _, oa, _ = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[v]), c.A[v], pix, jit, grad=False)
    assert rel(a, oa) <= FWD_TOL


def test_backward_gradients_match_oracle(ora, tiny):
    c = tiny
    p = random_params(ora, c.oc, 12, 0.1)
    c.set_params(p)
    pix, jit, tp, tj = _rays(c, 256, 13)
    v = 3
    dA = np.random.default_rng(14).standard_normal(256).astype(np.float32)
    c.model.zero_grad()
    c.model.backward(v, tp, tj, torch.tensor(dA, device="cuda"))
    g = c.grads()
    _, _, og = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[v]), c.A[v], pix, jit, dA=dA)
    nt = ora.n_params(c.oc)[1]
    assert rel(g[:nt], og[:nt]) <= GRAD_TOL
    assert rel(g[nt:], og[nt:]) <= GRAD_TOL
    lay = ora.dense_layout(c.oc)
    for name, on in lay.items():
        if name == "n":
            continue
        o, n = on
        assert rel(g[nt + o:nt + o + n], og[nt + o:nt + o + n]) <= GRAD_TOL, name


def test_backward_accumulates(ora, tiny):
    """Two backward calls without zeroing add up."""
    c = tiny
    p = random_params(ora, c.oc, 15, 0.1)
    c.set_params(p)
    pix, jit, tp, tj = _rays(c, 64, 16)
    dA = torch.full((64,), 0.5, device="cuda")
    c.model.zero_grad()
    c.model.backward(1, tp, tj, dA)
    g1 = c.grads()
    c.model.backward(1, tp, tj, dA)
    g2 = c.grads()
    assert rel(g2, 2 * g1) <= 1e-6


def test_adam_matches_oracle(ora, tiny):
    c = tiny
    p = random_params(ora, c.oc, 17, 0.1)
    c.set_params(p)
    P, G, M, V, _ = c.model.tensors()
    M.zero_()
    V.zero_()
    nt, nd, do = c.model.n_params()
    rng = np.random.default_rng(18)
    om, ov, op = np.zeros_like(p), np.zeros_like(p), p.copy()
    step0 = c.model.get_step()
    for t in range(1, 4):
        g = (rng.standard_normal(len(p)) * 1e-2).astype(np.float32).astype(np.float64)
        g[::5] = 0.0
        G.zero_()
        G[:nt].copy_(torch.tensor(g[:nt], dtype=torch.float32))
        G[do:do + nd].copy_(torch.tensor(g[nt:], dtype=torch.float32))
        c.model.adam()
        ora.adam(op, g, om, ov, step0 + t)
    assert rel(c.params(), op) <= GRAD_TOL
    assert float(G.abs().max()) == 0.0


def test_l1_step_matches_oracle(ora, tiny):
    """Full training steps (Eq. 3 loss, backward, Adam) with explicit rays and jitter."""
    c = tiny
    p = random_params(ora, c.oc, 19, 1e-4)
    c.set_params(p)
    c.model.zero_grad()
    c.model.tensors()[2].zero_()
    c.model.tensors()[3].zero_()
    t0 = c.model.get_step()
    op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
    loss = torch.zeros(1, device="cuda")
    for k in range(3):
        pix, jit, tp, tj = _rays(c, 1024, 20 + k)
        v = (5 * k + 2) % 50
        c.model.step(v, tp, tj, loss)
        ol, _, og = ora.ray_batch(c.oc, c.g, op, float(c.g.angles[v]), c.A[v], pix, jit)
        ora.adam(op, og, om, ov, t0 + k + 1)
        assert abs(loss.item() - ol) <= FWD_TOL * abs(ol)
    assert rel(c.params(), op) <= GRAD_TOL


def test_step_consumes_pending_gradient(ora, tiny):
    """A training step normally runs Adam inside its reductions (the gradient is never stored); when
    nic_backward has left a gradient pending, the step adds its own gradient to it and Adam consumes
    the sum, as a stored-gradient optimiser would."""
    c = tiny
    p = random_params(ora, c.oc, 31, 1e-2)
    c.set_params(p)
    c.model.zero_grad()
    c.model.tensors()[2].zero_()
    c.model.tensors()[3].zero_()
    t0 = c.model.get_step()
    pix1, jit1, tp1, tj1 = _rays(c, 200, 32)
    dA = np.random.default_rng(33).standard_normal(200).astype(np.float32)
    c.model.backward(4, tp1, tj1, torch.tensor(dA, device="cuda"))
    pix2, jit2, tp2, tj2 = _rays(c, 1024, 34)
    loss = torch.zeros(1, device="cuda")
    c.model.step(17, tp2, tj2, loss)
    _, _, g1 = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[4]), c.A[4], pix1, jit1, dA=dA)
    ol, _, g2 = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[17]), c.A[17], pix2, jit2)
    op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
    ora.adam(op, g1 + g2, om, ov, t0 + 1)
    assert abs(loss.item() - ol) <= FWD_TOL * abs(ol)
    assert rel(c.params(), op) <= GRAD_TOL
    assert float(c.model.tensors()[1].abs().max()) == 0.0       # consumed
    assert c.model.get_step() == t0 + 1
    # the next step has no pending gradient again: fused form, same oracle recurrence
    c.model.step(23, tp2, tj2, loss)
    _, _, g3 = ora.ray_batch(c.oc, c.g, op, float(c.g.angles[23]), c.A[23], pix2, jit2)
    ora.adam(op, g3, om, ov, t0 + 2)
    assert rel(c.params(), op) <= GRAD_TOL
    assert float(c.model.tensors()[1].abs().max()) == 0.0


@pytest.mark.parametrize("workload,precision", [("tiny64", 0), ("tiny64", 1), ("ct256", 0), ("ct256", 1),
                                                ("ct512", 1)])
def test_fused_step_equals_backward_then_adam(ora, workload, precision):
    """A training step runs Adam inside its reductions: in the bin reduction for bins one block
    holds, in the combine kernel for bins cut between blocks and for bins without records, and in
    the dense blocks for LayerNorm + MLP.  The same step as a stored-gradient backward pass (dA =
    sign(A - A_gt) / R, Eq. 3) followed by the one separate Adam pass gives the same parameters,
    moments and FP16 table bit for bit: the update does not depend on which kernel runs it.  At
    ct256 this is the benchmarked step (2048 rays x 192 samples, 745 bins over 256 reduction
    blocks), whose backward pass the paper-scale test checks against the oracle on sampled rays; at
    ct512 the largest benchmarked step (8192 rays x 320 samples, T = 2^21), against zero projections
    (generating the 100 views of the scan would take most of the test's time)."""
    print(f"[case] fused step {workload} precision {precision}", flush=True)
    w = synth.WORKLOADS[workload]
    if workload == "ct512":
        g = synth.cone_geometry(w.n_det, w.n_views)
        A = np.zeros((w.n_views, g.nv, g.nu), np.float32)
    else:
        _, g, A = synth.scan(w)
    proj = torch.tensor(A, device="cuda")
    models = []
    for _ in range(2):
        m = nic.Model(nic.config_for(w, seed=41, precision=precision), g)
        m.set_projections(proj)
        m.train(2, want_loss=False)            # moments away from zero
        models.append(m)
    a, b = models
    for k in range(4):
        assert torch.equal(a.tensors()[k], b.tensors()[k])
    R, v = w.rays, 29
    pix, jit = synth.ray_batch(45, g.n_pix, R, w.samples)
    tp, tj = torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")
    a.step(v, tp, tj)
    Ab = b.forward(v, tp, tj).cpu().numpy()
    res = Ab - A[v].reshape(-1)[pix]
    dA = np.sign(res).astype(np.float32) * (np.float32(1.0) / np.float32(R))
    b.backward(v, tp, tj, torch.tensor(dA, device="cuda"))
    b.adam()
    assert a.get_step() == b.get_step()
    ta, tb = a.tensors(), b.tensors()
    for k in (0, 1, 2, 3):                         # params, gradient (zero in both), moments
        assert torch.equal(ta[k], tb[k]), k
    if precision:
        assert torch.equal(ta[4], tb[4])
    for m in models:
        m.close()


def test_empty_and_out_of_range_inputs(ora, tiny):
    """Empty batches are no-ops (the null pointers of empty tensors are never used); more rays than a
    step holds, a view outside the scan and a negative point count are refused, and nothing moves."""
    c = tiny
    p = random_params(ora, c.oc, 47, 0.05)
    c.set_params(p)
    c.model.zero_grad()
    p0 = c.model.tensors()[0].clone()
    N = c.cfg.samples_per_ray
    e_i = torch.empty(0, dtype=torch.int32, device="cuda")
    e_f = torch.empty((0, N), dtype=torch.float32, device="cuda")
    assert c.model.forward(3, e_i, e_f).numel() == 0
    c.model.backward(3, e_i, e_f, torch.empty(0, device="cuda"))
    assert c.model.query(torch.empty((0, 3), device="cuda")).numel() == 0
    R = c.cfg.rays_per_step
    pix, jit = synth.ray_batch(48, c.g.n_pix, R + 1, N)
    tp, tj = torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")
    with pytest.raises(nic.NicError):
        c.model.forward(3, tp, tj)
    with pytest.raises(nic.NicError):
        c.model.backward(3, tp, tj, torch.zeros(R + 1, device="cuda"))
    with pytest.raises(nic.NicError):
        c.model.forward(len(c.g.angles), tp[:R], tj[:R])
    with pytest.raises(nic.NicError):
        nic._check(nic.lib().nic_query(c.model.h, None, -1, None))
    torch.cuda.synchronize()
    assert torch.equal(c.model.tensors()[0], p0)
    assert float(c.model.tensors()[1].abs().max()) == 0.0
    # the largest batch a step holds is accepted and matches the oracle
    a = c.model.forward(5, tp[:R], tj[:R]).cpu().numpy()
    _, oa, _ = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[5]), c.A[5], pix[:R], jit[:R], grad=False)
    assert rel(a, oa) <= FWD_TOL


def test_device_draws_match_oracle(ora, tiny):
    """Pixels (Feistel over Philox, cycle walking) and jitter drawn on the GPU, bit for bit."""
    c = tiny
    for step in [0, 1, 777]:
        pix, jit = c.model.draw_rays(step)
        opix, ojit = ora.draw_rays(c.cfg.seed, step, c.g.n_pix, c.cfg.rays_per_step, c.cfg.samples_per_ray)
        assert np.array_equal(pix.cpu().numpy(), opix)
        assert np.array_equal(jit.cpu().numpy(), ojit)
    for step in range(0, 120, 7):
        assert c.model.view_for_step(step) == ora.view_for_step(c.cfg.seed, step, 50)


def test_device_init_matches_oracle(ora, tiny):
    c = tiny
    c.model.init_params(1234)
    p = c.params()
    op = ora.init_params(c.oc, 1234)
    assert rel(p, op) <= 1e-6


def test_train_with_device_draws_matches_oracle(ora, tiny):
    """nic_train (every draw on the device) against the oracle's own Philox schedule."""
    c = tiny
    c.model.init_params(c.cfg.seed)
    p = c.params()
    losses = c.model.train(4)
    op, om, ov = p.copy(), np.zeros_like(p), np.zeros_like(p)
    ol = ora.train(c.oc, c.g, c.g.angles, c.A, op, om, ov, 0, 4, c.cfg.rays_per_step,
                   c.cfg.samples_per_ray, c.cfg.seed)
    assert rel(losses, ol) <= FWD_TOL
    assert rel(c.params(), op) <= GRAD_TOL


def test_rays_missing_the_box(ora):
    """A detector shifted far sideways: some rays miss the box (A = 0, no gradient)."""
    w = synth.WORKLOADS["tiny64"]
    cfg = nic.config_for(w, rays_per_step=256)
    g = synth.cone_geometry(64, 8)
    g.off_u = 150.0
    oc = ocfg(ora, cfg)
    m = nic.Model(cfg, g)
    p = random_params(ora, oc, 21, 0.1)
    m.load_params(p)
    pix, jit = synth.ray_batch(22, g.n_pix, 256, 64)
    a = m.forward(0, torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")).cpu().numpy()
    proj = np.zeros(g.n_pix, np.float32)
    _, oa, _ = ora.ray_batch(oc, g, p, float(g.angles[0]), proj, pix, jit, grad=False)
    assert (oa == 0).sum() > 10 and (oa > 0).sum() > 10
    assert np.all(a[oa == 0] == 0)
    assert rel(a, oa) <= FWD_TOL
    m.close()


@pytest.mark.parametrize("N,depth,ln", [(32, 1, 1), (320, 2, 1), (64, 3, 0)])
def test_other_shapes_forward_backward(ora, N, depth, ln):
    """Other sample counts and depths, and the encoder without its LayerNorm (plain hash encoding)."""
    w = synth.WORKLOADS["tiny64"]
    cfg = nic.config_for(w, samples_per_ray=N, mlp_depth=depth, rays_per_step=96, layernorm=ln)
    g = synth.cone_geometry(64, 50)
    ph = synth.make_phantom(1, 6)
    A = synth.project(ph, g).astype(np.float32)
    oc = ocfg(ora, cfg)
    m = nic.Model(cfg, g)
    m.set_projections(torch.tensor(A, device="cuda"))
    p = random_params(ora, oc, 23, 0.1)
    m.load_params(p)
    pix, jit = synth.ray_batch(24, g.n_pix, 96, N)
    tp, tj = torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")
    a = m.forward(9, tp, tj).cpu().numpy()
    dA = np.random.default_rng(25).standard_normal(96).astype(np.float32)
    m.zero_grad()
    m.backward(9, tp, tj, torch.tensor(dA, device="cuda"))
    gr = m.flat(m.tensors()[1])
    _, oa, og = ora.ray_batch(oc, g, p, float(g.angles[9]), A[9], pix, jit, dA=dA)
    assert rel(a, oa) <= FWD_TOL
    nt = ora.n_params(oc)[1]
    assert rel(gr[:nt], og[:nt]) <= GRAD_TOL
    assert rel(gr[nt:], og[nt:]) <= GRAD_TOL
    m.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_paper_scale_sampled_rays(ora, precision):
    """256^3 workload (16 levels, T = 2^19, 4x32 MLP, 192 samples): the full 2048-ray forward in the
    launch configuration of the benchmark, checked on a sample of rays computed by the oracle.  FP32
    to the parity bars.  The precision form: forward to the bound of its error table; gradients by
    the largest entry error (a ReLU decision that BF16 operands flip moves one point's whole
    contribution, so this is not a rounding bound) and by the error in the 2-norm."""
    c = Case(ora, "ct256", precision=precision)
    fwd_tol, grad_tol = (FWD_TOL, GRAD_TOL) if precision == 0 else (3e-2, 0.25)
    p = random_params(ora, c.oc, 26, 0.05)
    c.set_params(p)
    pix, jit, tp, tj = _rays(c, 2048, 27)
    v = 11
    a = c.model.forward(v, tp, tj).cpu().numpy()
    sel = np.random.default_rng(28).choice(2048, 24, replace=False)
    _, oa, _ = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[v]), c.A[v], pix[sel], jit[sel], grad=False)
    assert rel(a[sel], oa) <= fwd_tol
    # gradient of the sampled rays alone (dA zero elsewhere) against the oracle
    dA = np.zeros(2048, np.float32)
    dA[sel] = np.random.default_rng(29).standard_normal(24).astype(np.float32)
    c.model.zero_grad()
    c.model.backward(v, tp, tj, torch.tensor(dA, device="cuda"))
    g = c.grads()
    _, _, og = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[v]), c.A[v], pix[sel], jit[sel], dA=dA[sel])
    nt = ora.n_params(c.oc)[1]
    l2 = [float(np.linalg.norm(x - y) / np.linalg.norm(y)) for x, y in ((g[:nt], og[:nt]), (g[nt:], og[nt:]))]
    print(f"[case] ct256 precision {precision}: table gradient max {rel(g[:nt], og[:nt]):.3g} 2-norm {l2[0]:.3g}; "
          f"dense gradient max {rel(g[nt:], og[nt:]):.3g} 2-norm {l2[1]:.3g}", flush=True)
    assert rel(g[:nt], og[:nt]) <= grad_tol
    assert rel(g[nt:], og[nt:]) <= grad_tol
    if precision:   # measured: table 0.067, dense 0.0055 (24 rays x 192 samples, random network)
        assert max(l2) <= 0.15
    c.model.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_largest_workload_sampled_rays(ora, precision):
    """512^3 workload (T = 2^21, 8192 rays x 320 samples = 2.6 M points per launch, the largest
    configuration benchmarked): forward over all rays and backward, checked on sampled rays.  FP32 to
    the parity bars; the precision form to the bounds of its error table."""
    w = synth.WORKLOADS["ct512"]
    cfg = nic.config_for(w, precision=precision, seed=3)
    g = synth.cone_geometry(w.n_det, w.n_views)
    oc = ocfg(ora, cfg)
    print(f"[case] ct512 precision {precision} creating model", flush=True)
    m = nic.Model(cfg, g)
    p = random_params(ora, oc, 41, 0.05)
    m.load_params(p)
    R = cfg.rays_per_step
    pix, jit = synth.ray_batch(42, g.n_pix, R, cfg.samples_per_ray)
    tp, tj = torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")
    v = 37
    a = m.forward(v, tp, tj).cpu().numpy()
    sel = np.random.default_rng(43).choice(R, 16, replace=False)
    zero_proj = np.zeros(g.n_pix, np.float32)
    _, oa, _ = ora.ray_batch(oc, g, p, float(g.angles[v]), zero_proj, pix[sel], jit[sel], grad=False)
    fwd_tol, grad_tol = (FWD_TOL, GRAD_TOL) if precision == 0 else (3e-2, 0.1)
    assert rel(a[sel], oa) <= fwd_tol
    dA = np.zeros(R, np.float32)
    dA[sel] = np.random.default_rng(44).standard_normal(16).astype(np.float32)
    m.zero_grad()
    m.backward(v, tp, tj, torch.tensor(dA, device="cuda"))
    gr = m.flat(m.tensors()[1])
    _, _, og = ora.ray_batch(oc, g, p, float(g.angles[v]), zero_proj, pix[sel], jit[sel], dA=dA[sel])
    nt = ora.n_params(oc)[1]
    assert rel(gr[:nt], og[:nt]) <= grad_tol
    assert rel(gr[nt:], og[nt:]) <= grad_tol
    m.close()


def test_autograd_function_matches_oracle_and_fd(ora, tiny):
    """The hand-written backward behind torch.autograd.Function: Eq. (3) loss written in torch on
    top of the rendered ray sums; gradient vs the oracle (1e-4) and vs FP32 central differences."""
    from paper_2506_19742_amd import autograd as ag
    c = tiny
    p = random_params(ora, c.oc, 30, 0.1)
    c.set_params(p)
    pix, jit, tp, tj = _rays(c, 128, 31)
    v = 4
    params = ag.leaf_params(c.model)
    params.grad = None
    gt = torch.tensor(c.A[v].ravel()[pix], device="cuda")
    A = ag.render(params, c.model, v, tp, tj)
    loss = (A - gt).abs().mean()
    loss.backward()
    g = c.model.flat(params.grad)
    ol, _, og = ora.ray_batch(c.oc, c.g, p, float(c.g.angles[v]), c.A[v], pix, jit)
    nt = ora.n_params(c.oc)[1]
    assert abs(loss.item() - ol) <= FWD_TOL * abs(ol)
    assert rel(g[:nt], og[:nt]) <= GRAD_TOL
    assert rel(g[nt:], og[nt:]) <= GRAD_TOL
    # FP32 central differences of a smooth functional sum_r w_r A_r on the largest gradients
    w = torch.tensor(np.random.default_rng(32).standard_normal(128), dtype=torch.float32, device="cuda")
    params.grad = None
    (ag.render(params, c.model, v, tp, tj) * w).sum().backward()
    gw = params.grad.detach().clone()
    nt_, nd_, do_ = c.model.n_params()
    # finest level: an entry touches few samples, so the perturbation crosses few ReLU kinks
    fine0 = 2 * c.model.layout["offset"][-1]
    cand = torch.cat([fine0 + torch.topk(gw[fine0:nt_].abs(), 4).indices,
                      do_ + torch.topk(gw[do_:do_ + nd_].abs(), 4).indices])
    def central(k, h):
        old = params[k].item()
        params[k] = old + h
        fp = float((c.model.forward(v, tp, tj).double() * w.double()).sum())
        params[k] = old - h
        fm = float((c.model.forward(v, tp, tj).double() * w.double()).sum())
        params[k] = old
        return (fp - fm) / (2 * h)

    # Rays the perturbed entry does not touch give bit-identical sums in fp and fm, so their FP32
    # rounding cancels; the remaining noise is a few 1e-6 of the touched rays' sums.
    with torch.no_grad():
        for k in cand.tolist():
            h = 1e-3 * max(1.0, abs(params[k].item()))
            fd = central(k, h)
            assert abs(fd - gw[k].item()) <= 3e-2 * abs(gw[k].item()) + 2e-3, (k, fd, gw[k].item())
    params.requires_grad_(False)


def test_autograd_precision_form_with_torch_optimizer(ora):
    """Precision form (FP16 table copy, BF16 network operands) under autograd with a torch
    optimiser: the update torch makes is seen by the next forward (the FP16 copy is refreshed),
    no gradient stays pending, and a library step afterwards equals the same step of a fresh model
    holding the torch-updated parameters, bit for bit.  The loss agrees with the FP64 oracle within
    the precision form's bound."""
    from paper_2506_19742_amd import autograd as ag
    w = synth.WORKLOADS["tiny64"]
    ph, g, A = synth.scan(w)
    proj = torch.tensor(A, device="cuda")
    cfg = nic.config_for(w, seed=35, precision=1)
    print("[case] autograd precision form", flush=True)
    ma, mb = nic.Model(cfg, g), nic.Model(cfg, g)
    for m in (ma, mb):
        m.set_projections(proj)
    oc = ocfg(ora, cfg)
    p = random_params(ora, oc, 36, 0.05)
    ma.load_params(p)
    pix, jit = synth.ray_batch(37, g.n_pix, 256, cfg.samples_per_ray)
    tp, tj = torch.tensor(pix, device="cuda"), torch.tensor(jit, device="cuda")
    v = 9
    params = ag.leaf_params(ma)
    opt = torch.optim.SGD([params], lr=0.5)
    gt = torch.tensor(A[v].ravel()[pix], device="cuda")
    loss = (ag.render(params, ma, v, tp, tj) - gt).abs().mean()
    ol, _, _ = ora.ray_batch(oc, g, p, float(g.angles[v]), A[v], pix, jit, grad=False)
    assert abs(loss.item() - ol) <= 3e-2 * abs(ol)
    loss.backward()
    assert float(params.grad.abs().max()) > 0
    opt.step()
    params.requires_grad_(False)
    assert float(ma.tensors()[1].abs().max()) == 0.0           # nothing pending in the library
    # a fresh model holding the torch-updated parameters renders the same ray sums, bit for bit
    mb.load_params(ma.flat(ma.tensors()[0]))
    assert torch.equal(ma.tensors()[0], mb.tensors()[0])
    with torch.no_grad():
        a1 = ag.render(ma.tensors()[0], ma, v, tp, tj)
    assert torch.equal(a1, mb.forward(v, tp, tj))
    # and the library's own step continues from there identically (no stale gradient applied)
    for m in (ma, mb):
        m.step(v, tp, tj)
        m.sync()
    for k in range(5):
        assert torch.equal(ma.tensors()[k], mb.tensors()[k]), k
    ma.close()
    mb.close()


def test_autograd_refuses_a_foreign_parameter_tensor(tiny):
    from paper_2506_19742_amd import autograd as ag
    c = tiny
    pix, jit, tp, tj = _rays(c, 16, 38)
    with pytest.raises(ValueError):
        ag.render(c.model.tensors()[0].clone().requires_grad_(True), c.model, 2, tp, tj)


def test_repeated_steps_are_bitwise_reproducible(ora):
    """The whole step is deterministic (integer table-gradient sums, fixed-order dense reductions)."""
    w = synth.WORKLOADS["tiny64"]
    ph, g, A = synth.scan(w)
    outs = []
    for _ in range(2):
        m = nic.Model(nic.config_for(w, seed=13), g)
        m.set_projections(torch.tensor(A, device="cuda"))
        m.train(5, want_loss=False)
        outs.append(m.tensors()[0].clone())
        m.close()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("workload", ["tiny64", "ct256"])
def test_train_call_split_is_bitwise(workload):
    """Within a training call each step's last kernel draws the next step's rays; a call of 7 steps,
    7 calls of one step and calls of 2 + 5 steps give the same losses, parameters, gradients and
    Adam moments bit for bit (tiny64 encodes in the forward kernel, ct256 level-major)."""
    print(f"[case] training call split {workload}", flush=True)
    w = synth.WORKLOADS[workload]
    _, g, A = synth.scan(w)
    proj = torch.tensor(A, device="cuda")
    runs = []
    for split in ((7,), (1,) * 7, (2, 5)):
        m = nic.Model(nic.config_for(w, seed=23), g)
        m.set_projections(proj)
        losses = np.concatenate([m.train(k) for k in split])
        assert m.get_step() == 7
        runs.append((losses, [None if t is None else t.clone() for t in m.tensors()]))
        m.close()
    for losses, ts in runs[1:]:
        assert np.array_equal(losses, runs[0][0])
        for k, (x, y) in enumerate(zip(ts, runs[0][1])):
            assert (x is None) == (y is None), k
            if x is not None:
                assert torch.equal(x, y), k


def test_checkpoint_resume_is_bitwise(ora):
    """Kill/resume: 3 steps, save, load into a fresh model, 3 more steps == 6 uninterrupted steps."""
    w = synth.WORKLOADS["tiny64"]
    ph, g, A = synth.scan(w)
    proj = torch.tensor(A, device="cuda")
    ref = nic.Model(nic.config_for(w, seed=21), g)
    ref.set_projections(proj)
    ref_losses = ref.train(6)
    a = nic.Model(nic.config_for(w, seed=21), g)
    a.set_projections(proj)
    a.train(3)
    blob = a.save_state()
    a.close()
    b = nic.Model(nic.config_for(w, seed=21), g)
    b.set_projections(proj)
    b.init_params(999)                       # different state before loading
    b.load_state(blob)
    assert b.get_step() == 3
    losses = b.train(3)
    assert torch.equal(b.tensors()[0], ref.tensors()[0])
    assert np.array_equal(losses, ref_losses[3:])
    c = nic.Model(nic.config_for(w, seed=22), g)
    with pytest.raises(nic.NicError) as ei:
        c.load_state(blob)
    assert ei.value.status == nic.NIC_EVERSION
    for mm in (ref, b, c):
        mm.close()
