"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a published known-answer vector, a closed form,
brute force with arbitrary-precision integers, an independent library implementation (torch's
LayerNorm/Linear/autograd in float64), an invariant of the definition, or central finite
differences.  A plausible slip in the oracle (dropped term, wrong sign, swapped index or operand)
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2506_19742_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------------------------
# Random draws
# ---------------------------------------------------------------------------------------------

def test_philox_known_answers(ora):
    """Philox4x32-10 reproduces the vectors published with Random123 (Salmon et al., SC'11)."""
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = ora.philox(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10]
        n += 1
    assert n == 3


@pytest.mark.parametrize("n_pix,R", [(4096, 1024), (65536, 2048), (1000, 1000), (5, 3), (65, 64)])
def test_ray_pixels_distinct_and_in_range(ora, n_pix, R):
    """Ray slots of one step map to distinct pixels in [0, n_pix) (sampling without replacement)."""
    pix, jit = ora.draw_rays(1234, 7, n_pix, R, 4)
    assert pix.min() >= 0 and pix.max() < n_pix
    assert len(np.unique(pix)) == R
    assert jit.min() >= 0.0 and jit.max() < 1.0
    # jitter lies on the 2^-24 grid (exact in FP32 and FP64)
    assert np.all(jit * (1 << 24) == np.floor(jit * (1 << 24)))


def test_ray_pixels_full_permutation(ora):
    """With R = n_pix the slots enumerate every pixel exactly once (a bijection)."""
    pix, _ = ora.draw_rays(99, 3, 300, 300, 1)
    assert sorted(pix.tolist()) == list(range(300))


def test_voxel_points_are_philox_words(ora):
    """Pre-training points: the first three words of Philox block (p, t, 0, 6), each as a 24-bit
    uniform; checked against the published generator (pinned by its known answers above)."""
    xn = ora.voxel_points(77, 5, 300)
    for p in (0, 1, 299):
        w = ora.philox([p, 5, 0, 6], [77, 0])
        assert xn[p].tolist() == [float(int(x) >> 8) / 2 ** 24 for x in w[:3]]
    assert xn.min() >= 0 and xn.max() < 1 and abs(xn.mean() - 0.5) < 0.05


def test_view_order_visits_every_view_each_epoch(ora):
    V = 50
    for e in range(3):
        views = [ora.view_for_step(5, e * V + k, V) for k in range(V)]
        assert sorted(views) == list(range(V))
    # different epochs use different orders
    a = [ora.view_for_step(5, k, V) for k in range(V)]
    b = [ora.view_for_step(5, V + k, V) for k in range(V)]
    assert a != b


# ---------------------------------------------------------------------------------------------
# Multiresolution grid and hash encoding
# ---------------------------------------------------------------------------------------------

def test_level_resolutions_closed_forms(ora):
    # geometric progression endpoints: N_0 = N_min and N_{L-1} = N_max
    for L, lo, hi in [(8, 16, 256), (16, 16, 2048), (4, 2, 5)]:
        res, dense, off, size, n = ora.levels(ora.Config(n_levels=L, base_res=lo, max_res=hi))
        assert res[0] == lo and res[-1] == hi
        assert np.all(np.diff(res) >= 0)
    # b = 2 exactly: a doubling progression
    res, *_ = ora.levels(ora.Config(n_levels=5, base_res=16, max_res=256))
    assert res.tolist() == [16, 32, 64, 128, 256]
    # N_min = N_max: every level equal
    res, *_ = ora.levels(ora.Config(n_levels=4, base_res=20, max_res=20))
    assert res.tolist() == [20] * 4


def test_level_sizes_and_offsets(ora):
    cfg = ora.Config(n_levels=16, log2_table=19, base_res=16, max_res=2048)
    res, dense, off, size, n = ora.levels(cfg)
    T = 1 << 19
    for l in range(16):
        nv = (int(res[l]) + 1) ** 3
        assert dense[l] == (nv <= T)
        assert size[l] == (nv if nv <= T else T)
    assert off[0] == 0 and np.all(off[1:] == np.cumsum(size)[:-1]) and n == int(size.sum())


def _py_hash(v0, v1, v2, T):
    """Instant-NGP spatial hash with Python integers (no fixed-width arithmetic)."""
    return ((v0 * 1) ^ (v1 * 2654435761) ^ (v2 * 805459861)) % (1 << 32) % T


def test_vertex_index_bruteforce(ora):
    cfg = ora.Config(n_levels=8, log2_table=14, base_res=16, max_res=256)
    res, dense, *_ = ora.levels(cfg)
    T = 1 << 14
    rng = np.random.default_rng(0)
    for l in range(8):
        N = int(res[l])
        vs = rng.integers(0, N + 1, size=(300, 3))
        for v in vs.tolist():
            got = ora.vertex_index(cfg, l, *v)
            if dense[l]:
                want = v[0] + (N + 1) * (v[1] + (N + 1) * v[2])
            else:
                want = _py_hash(v[0], v[1], v[2], T)
            assert got == want
    # every vertex of a tiny hashed level (forced collisions, T = 32)
    tiny = ora.Config(n_levels=1, log2_table=5, base_res=5, max_res=5)
    for v0 in range(6):
        for v1 in range(6):
            for v2 in range(6):
                assert ora.vertex_index(tiny, 0, v0, v1, v2) == _py_hash(v0, v1, v2, 32)


def test_encode_indices_bruteforce(ora):
    """Corner entries of the encoder (cell by one FP32 multiply, corner order c0 + 2c1 + 4c2,
    level offsets, clamping of x = 1) against a brute-force recomputation."""
    cfg = ora.Config(n_levels=8, log2_table=14, base_res=16, max_res=256)
    res, dense, off, size, n = ora.levels(cfg)
    rng = np.random.default_rng(1)
    xn = rng.random((200, 3)).astype(np.float32)
    xn[:10] = np.array([0.0, 1.0, 0.5], np.float32)   # faces of the unit cube
    xn[10:20] = 1.0
    table = rng.standard_normal(n * 2)
    enc, idx, w = ora.encode(cfg, table, xn, want_idx=True)
    T = 1 << 14
    for p in range(len(xn)):
        for l in range(8):
            N = int(res[l])
            pos = xn[p] * np.float32(N)            # numpy float32 multiply: IEEE single, RNE
            g = np.minimum(np.floor(pos).astype(np.int64), N - 1)
            f = (pos - g.astype(np.float32)).astype(np.float64)
            for c in range(8):
                cb = [(c >> k) & 1 for k in range(3)]
                v = [int(g[k]) + cb[k] for k in range(3)]
                loc = (v[0] + (N + 1) * (v[1] + (N + 1) * v[2])) if dense[l] else _py_hash(*v, T)
                assert idx[p, l, c] == off[l] + loc
                wt = np.prod([f[k] if cb[k] else 1 - f[k] for k in range(3)])
                assert w[p, l, c] == pytest.approx(wt, abs=1e-15)


@pytest.mark.parametrize("N,log2T", [(16, 14), (64, 10), (8, 5)])
def test_grid_vertices_return_exact_entries(ora, N, log2T):
    """At x = k/N with N a power of two, one corner has weight 1: the encoding equals the table
    entry bit for bit (dense and hashed levels)."""
    cfg = ora.Config(n_levels=1, log2_table=log2T, base_res=N, max_res=N)
    res, dense, off, size, n = ora.levels(cfg)
    rng = np.random.default_rng(2)
    table = rng.standard_normal(n * 2)
    ks = rng.integers(0, N + 1, size=(100, 3))
    xn = (ks / N).astype(np.float32)
    enc, idx, w = ora.encode(cfg, table, xn, want_idx=True)
    T = 1 << log2T
    for p in range(100):
        v = [int(k) for k in ks[p]]
        e = (v[0] + (N + 1) * (v[1] + (N + 1) * v[2])) if dense[0] else _py_hash(*v, T)
        assert enc[p, 0] == table[2 * e] and enc[p, 1] == table[2 * e + 1]


def test_affine_reproduction_on_dense_level(ora):
    """Trilinear interpolation reproduces an affine function of the vertex coordinates."""
    N = 20
    cfg = ora.Config(n_levels=1, log2_table=16, base_res=N, max_res=N)
    res, dense, off, size, n = ora.levels(cfg)
    assert dense[0]
    a = np.array([0.3, -1.7, 2.2]); b = 0.25
    table = np.zeros(n * 2)
    for e in range(n):
        v = np.array([e % (N + 1), (e // (N + 1)) % (N + 1), e // (N + 1) ** 2])
        table[2 * e] = a @ v + b
        table[2 * e + 1] = -(a @ v) + 3 * b
    xn = np.random.default_rng(3).random((500, 3)).astype(np.float32)
    enc = ora.encode(cfg, table, xn)
    pos = xn.astype(np.float32) * np.float32(N)
    np.testing.assert_allclose(enc[:, 0], pos.astype(np.float64) @ a + b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(enc[:, 1], -(pos.astype(np.float64) @ a) + 3 * b, rtol=0, atol=1e-12)


def test_encoding_continuous_across_cell_faces(ora):
    """Crossing a cell face changes the encoding by O(step), so an FP32 cell flip cannot break
    value parity."""
    cfg = ora.Config(n_levels=8, log2_table=14, base_res=16, max_res=256)
    res, dense, off, size, n = ora.levels(cfg)
    table = np.random.default_rng(4).standard_normal(n * 2)
    base = np.array([7 / 16, 0.31, 0.77], np.float32)     # on a face of level 0 (N = 16)
    lo = base.copy(); lo[0] = np.nextafter(base[0], np.float32(0))
    hi = base.copy(); hi[0] = np.nextafter(base[0], np.float32(1))
    e = ora.encode(cfg, table, np.stack([lo, base, hi]))
    assert np.max(np.abs(e[0] - e[2])) < 1e-4


# ---------------------------------------------------------------------------------------------
# LayerNorm + MLP against torch (float64, CPU) and invariants
# ---------------------------------------------------------------------------------------------

CFG_SMALL = dict(n_levels=8, log2_table=12, base_res=4, max_res=64, depth=3, width=16)


def _torch_field(ora, cfg, params, xn, enc_idx, enc_w):
    """mu(x) from torch primitives: gather with the oracle's (brute-force pinned) corner indices and
    weights, F.layer_norm, F.linear, relu, sigmoid.  Returns mu and the leaf parameter tensors."""
    _, nt, nd = ora.n_params(cfg)
    lay = ora.dense_layout(cfg)
    C = cfg.n_levels * cfg.feats
    p = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    table = p[:nt].view(-1, cfg.feats)
    d = p[nt:]

    def seg(name, shape):
        o, n = lay[name]
        return d[o:o + n].view(*shape)

    idx = torch.tensor(enc_idx.astype(np.int64))            # [P,L,8]
    w = torch.tensor(enc_w)                                  # [P,L,8]
    enc = (table[idx] * w[..., None]).sum(2).reshape(len(xn), C)
    if cfg.layernorm:
        z = F.layer_norm(enc, (C,), seg("ln_g", (C,)), seg("ln_b", (C,)), cfg.ln_eps)
    else:
        z = enc
    h = z
    for k in range(cfg.depth):
        fin = C if k == 0 else cfg.width
        h = torch.relu(F.linear(h, seg(f"W{k}", (cfg.width, fin)), seg(f"b{k}", (cfg.width,))))
    y = F.linear(h, seg("w_out", (1, cfg.width)), seg("b_out", (1,)))[:, 0]
    if cfg.out_act == 1:
        mu = y
    elif cfg.out_act == 2:
        mu = F.softplus(y)          # beta 1, threshold 20 (PyTorch's defaults)
    else:
        mu = cfg.mu_max * torch.sigmoid(y)
    return mu, p, enc, z


@pytest.mark.parametrize("layernorm", [1, 0])
def test_field_and_gradient_match_torch(ora, layernorm):
    cfg = ora.Config(**CFG_SMALL, layernorm=layernorm)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(5)
    params = rng.standard_normal(tot) * 0.5
    lay = ora.dense_layout(cfg)
    o, n = lay["ln_g"]; params[nt + o:nt + o + n] = 1 + 0.2 * rng.standard_normal(n)
    xn = rng.random((64, 3)).astype(np.float32)
    _, idx, w = ora.encode(cfg, params[:nt], xn, want_idx=True)
    mu, enc, z = ora.field(cfg, params, xn, want=True)
    tmu, tp, tenc, tz = _torch_field(ora, cfg, params, xn, idx, w)
    np.testing.assert_allclose(enc, tenc.detach().numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(z, tz.detach().numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(mu, tmu.detach().numpy(), rtol=1e-12, atol=1e-14)
    dmu = rng.standard_normal(64)
    g = ora.field_backward(cfg, params, xn, dmu)
    (tmu * torch.tensor(dmu)).sum().backward()
    tg = tp.grad.numpy()
    np.testing.assert_allclose(g, tg, rtol=1e-9, atol=1e-12 * np.abs(tg).max())


@pytest.mark.parametrize("out_act", [1, 2])
def test_output_activations_match_torch(ora, out_act):
    """Identity and softplus heads (the alternatives to mu_max * sigmoid) against torch's identity
    and F.softplus (beta 1, threshold 20) with autograd: the output bias is set so that the head's
    input y straddles the softplus threshold (points on both branches)."""
    cfg = ora.Config(**CFG_SMALL, out_act=out_act)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(25)
    params = rng.standard_normal(tot) * 0.5
    lay = ora.dense_layout(cfg)
    o, n = lay["ln_g"]; params[nt + o:nt + o + n] = 1 + 0.2 * rng.standard_normal(n)
    xn = rng.random((96, 3)).astype(np.float32)
    _, idx, w = ora.encode(cfg, params[:nt], xn, want_idx=True)
    # shift the head bias so that the median y sits at the softplus threshold
    ob = nt + lay["b_out"][0]
    params[ob] = 0.0
    cfg0 = ora.Config(**CFG_SMALL, out_act=1)
    y0 = ora.field(cfg0, params, xn)
    params[ob] = 20.0 - np.median(y0)
    mu = ora.field(cfg, params, xn)
    tmu, tp, _, _ = _torch_field(ora, cfg, params, xn, idx, w)
    y = y0 + params[ob]
    assert (y > 20).sum() >= 20 and (y <= 20).sum() >= 20
    np.testing.assert_allclose(mu, tmu.detach().numpy(), rtol=1e-13, atol=1e-15)
    dmu = rng.standard_normal(96)
    g = ora.field_backward(cfg, params, xn, dmu)
    (tmu * torch.tensor(dmu)).sum().backward()
    tg = tp.grad.numpy()
    np.testing.assert_allclose(g, tg, rtol=1e-9, atol=1e-12 * np.abs(tg).max())


def test_layernorm_invariants(ora):
    """Row mean of the normalised features is 0 and their mean square is v/(v + eps); adding a
    constant to every channel leaves the output unchanged."""
    cfg = ora.Config(**CFG_SMALL)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(6)
    params = np.zeros(tot)
    params[:nt] = rng.standard_normal(nt) * 1e-2
    lay = ora.dense_layout(cfg)
    o, n = lay["ln_g"]; params[nt + o:nt + o + n] = 1.0
    xn = rng.random((50, 3)).astype(np.float32)
    mu, enc, z = ora.field(cfg, params, xn, want=True)        # gain 1, bias 0: z = x_hat
    v = enc.var(axis=1)
    np.testing.assert_allclose(z.mean(1), 0, atol=1e-12)
    np.testing.assert_allclose((z ** 2).mean(1), v / (v + cfg.ln_eps), rtol=1e-10)
    shifted = params.copy(); shifted[:nt] += 0.125
    mu2, enc2, z2 = ora.field(cfg, shifted, xn, want=True)
    np.testing.assert_allclose(z2, z, atol=1e-9)


def test_layernorm_backward_invariants(ora):
    """With gain 1 the channel gradient of LayerNorm sums to zero for each point."""
    cfg = ora.Config(n_levels=4, log2_table=13, base_res=4, max_res=16, depth=1, width=8)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(7)
    params = rng.standard_normal(tot) * 0.3
    lay = ora.dense_layout(cfg)
    o, n = lay["ln_g"]; params[nt + o:nt + o + n] = 1.0
    res, dense, off, size, ne = ora.levels(cfg)
    assert all(dense)
    # one point at a grid vertex of every level (x = 0): channel gradient = table gradient there
    xn = np.zeros((1, 3), np.float32)
    g = ora.field_backward(cfg, params, xn, np.array([1.0]))
    gx = np.array([g[2 * off[l]: 2 * off[l] + 2] for l in range(4)]).ravel()
    assert abs(gx.sum()) < 1e-12 * max(1.0, np.abs(gx).max())


def test_zero_network_gives_constant_field(ora):
    """All weights zero, output bias b: mu = mu_max * sigmoid(b) everywhere."""
    cfg = ora.Config(**CFG_SMALL)
    tot, nt, nd = ora.n_params(cfg)
    params = np.zeros(tot)
    params[:nt] = np.random.default_rng(8).standard_normal(nt)
    params[-1] = 0.7
    mu = ora.field(cfg, params, np.random.default_rng(9).random((30, 3)).astype(np.float32))
    np.testing.assert_allclose(mu, cfg.mu_max / (1 + math.exp(-0.7)), rtol=1e-15)


# ---------------------------------------------------------------------------------------------
# Geometry, sampling and Eq. (1) against closed forms
# ---------------------------------------------------------------------------------------------

def _geom(n=65, V=8):
    return synth.cone_geometry(n, V)


def _world(xn, g):
    return xn.astype(np.float64) * np.array(g.vol) - np.array(g.vol) / 2


def test_central_ray_passes_through_origin(ora):
    g = _geom(65)
    centre = 32 * 65 + 32
    for a in [0.0, 0.7, 2.5]:
        hit, xn, delta = ora.ray_samples(g, a, centre, 64, np.full(64, 0.5, np.float32))
        assert hit
        w = _world(xn, g)
        dirn = np.array([math.cos(a), math.sin(a), 0.0])
        perp = w - np.outer(w @ dirn, dirn)
        assert np.abs(perp).max() < 1e-4          # FP32 rounding of the normalised coordinate
        # the central chord of a cube along a direction in the xy-plane
        chord = 256.0 / max(abs(math.cos(a)), abs(math.sin(a)))
        assert delta * 64 == pytest.approx(chord, rel=1e-12)


def test_mirror_rays_have_equal_chords(ora):
    """Pixels (r, c) and (n-1-r, n-1-c) are related by a half-turn about the central ray; when that
    ray runs along a symmetry axis of the box (a multiple of pi/4) both chords are equal."""
    g = _geom(64)
    rng = np.random.default_rng(10)
    for _ in range(20):
        r, c = rng.integers(0, 64, 2)
        a = float(rng.integers(0, 8)) * math.pi / 4
        j = np.full(16, 0.5, np.float32)
        h1, _, d1 = ora.ray_samples(g, a, int(r * 64 + c), 16, j)
        h2, _, d2 = ora.ray_samples(g, a, int((63 - r) * 64 + (63 - c)), 16, j)
        assert h1 == h2 and d1 == pytest.approx(d2, rel=1e-12)


def test_samples_follow_pixel_ray(ora):
    """Every sample lies on the line from the source to its pixel (closed-form pixel position)."""
    g = _geom(64)
    rng = np.random.default_rng(11)
    for _ in range(10):
        pix = int(rng.integers(0, 64 * 64)); v = int(rng.integers(0, 8))
        s, P = synth.source_and_pixels(g, v)
        jit = rng.random(32).astype(np.float32)
        hit, xn, delta = ora.ray_samples(g, float(g.angles[v]), pix, 32, jit)
        assert hit
        d = P[pix] - s; d /= np.linalg.norm(d)
        w = _world(xn, g) - s
        perp = w - np.outer(w @ d, d)
        assert np.abs(perp).max() < 2e-4
        t = w @ d
        assert np.all(np.diff(t) > 0)                 # ordered along the ray, one per bin
        k = np.floor((t - t[0]) / delta + jit[0]).astype(int)
        assert k.tolist() == list(range(32))
        # sample i sits at fraction jit[i] of its bin (stratified sampling with the given jitter)
        np.testing.assert_allclose((t - t[0]) / delta, np.arange(32) + jit - jit[0], atol=1e-3)


def test_constant_field_line_integral_closed_form(ora):
    """A constant field mu gives A = mu * (chord of the ray through the box), whatever the jitter
    (Eq. 1 with equal steps)."""
    g = _geom(48, 6)
    cfg = ora.Config(n_levels=4, log2_table=10, base_res=4, max_res=16, depth=2, width=8)
    tot, nt, nd = ora.n_params(cfg)
    params = np.zeros(tot); params[-1] = -0.3
    mu = cfg.mu_max / (1 + math.exp(0.3))
    rng = np.random.default_rng(12)
    pix, jit = synth.ray_batch(1, g.n_pix, 40, 16)
    for v in range(3):
        s, P = synth.source_and_pixels(g, v)
        _, A, _ = ora.ray_batch(cfg, g, params, float(g.angles[v]), np.zeros(g.n_pix, np.float32),
                                pix, jit, grad=False)
        d = P[pix] - s; d /= np.linalg.norm(d, axis=1, keepdims=True)
        # independent slab chord on the unit direction
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-128.0 - s) / d; t2 = (128.0 - s) / d
        tn = np.nanmax(np.minimum(t1, t2), axis=1); tf = np.nanmin(np.maximum(t1, t2), axis=1)
        chord = np.maximum(tf - tn, 0)
        np.testing.assert_allclose(A, mu * chord, rtol=1e-12, atol=1e-12)


def test_sampled_phantom_within_bin_bound(ora):
    """Sum of the analytic phantom at the samples, times delta, agrees with the closed-form chord
    integral within 2 * delta * sum_k mu_k (each ellipsoid boundary spoils at most two bins)."""
    g = _geom(32, 4)
    ph = synth.make_phantom(3, 5)
    A = synth.project(ph, g)
    rng = np.random.default_rng(13)
    for v in range(4):
        for pix in rng.integers(0, g.n_pix, 25).tolist():
            for N in (64, 512):
                jit = rng.random(N).astype(np.float32)
                hit, xn, delta = ora.ray_samples(g, float(g.angles[v]), pix, N, jit)
                est = synth.phantom_mu(ph, _world(xn, g)).sum() * delta
                bound = 2 * delta * ph.mu.sum() + 1e-6
                assert abs(est - A[v].ravel()[pix]) <= bound


def test_projector_sphere_chord():
    """Closed-form projector: a sphere of radius r at distance p from the ray gives 2 sqrt(r^2-p^2)."""
    ph = synth.Phantom(np.array([[0.0, 0.0, 0.0]]), np.array([[50.0, 50.0, 50.0]]),
                       np.eye(3)[None], np.array([1.0]))
    s = np.array([-1000.0, 0.0, 0.0])
    ps = np.array([0.0, 10.0, 30.0, 49.0, 60.0])
    d = np.stack([np.full(5, 1000.0), ps, np.zeros(5)], 1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    got = synth.chord_lengths(ph, s, d)
    dist = np.abs(np.cross(-s, d)[:, 2])
    want = 2 * np.sqrt(np.maximum(50.0 ** 2 - dist ** 2, 0))
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-9)


def test_projector_bruteforce_integration():
    ph = synth.make_phantom(4, 4)
    g = _geom(16, 2)
    A = synth.project(ph, g)
    s, P = synth.source_and_pixels(g, 1)
    for pix in [0, 37, 100, 200, 255]:
        d = P[pix] - s
        L = np.linalg.norm(d)
        n = 400000
        t = (np.arange(n) + 0.5) / n
        pts = s + np.outer(t, d)
        est = synth.phantom_mu(ph, pts).sum() * L / n
        assert abs(est - A[1].ravel()[pix]) < 2 * (L / n) * ph.mu.sum() * 4 + 1e-9


# ---------------------------------------------------------------------------------------------
# Full ray batch: torch autograd and central finite differences
# ---------------------------------------------------------------------------------------------

def test_ray_batch_gradient_matches_torch(ora):
    """Loss of Eq. (3) and its gradient against torch autograd of the same rendering built from
    library primitives at the oracle's (geometry-pinned) sample points."""
    cfg = ora.Config(**CFG_SMALL)
    g = _geom(32, 4)
    ph = synth.make_phantom(1, 4)
    A = synth.project(ph, g).astype(np.float32)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(14)
    params = rng.standard_normal(tot) * 0.2
    lay = ora.dense_layout(cfg); o, n = lay["ln_g"]; params[nt + o:nt + o + n] = 1.0
    pix, jit = synth.ray_batch(2, g.n_pix, 12, 16)
    v = 2
    loss, a, grad = ora.ray_batch(cfg, g, params, float(g.angles[v]), A[v], pix, jit)
    xs, deltas = [], []
    for r in range(12):
        hit, xn, dl = ora.ray_samples(g, float(g.angles[v]), int(pix[r]), 16, jit[r])
        xs.append(xn); deltas.append(dl)
    xs = np.concatenate(xs)
    _, idx, w = ora.encode(cfg, params[:nt], xs, want_idx=True)
    tmu, tp, _, _ = _torch_field(ora, cfg, params, xs, idx, w)
    tA = (tmu.view(12, 16) * torch.tensor(deltas, dtype=torch.float64)[:, None]).sum(1)
    tl = (tA - torch.tensor(A[v].ravel()[pix], dtype=torch.float64)).abs().mean()
    tl.backward()
    np.testing.assert_allclose(a, tA.detach().numpy(), rtol=1e-12)
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    tg = tp.grad.numpy()
    np.testing.assert_allclose(grad, tg, rtol=1e-9, atol=1e-12 * np.abs(tg).max())


def test_ray_batch_thread_count_invariance(ora):
    """Rays split over host threads: ray sums and the loss (summed in ray order) are bitwise the
    serial ones, the gradient (per-thread buffers added in thread order) agrees to rounding."""
    cfg = ora.Config(**CFG_SMALL)
    g = _geom(32, 4)
    A = synth.project(synth.make_phantom(1, 4), g).astype(np.float32)
    tot, nt, nd = ora.n_params(cfg)
    params = np.random.default_rng(26).standard_normal(tot) * 0.2
    pix, jit = synth.ray_batch(4, g.n_pix, 37, 16)
    out = {}
    for th in (1, 3, 8):
        ora.set_threads(th)
        try:
            out[th] = ora.ray_batch(cfg, g, params, float(g.angles[1]), A[1], pix, jit)
        finally:
            ora.set_threads(1)
    l1, a1, g1 = out[1]
    for th in (3, 8):
        l, a, gg = out[th]
        assert l == l1
        np.testing.assert_array_equal(a, a1)
        np.testing.assert_allclose(gg, g1, rtol=1e-12, atol=1e-15 * np.abs(g1).max())


def test_train_is_the_composed_schedule(ora):
    """ora_train over n steps equals the composition of its pinned parts: view of step t from the
    epoch permutation, Philox pixel and jitter draws of step t, Eq. (3) batch gradient from zero,
    then Adam with step index t + 1 (Sec. 3.1: one view per step, Adam).  Starts mid-epoch
    (t_start = 2 of V = 3 views) so the run crosses two epoch boundaries."""
    cfg = ora.Config(n_levels=4, log2_table=10, base_res=4, max_res=32, depth=2, width=16)
    g = synth.cone_geometry(24, 3)
    A = synth.project(synth.make_phantom(3, 5), g).astype(np.float32)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(27)
    p0 = rng.standard_normal(tot) * 0.1
    m0 = np.abs(rng.standard_normal(tot)) * 1e-4
    v0 = np.abs(rng.standard_normal(tot)) * 1e-7
    R, N, seed, t_start, n = 40, 16, 11, 2, 5
    p1, m1, v1 = p0.copy(), m0.copy(), v0.copy()
    losses = ora.train(cfg, g, g.angles, A, p1, m1, v1, t_start, n, R, N, seed)
    p2, m2, v2 = p0.copy(), m0.copy(), v0.copy()
    views = []
    for k in range(n):
        t = t_start + k
        view = ora.view_for_step(seed, t, g.n_views)
        views.append(view)
        pix, jit = ora.draw_rays(seed, t, g.n_pix, R, N)
        loss, _, grad = ora.ray_batch(cfg, g, p2, float(g.angles[view]), A[view], pix, jit)
        assert losses[k] == loss
        ora.adam(p2, grad, m2, v2, t + 1)
    assert sorted(views[1:4]) == [0, 1, 2]         # steps 3..5 are one whole epoch
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(m1, m2)
    np.testing.assert_array_equal(v1, v2)


def _fd_setup(ora):
    # one dense level (N = 2) and one hashed level (N = 5, T = 32: collisions forced)
    cfg = ora.Config(n_levels=2, log2_table=5, base_res=2, max_res=5, depth=2, width=8)
    res, dense, *_ = ora.levels(cfg)
    assert res.tolist() == [2, 5] and dense.tolist() == [True, False]
    g = _geom(16, 3)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(21)
    params = rng.standard_normal(tot) * 0.5
    lay = ora.dense_layout(cfg); o, n = lay["ln_g"]; params[nt + o:nt + o + n] += 1.0
    pix, jit = synth.ray_batch(3, g.n_pix, 4, 8)
    return cfg, g, params, pix, jit


def test_finite_differences_upstream_gradient(ora):
    """Central differences in FP64 of sum_r dA_r * A_r with respect to every parameter."""
    cfg, g, params, pix, jit = _fd_setup(ora)
    v, ang = 1, float(g.angles[1])
    proj = np.zeros(g.n_pix, np.float32)
    dA = np.array([0.7, -1.3, 0.4, 2.0])
    _, _, grad = ora.ray_batch(cfg, g, params, ang, proj, pix, jit, dA=dA)

    def f(p):
        _, a, _ = ora.ray_batch(cfg, g, p, ang, proj, pix, jit, grad=False)
        return float(dA @ a)

    fd = np.zeros_like(params)
    for i in range(len(params)):
        h = 1e-6 * max(1.0, abs(params[i]))
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd[i] = (f(pp) - f(pm)) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(grad - fd).max() <= 1e-7 * scale
    # the hashed level's table receives a gradient (collisions included)
    assert np.abs(grad[2 * 27:2 * (27 + 32)]).max() > 0


def test_finite_differences_l1_loss(ora):
    """Eq. (3) loss: central differences away from the kink of |.|."""
    cfg, g, params, pix, jit = _fd_setup(ora)
    ang = float(g.angles[0])
    _, a0, _ = ora.ray_batch(cfg, g, params, ang, np.zeros(g.n_pix, np.float32), pix, jit,
                             grad=False)
    proj = np.zeros(g.n_pix, np.float32)
    proj[pix] = (a0 + np.array([0.5, -0.5, 0.8, -0.9])).astype(np.float32)   # residuals far from 0
    loss, _, grad = ora.ray_batch(cfg, g, params, ang, proj, pix, jit)

    def f(p):
        return ora.ray_batch(cfg, g, p, ang, proj, pix, jit, grad=False)[0]

    idx = np.random.default_rng(5).choice(len(params), 120, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(params[i]))
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(grad[i] - fd) <= 1e-7 * max(1e-3, np.abs(grad).max())


# ---------------------------------------------------------------------------------------------
# Adam, volume rendering, PSNR, pre-training voxel loss
# ---------------------------------------------------------------------------------------------

def test_adam_first_step_closed_form(ora):
    rng = np.random.default_rng(15)
    g = rng.standard_normal(1000) * np.logspace(-9, 1, 1000)
    g[::7] = 0.0
    p0 = rng.standard_normal(1000)
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    ora.adam(p, g.copy(), m, v, 1)
    np.testing.assert_allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.all(p[::7] == p0[::7])


def test_adam_matches_torch(ora):
    rng = np.random.default_rng(16)
    p0 = rng.standard_normal(257)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(257), np.zeros(257)
    for t in range(1, 6):
        g = rng.standard_normal(257)
        ora.adam(p, g.copy(), m, v, t)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_render_volume_matches_field(ora):
    cfg = ora.Config(**CFG_SMALL)
    tot, nt, nd = ora.n_params(cfg)
    params = np.random.default_rng(17).standard_normal(tot) * 0.3
    vol = ora.render_volume(cfg, params, 5, 4, 3)
    z, y, x = 2, 1, 3
    pt = np.array([[(x + .5) / 5, (y + .5) / 4, (z + .5) / 3]], np.float32)
    assert vol[z, y, x] == ora.field(cfg, params, pt)[0]


def test_psnr_closed_forms(ora):
    gt = np.random.default_rng(18).random(1000) * 0.05
    assert math.isinf(ora.psnr(gt, gt))
    off = 1e-3
    assert ora.psnr(gt, gt + off) == pytest.approx(20 * math.log10(gt.max() / off), rel=1e-10)


def test_trilinear_reproduces_affine_and_voxels(ora):
    n = 9
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    vol = (0.5 * xx - 0.25 * yy + 0.125 * zz + 1.0).astype(np.float32)
    rng = np.random.default_rng(19)
    for _ in range(50):
        x = rng.uniform(0.5 / n, 1 - 0.5 / n, 3).astype(np.float32)
        u = x.astype(np.float64) * n - 0.5
        assert ora.trilinear(vol, x) == pytest.approx(0.5 * u[0] - 0.25 * u[1] + 0.125 * u[2] + 1,
                                                      abs=1e-12)
    x = np.array([(3 + .5) / n, (4 + .5) / n, (5 + .5) / n], np.float32)
    assert ora.trilinear(vol, x) == pytest.approx(vol[5, 4, 3], abs=1e-6)


def test_voxel_loss_finite_differences(ora):
    """Eq. (2) voxel loss over two tables with a shared network: central differences."""
    cfg = ora.Config(n_levels=2, log2_table=5, base_res=2, max_res=5, depth=2, width=8)
    tot, nt, nd = ora.n_params(cfg)
    K = 2
    rng = np.random.default_rng(20)
    params = np.concatenate([rng.standard_normal(K * nt) * 0.5, rng.standard_normal(nd) * 0.5])
    lay = ora.dense_layout(cfg); o, n = lay["ln_g"]; params[K * nt + o:K * nt + o + n] += 1.0
    vols = (rng.random((K, 6, 6, 6)) * 0.02).astype(np.float32)
    xn = rng.random((24, 3)).astype(np.float32)
    tid = np.arange(24) % K
    loss, mu, grad = ora.voxel_batch(cfg, params, vols, xn, tid)
    tg = np.array([ora.trilinear(vols[t], x) for t, x in zip(tid, xn)])
    assert loss == pytest.approx(np.abs(mu - tg).mean(), rel=1e-12)
    assert np.abs(mu - tg).min() > 1e-4
    for i in rng.choice(len(params), 80, replace=False):
        h = 1e-6 * max(1.0, abs(params[i]))
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd = (ora.voxel_batch(cfg, pp, vols, xn, tid, grad=False)[0]
              - ora.voxel_batch(cfg, pm, vols, xn, tid, grad=False)[0]) / (2 * h)
        assert abs(grad[i] - fd) <= 1e-7 * max(1e-3, np.abs(grad).max())


def test_init_params_distribution(ora):
    cfg = ora.Config(**CFG_SMALL)
    tot, nt, nd = ora.n_params(cfg)
    p = ora.init_params(cfg, 42)
    assert np.abs(p[:nt]).max() <= 1e-4 and np.abs(p[:nt]).max() > 0.9e-4
    lay = ora.dense_layout(cfg)
    o, n = lay["ln_g"]; assert np.all(p[nt + o:nt + o + n] == 1)
    o, n = lay["ln_b"]; assert np.all(p[nt + o:nt + o + n] == 0)
    o, n = lay["W1"]; assert np.abs(p[nt + o:nt + o + n]).max() <= 1 / math.sqrt(cfg.width)
    o, n = lay["W0"]; C = cfg.n_levels * cfg.feats
    assert np.abs(p[nt + o:nt + o + n]).max() <= 1 / math.sqrt(C)


@pytest.mark.parametrize("layernorm", [1, 0])
def test_field_from_features_pins(ora, layernorm):
    """The feature-to-attenuation mapping alone (Sec. 2.3, Fig. 3): composed with the encoder it is
    the field; with a zero network it is the constant mu_max sigmoid(b_out); with LayerNorm a shift
    of all channels of a point changes nothing (the mean is removed), without it the shift shows."""
    cfg = ora.Config(**CFG_SMALL, layernorm=layernorm)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(71)
    params = rng.standard_normal(tot) * 0.5
    x = rng.random((40, 3)).astype(np.float32)
    mu, enc, _ = ora.field(cfg, params, x, want=True)
    assert np.array_equal(ora.field_from_features(cfg, params, enc), mu)
    lay = ora.dense_layout(cfg)
    zero = params.copy()
    zero[nt:] = 0.0
    o, n = lay["ln_g"]
    zero[nt + o:nt + o + n] = 1.0
    b = 0.37
    zero[nt + lay["b_out"][0]] = b
    feats = rng.standard_normal((25, enc.shape[1]))
    want = 0.25 / (1.0 + np.exp(-b))
    assert np.allclose(ora.field_from_features(cfg, zero, feats), want, rtol=0, atol=1e-15)
    shifted = ora.field_from_features(cfg, params, enc + 0.3)
    if layernorm:
        assert np.allclose(shifted, mu, rtol=1e-12, atol=1e-15)
    else:
        assert np.abs(shifted - mu).max() > 1e-6


def _ssim_scipy(gt, pred):
    """3-D SSIM through scipy.ndimage.gaussian_filter (sigma 1.5, radius 5), cropped to the voxels
    whose window lies inside the volume: an independent implementation of the filtering."""
    from scipy.ndimage import gaussian_filter
    f = lambda v: gaussian_filter(v, sigma=1.5, truncate=5.0 / 1.5, mode="constant")[5:-5, 5:-5, 5:-5]
    L = gt.max()
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    ma, mb = f(gt), f(pred)
    va, vb, cab = f(gt * gt) - ma * ma, f(pred * pred) - mb * mb, f(gt * pred) - ma * mb
    return float(np.mean((2 * ma * mb + c1) * (2 * cab + c2) / ((ma * ma + mb * mb + c1) * (va + vb + c2))))


def test_ssim_pins(ora):
    """SSIM (Wang et al. 2004, named in Sec. 3.1) over volumes: 1 for identical volumes, symmetric, and
    equal to a scipy gaussian_filter computation of the same definition."""
    rng = np.random.default_rng(81)
    z, y, x = np.meshgrid(np.arange(14), np.arange(17), np.arange(20), indexing="ij")
    gt = 0.02 + 0.01 * np.sin(x / 3.0) * np.cos(y / 4.0) + 0.005 * z / 14 + 0.002 * rng.random(x.shape)
    pred = gt + 0.003 * rng.standard_normal(gt.shape)
    assert ora.ssim(gt, gt) == pytest.approx(1.0, abs=1e-12)
    s = ora.ssim(gt, pred)
    assert 0.0 < s < 1.0
    assert s == pytest.approx(_ssim_scipy(gt, pred), rel=1e-10)
    # symmetric in everything but L = max(gt): with equal maxima the two orders agree
    p2 = pred.copy()
    p2[0, 0, 0] = gt.max() + 1.0
    g2 = gt.copy()
    g2[0, 0, 0] = gt.max() + 1.0
    assert ora.ssim(g2, p2) == pytest.approx(ora.ssim(p2, g2), rel=1e-12)
    assert np.isnan(ora.ssim(gt[:10], pred[:10]))


@pytest.mark.parametrize("layernorm", [1, 0])
def test_channel_mask_pins(ora, layernorm):
    """Channel mask before LayerNorm (Sec. 2.3, masking noisy channels): an all-ones mask changes
    nothing; masking channel (l, f) is the same field as zeroing feature f of every entry of level l,
    and the masked channel's table entries receive no gradient."""
    import dataclasses
    cfg = ora.Config(**CFG_SMALL, layernorm=layernorm)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(91)
    params = rng.standard_normal(tot) * 0.5
    x = rng.random((30, 3)).astype(np.float32)
    C_ = cfg.n_levels * cfg.feats
    ones = dataclasses.replace(cfg, mask=tuple([1.0] * C_))
    assert np.array_equal(ora.field(ones, params, x), ora.field(cfg, params, x))
    drop = [3, 10]
    mcfg = dataclasses.replace(cfg, mask=tuple(0.0 if i in drop else 1.0 for i in range(C_)))
    res, dense, off, size, n = ora.levels(cfg)
    zeroed = params.copy()
    for i in drop:
        l, f = divmod(i, cfg.feats)
        zeroed[2 * off[l] + f:2 * (off[l] + size[l]):2] = 0.0
    assert np.allclose(ora.field(mcfg, params, x), ora.field(cfg, zeroed, x), rtol=0, atol=1e-15)
    dmu = rng.standard_normal(30)
    g = ora.field_backward(mcfg, params, x, dmu)
    for i in drop:
        l, f = divmod(i, cfg.feats)
        assert np.all(g[2 * off[l] + f:2 * (off[l] + size[l]):2] == 0.0)
    gz = ora.field_backward(cfg, zeroed, x, dmu)
    assert np.allclose(g[nt:], gz[nt:], rtol=1e-12, atol=1e-15)


def test_channel_spectrum_pins(ora):
    """FFT noise measure of the encoder channels (Sec. 2.3): a table of independent random entries
    reads as white noise (high-band share near 1 - 1/8 = 0.875); a dense level holding one cosine
    period along x over its vertices has all its power at |k| = 1, so its high-band share is 0."""
    cfg = ora.Config(n_levels=8, log2_table=14, base_res=8, max_res=64, depth=2, width=16)
    tot, nt, nd = ora.n_params(cfg)
    rng = np.random.default_rng(95)
    hf = ora.channel_hf_fraction(cfg, rng.standard_normal(nt), g_max=32)
    res, dense, off, size, n = ora.levels(cfg)
    for l in range(cfg.n_levels):
        if min(32, res[l]) >= 16:
            assert 0.8 < hf[2 * l] < 0.95 and 0.8 < hf[2 * l + 1] < 0.95, (l, hf[2 * l:2 * l + 2])
    table = np.zeros(nt)
    for l in range(cfg.n_levels):
        if not dense[l]:
            continue
        N = int(res[l])
        v = np.arange((N + 1) ** 3)
        v0 = v % (N + 1)
        table[2 * (off[l] + v)] = np.cos(2 * np.pi * v0 / N)
        table[2 * (off[l] + v) + 1] = np.sin(2 * np.pi * v0 / N)
    hf = ora.channel_hf_fraction(cfg, table, g_max=32)
    checked = 0
    for l in range(cfg.n_levels):
        if dense[l] and res[l] <= 32:
            assert hf[2 * l] < 1e-12 and hf[2 * l + 1] < 1e-12, (l, hf[2 * l:2 * l + 2])
            checked += 1
    assert checked >= 2
