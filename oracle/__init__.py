"""FP64 CPU oracle (test infrastructure only).

Thin ctypes wrapper over ``nic_oracle.c``: a plain, slow, FP64 reference of the training step of a
hash-encoded attenuation field for sparse-view cone-beam CT (Xu et al., "NeRF-based CBCT
Reconstruction needs Normalization and Initialization").  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the HIP library never does, and the two
share no code.  Each wrapped function names the passage its C implementation follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add, strict IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("feats", C.c_int32), ("log2_table", C.c_int32),
                ("base_res", C.c_int32), ("max_res", C.c_int32), ("depth", C.c_int32),
                ("width", C.c_int32), ("out_act", C.c_int32), ("layernorm", C.c_int32),
                ("masked", C.c_int32), ("mu_max", C.c_double), ("ln_eps", C.c_double),
                ("mask", C.c_double * 64)]


class Geom(C.Structure):
    _fields_ = [("dso", C.c_double), ("dsd", C.c_double), ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_double), ("dv", C.c_double), ("off_u", C.c_double),
                ("off_v", C.c_double), ("vol", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, f, i32, u32, i64 = (P(C.c_double), P(C.c_float), P(C.c_int32), P(C.c_uint32),
                               P(C.c_int64))
        L.ora_levels.argtypes = [P(Cfg), i32, i32, i64, i64, i64]
        L.ora_set_threads.argtypes = [C.c_int32]
        L.ora_get_threads.restype = C.c_int32
        L.ora_n_params.argtypes = [P(Cfg), i64, i64]
        L.ora_n_params.restype = C.c_int64
        L.ora_philox4x32_10.argtypes = [u32, u32, u32]
        L.ora_jitter.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.ora_jitter.restype = C.c_double
        L.ora_ray_pixel.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32]
        L.ora_ray_pixel.restype = C.c_int32
        L.ora_view_for_step.argtypes = [C.c_uint64, C.c_uint32, C.c_int32]
        L.ora_view_for_step.restype = C.c_int32
        L.ora_draw_rays.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int32, C.c_int32, i32, f]
        L.ora_init_params.argtypes = [P(Cfg), C.c_uint64, d]
        L.ora_voxel_points.argtypes = [C.c_uint64, C.c_uint32, C.c_int32, f]
        L.ora_vertex_index.argtypes = [P(Cfg), C.c_int, C.c_uint32, C.c_uint32, C.c_uint32]
        L.ora_vertex_index.restype = C.c_uint32
        L.ora_encode.argtypes = [P(Cfg), d, f, C.c_int64, d, u32, d]
        L.ora_field.argtypes = [P(Cfg), d, f, C.c_int64, d, d, d]
        L.ora_field_from_features.argtypes = [P(Cfg), d, d, C.c_int64, d]
        L.ora_ssim.argtypes = [d, d, C.c_int32, C.c_int32, C.c_int32]
        L.ora_ssim.restype = C.c_double
        L.ora_field_backward.argtypes = [P(Cfg), d, f, C.c_int64, d, d]
        L.ora_ray_samples.argtypes = [P(Geom), C.c_double, C.c_int32, C.c_int32, f, f, d]
        L.ora_ray_samples.restype = C.c_int
        L.ora_ray_batch.argtypes = [P(Cfg), P(Geom), d, C.c_double, f, C.c_int32, i32, C.c_int32,
                                    f, C.c_int32, d, d, d]
        L.ora_ray_batch.restype = C.c_double
        L.ora_adam.argtypes = [d, d, d, d, C.c_int64, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double]
        L.ora_train.argtypes = [P(Cfg), P(Geom), d, C.c_int32, f, d, d, d, C.c_int64, C.c_int32,
                                C.c_int32, C.c_int32, C.c_uint64, C.c_double, C.c_double,
                                C.c_double, C.c_double, d]
        L.ora_train.restype = C.c_int
        L.ora_render_volume.argtypes = [P(Cfg), d, C.c_int32, C.c_int32, C.c_int32, d]
        L.ora_psnr.argtypes = [d, d, C.c_int64]
        L.ora_psnr.restype = C.c_double
        L.ora_trilinear.argtypes = [f, C.c_int32, f]
        L.ora_trilinear.restype = C.c_double
        L.ora_voxel_batch.argtypes = [P(Cfg), d, C.c_int32, f, C.c_int32, C.c_int32, f, i32, d, d]
        L.ora_voxel_batch.restype = C.c_double
        _lib = L
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class Config:
    """Encoder + network configuration (mirrors the fields the method needs)."""
    n_levels: int = 8
    feats: int = 2
    log2_table: int = 14
    base_res: int = 16
    max_res: int = 256
    depth: int = 3
    width: int = 32
    out_act: int = 0
    layernorm: int = 1
    mu_max: float = 0.25
    ln_eps: float = 1e-5
    mask: tuple = ()          # per-channel mask before LayerNorm (Sec. 2.3); empty = none

    def c(self) -> Cfg:
        m = (C.c_double * 64)(*([float(v) for v in self.mask] + [1.0] * (64 - len(self.mask))))
        return Cfg(self.n_levels, self.feats, self.log2_table, self.base_res, self.max_res,
                   self.depth, self.width, self.out_act, self.layernorm, 1 if len(self.mask) else 0,
                   self.mu_max, self.ln_eps, m)


def geom_struct(g) -> Geom:
    """Accepts any object with dso, dsd, nu, nv, du, dv, off_u, off_v, vol attributes."""
    return Geom(g.dso, g.dsd, g.nu, g.nv, g.du, g.dv, g.off_u, g.off_v, (C.c_double * 3)(*g.vol))


def levels(cfg: Config):
    c = cfg.c()
    L = cfg.n_levels
    res = np.zeros(L, np.int32); dense = np.zeros(L, np.int32)
    off = np.zeros(L, np.int64); size = np.zeros(L, np.int64); n = np.zeros(1, np.int64)
    if lib().ora_levels(C.byref(c), _p(res, C.c_int32), _p(dense, C.c_int32), _p(off, C.c_int64),
                        _p(size, C.c_int64), _p(n, C.c_int64)) != 0:
        raise ValueError("invalid config")
    return res, dense.astype(bool), off, size, int(n[0])


def n_params(cfg: Config):
    nt = np.zeros(1, np.int64); nd = np.zeros(1, np.int64)
    tot = lib().ora_n_params(C.byref(cfg.c()), _p(nt, C.c_int64), _p(nd, C.c_int64))
    return int(tot), int(nt[0]), int(nd[0])


def dense_layout(cfg: Config):
    """Offsets (within the dense block) of ln_gain, ln_bias, W_k, b_k, w_out, b_out."""
    C_ = cfg.n_levels * cfg.feats
    W = cfg.width
    o = {}
    p = 0
    o["ln_g"] = (p, C_); p += C_
    o["ln_b"] = (p, C_); p += C_
    for k in range(cfg.depth):
        fin = C_ if k == 0 else W
        o[f"W{k}"] = (p, W * fin); p += W * fin
        o[f"b{k}"] = (p, W); p += W
    o["w_out"] = (p, W); p += W
    o["b_out"] = (p, 1); p += 1
    o["n"] = p
    return o


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32); k = np.asarray(key, np.uint32); out = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def draw_rays(seed: int, t: int, n_pix: int, R: int, N: int):
    pix = np.zeros(R, np.int32); jit = np.zeros((R, N), np.float32)
    lib().ora_draw_rays(seed, t, n_pix, R, N, _p(pix, C.c_int32), _p(jit, C.c_float))
    return pix, jit


def view_for_step(seed: int, t: int, V: int) -> int:
    return int(lib().ora_view_for_step(seed, t, V))


def voxel_points(seed: int, t: int, n: int):
    xn = np.zeros((n, 3), np.float32)
    lib().ora_voxel_points(seed, t, n, _p(xn, C.c_float))
    return xn


def init_params(cfg: Config, seed: int):
    tot, _, _ = n_params(cfg)
    p = np.zeros(tot, np.float64)
    lib().ora_init_params(C.byref(cfg.c()), seed, _p(p, C.c_double))
    return p


def vertex_index(cfg: Config, level: int, v0: int, v1: int, v2: int) -> int:
    return int(lib().ora_vertex_index(C.byref(cfg.c()), level, v0, v1, v2))


def encode(cfg: Config, table, xn, want_idx=False):
    xn = _c32(xn).reshape(-1, 3)
    table = _c64(table)
    n = xn.shape[0]
    Cc = cfg.n_levels * cfg.feats
    enc = np.zeros((n, Cc), np.float64)
    idx = np.zeros((n, cfg.n_levels, 8), np.uint32) if want_idx else None
    w = np.zeros((n, cfg.n_levels, 8), np.float64) if want_idx else None
    lib().ora_encode(C.byref(cfg.c()), _p(table, C.c_double), _p(xn, C.c_float), n,
                     _p(enc, C.c_double), _p(idx, C.c_uint32), _p(w, C.c_double))
    return (enc, idx, w) if want_idx else enc


def field(cfg: Config, params, xn, want=False):
    xn = _c32(xn).reshape(-1, 3)
    params = _c64(params)
    n = xn.shape[0]
    Cc = cfg.n_levels * cfg.feats
    mu = np.zeros(n, np.float64)
    enc = np.zeros((n, Cc), np.float64) if want else None
    z = np.zeros((n, Cc), np.float64) if want else None
    lib().ora_field(C.byref(cfg.c()), _p(params, C.c_double), _p(xn, C.c_float), n,
                    _p(mu, C.c_double), _p(enc, C.c_double), _p(z, C.c_double))
    return (mu, enc, z) if want else mu


def field_from_features(cfg: Config, params, enc):
    """mu from given encoder outputs [n][L*F] (LayerNorm + MLP + activation only)."""
    params = _c64(params)
    enc = _c64(enc).reshape(-1, cfg.n_levels * cfg.feats)
    mu = np.zeros(enc.shape[0], np.float64)
    lib().ora_field_from_features(C.byref(cfg.c()), _p(params, C.c_double), _p(enc, C.c_double),
                                  enc.shape[0], _p(mu, C.c_double))
    return mu


def channel_hf_fraction(cfg: Config, table, g_max: int = 64) -> np.ndarray:
    """FFT noise measure of every encoder channel (Sec. 2.3 masks channels found noisy with an FFT):
    for level l of resolution N, the channel's field at the G^3 vertices v0 + i of that level
    (G = min(g_max, N), v0 = (N - G) // 2, points (v0 + i) / N in FP32), numpy's 3-D FFT, and the
    power with max_d |k_d| > G/4 (signed frequencies) over all non-DC power."""
    res, dense, off, size, n = levels(cfg)
    out = np.zeros(cfg.n_levels * cfg.feats)
    for l in range(cfg.n_levels):
        N = int(res[l])
        G = min(g_max, N)
        v0 = (N - G) // 2
        iz, iy, ix = np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij")
        pts = np.stack([(np.float32(v0) + ix.astype(np.float32)) / np.float32(N),
                        (np.float32(v0) + iy.astype(np.float32)) / np.float32(N),
                        (np.float32(v0) + iz.astype(np.float32)) / np.float32(N)], -1).reshape(-1, 3)
        enc = encode(cfg, table, pts.astype(np.float32))
        f = np.fft.fftfreq(G) * G
        kz, ky, kx = np.meshgrid(np.abs(f), np.abs(f), np.abs(f), indexing="ij")
        high = np.maximum(np.maximum(kx, ky), kz) * 4 > G
        for c in range(cfg.feats):
            ch = l * cfg.feats + c
            P = np.abs(np.fft.fftn(enc[:, ch].reshape(G, G, G))) ** 2
            P[0, 0, 0] = 0.0
            tot = P.sum()
            out[ch] = P[high].sum() / tot if tot > 0 else 0.0
    return out


def ssim(gt, pred) -> float:
    """3-D SSIM of two [nz][ny][nx] volumes (Gaussian window sigma 1.5, 11 taps; L = max(gt))."""
    gt = _c64(gt)
    pred = _c64(pred)
    nz, ny, nx = gt.shape
    return float(lib().ora_ssim(_p(gt, C.c_double), _p(pred, C.c_double), nx, ny, nz))


def field_backward(cfg: Config, params, xn, dmu):
    xn = _c32(xn).reshape(-1, 3)
    params = _c64(params)
    dmu = _c64(dmu)
    g = np.zeros_like(params)
    lib().ora_field_backward(C.byref(cfg.c()), _p(params, C.c_double), _p(xn, C.c_float),
                             xn.shape[0], _p(dmu, C.c_double), _p(g, C.c_double))
    return g


def set_threads(n: int) -> None:
    """Host threads of ray_batch (1 = serial; each thread takes a contiguous range of rays)."""
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


def ray_samples(geom, angle: float, pix: int, N: int, jitter):
    jitter = _c32(jitter)
    xn = np.zeros((N, 3), np.float32)
    delta = np.zeros(1, np.float64)
    hit = lib().ora_ray_samples(C.byref(geom_struct(geom)), angle, pix, N, _p(jitter, C.c_float),
                                _p(xn, C.c_float), _p(delta, C.c_double))
    return bool(hit), xn, float(delta[0])


def ray_batch(cfg: Config, geom, params, angle: float, proj_view, pix, jitter, grad=True,
              dA=None):
    """Eq. (1) rendering of one view's rays; Eq. (3) loss (mode 0) or an upstream dA (mode 1)."""
    params = _c64(params)
    proj_view = _c32(proj_view)
    pix = _i32(pix)
    jitter = _c32(jitter)
    R = pix.shape[0]
    N = jitter.shape[1] if jitter.ndim == 2 else jitter.shape[0] // max(R, 1)
    a = np.zeros(R, np.float64)
    g = np.zeros_like(params) if grad else None
    mode = 0 if dA is None else 1
    dA_ = _c64(dA) if dA is not None else None
    loss = lib().ora_ray_batch(C.byref(cfg.c()), C.byref(geom_struct(geom)), _p(params, C.c_double),
                               angle, _p(proj_view, C.c_float), R, _p(pix, C.c_int32), N,
                               _p(jitter, C.c_float), mode, _p(dA_, C.c_double), _p(a, C.c_double),
                               _p(g, C.c_double))
    return loss, a, g


def adam(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place FP64 Adam on contiguous float64 arrays."""
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().ora_adam(_p(p, C.c_double), _p(g, C.c_double), _p(m, C.c_double), _p(v, C.c_double),
                   p.size, t, lr, b1, b2, eps)


def train(cfg: Config, geom, angles, proj, params, m, v, t_start: int, n_steps: int, R: int,
          N: int, seed: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    angles = _c64(angles)
    proj = _c32(proj)
    losses = np.zeros(n_steps, np.float64)
    rc = lib().ora_train(C.byref(cfg.c()), C.byref(geom_struct(geom)), _p(angles, C.c_double),
                         angles.shape[0], _p(proj, C.c_float), _p(params, C.c_double),
                         _p(m, C.c_double), _p(v, C.c_double), t_start, n_steps, R, N, seed, lr,
                         b1, b2, eps, _p(losses, C.c_double))
    if rc != 0:
        raise ValueError("oracle train failed")
    return losses


def render_volume(cfg: Config, params, nx: int, ny: int, nz: int):
    params = _c64(params)
    vol = np.zeros((nz, ny, nx), np.float64)
    lib().ora_render_volume(C.byref(cfg.c()), _p(params, C.c_double), nx, ny, nz,
                            _p(vol, C.c_double))
    return vol


def psnr(gt, pred) -> float:
    gt = _c64(gt).ravel(); pred = _c64(pred).ravel()
    return float(lib().ora_psnr(_p(gt, C.c_double), _p(pred, C.c_double), gt.size))


def trilinear(vol, x) -> float:
    vol = _c32(vol)
    x = _c32(x)
    return float(lib().ora_trilinear(_p(vol, C.c_float), vol.shape[0], _p(x, C.c_float)))


def voxel_batch(cfg: Config, params, vols, xn, tid, grad=True):
    """Eq. (2) voxel loss over points with per-point table id (K tables + shared LN/MLP)."""
    params = _c64(params)
    vols = _c32(vols)
    K, n = vols.shape[0], vols.shape[1]
    xn = _c32(xn).reshape(-1, 3)
    tid = _i32(tid)
    B = xn.shape[0]
    mu = np.zeros(B, np.float64)
    g = np.zeros_like(params) if grad else None
    loss = lib().ora_voxel_batch(C.byref(cfg.c()), _p(params, C.c_double), K, _p(vols, C.c_float),
                                 n, B, _p(xn, C.c_float), _p(tid, C.c_int32), _p(mu, C.c_double),
                                 _p(g, C.c_double))
    return loss, mu, g
