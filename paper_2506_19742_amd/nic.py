"""ctypes binding of libnic (include/nic.h) with the same entry-point names.

Only argument marshalling lives here: every step of the training path runs in the HIP kernels of
libnic.so.  Loading fails loudly when the library has not been built; there is no fallback.
PyTorch provides device memory (one uint8 workspace tensor) and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnic.so")

NIC_OK, NIC_EINVAL, NIC_ENOMEM, NIC_EHIP, NIC_ENONFINITE, NIC_EVERSION, NIC_ESTATE = 0, -1, -2, -3, -4, -5, -6


class NicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libnic status {status}: {msg}")
        self.status = status


class nic_geometry(C.Structure):
    _fields_ = [("dso", C.c_double), ("dsd", C.c_double), ("det_nu", C.c_int32), ("det_nv", C.c_int32),
                ("det_du", C.c_double), ("det_dv", C.c_double), ("det_off_u", C.c_double),
                ("det_off_v", C.c_double), ("vol_size", C.c_double * 3), ("n_views", C.c_int32),
                ("pad_", C.c_int32), ("angles_rad", C.POINTER(C.c_double))]


class nic_config(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("feats_per_level", C.c_int32), ("log2_table", C.c_int32),
                ("base_res", C.c_int32), ("max_res", C.c_int32), ("mlp_depth", C.c_int32),
                ("mlp_width", C.c_int32), ("out_act", C.c_int32), ("samples_per_ray", C.c_int32),
                ("rays_per_step", C.c_int32), ("layernorm", C.c_int32), ("precision", C.c_int32),
                ("n_tables", C.c_int32), ("pad_", C.c_int32), ("mu_max", C.c_double), ("ln_eps", C.c_double), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("seed", C.c_uint64)]


class nic_layout(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("res", C.c_int32 * 16), ("dense", C.c_int32 * 16),
                ("offset", C.c_int64 * 16), ("n_entries", C.c_int64), ("n_table", C.c_int64),
                ("n_dense", C.c_int64), ("dense_offset", C.c_int64), ("n_params_padded", C.c_int64),
                ("bin_shift", C.c_int32), ("n_bins", C.c_int32)]


class nic_tensor(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("numel", C.c_int64), ("dtype", C.c_int32), ("pad_", C.c_int32)]


# Every symbol declared in include/nic.h (checked by the CPU test suite).
EXPORTS = ["nic_describe", "nic_workspace_size", "nic_create", "nic_destroy", "nic_last_error",
           "nic_set_projections", "nic_tensors", "nic_sync_params", "nic_init_params", "nic_step",
           "nic_train", "nic_view_for_step", "nic_draw_rays", "nic_forward", "nic_backward",
           "nic_adam", "nic_zero_grad", "nic_query", "nic_render_volume", "nic_encode",
           "nic_get_step", "nic_set_timing", "nic_kernel_times", "nic_voxel_step",
           "nic_set_encoder_placement", "nic_encoder_level_major", "nic_voxel_train", "nic_set_volumes", "nic_export_mlp", "nic_import_mlp", "nic_psnr",
           "nic_save_state", "nic_load_state", "nic_field_from_features", "nic_ssim",
           "nic_set_channel_mask", "nic_channel_spectrum", "nic_sync", "nic_psnr_noalloc"]

_lib = None


def lib():
    """Loads libnic.so (raises if it is missing: build it with paper_2506_19742_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; run `python -m paper_2506_19742_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        sig = {
            "nic_describe": ([P(nic_config), P(nic_layout)], C.c_int32),
            "nic_workspace_size": ([P(nic_config), P(nic_geometry)], C.c_size_t),
            "nic_create": ([P(nic_config), P(nic_geometry), vp, vp, C.c_size_t, P(vp)], C.c_int32),
            "nic_destroy": ([vp], None),
            "nic_last_error": ([], C.c_char_p),
            "nic_set_projections": ([vp, vp], C.c_int32),
            "nic_tensors": ([vp, P(nic_tensor), P(C.c_int32)], C.c_int32),
            "nic_sync_params": ([vp], C.c_int32),
            "nic_init_params": ([vp, C.c_uint64], C.c_int32),
            "nic_step": ([vp, C.c_int32, vp, vp, vp], C.c_int32),
            "nic_train": ([vp, C.c_int32, P(C.c_float)], C.c_int32),
            "nic_view_for_step": ([vp, C.c_int64], C.c_int32),
            "nic_draw_rays": ([vp, C.c_int64, vp, vp], C.c_int32),
            "nic_forward": ([vp, C.c_int32, vp, vp, C.c_int32, vp], C.c_int32),
            "nic_backward": ([vp, C.c_int32, vp, vp, C.c_int32, vp], C.c_int32),
            "nic_adam": ([vp], C.c_int32),
            "nic_zero_grad": ([vp], C.c_int32),
            "nic_query": ([vp, vp, C.c_int64, vp], C.c_int32),
            "nic_render_volume": ([vp, P(C.c_int32), vp], C.c_int32),
            "nic_encode": ([vp, vp, C.c_int64, vp, vp], C.c_int32),
            "nic_get_step": ([vp], C.c_int64),
            "nic_set_timing": ([vp, C.c_int32], C.c_int32),
            "nic_set_encoder_placement": ([vp, C.c_int32], C.c_int32),
            "nic_encoder_level_major": ([vp], C.c_int32),
            "nic_kernel_times": ([vp, P(C.c_double), P(C.c_int64), P(C.c_int32)], C.c_int32),
            "nic_voxel_step": ([vp, vp, C.c_int32, vp], C.c_int32),
            "nic_voxel_train": ([vp, C.c_int32, C.c_int32, P(C.c_float)], C.c_int32),
            "nic_set_volumes": ([vp, vp, C.c_int32], C.c_int32),
            "nic_export_mlp": ([vp, vp, P(C.c_size_t)], C.c_int32),
            "nic_import_mlp": ([vp, vp, C.c_size_t], C.c_int32),
            "nic_psnr": ([vp, vp, vp, C.c_int64, P(C.c_double)], C.c_int32),
            "nic_save_state": ([vp, vp, P(C.c_size_t)], C.c_int32),
            "nic_load_state": ([vp, vp, C.c_size_t], C.c_int32),
            "nic_field_from_features": ([vp, vp, C.c_int64, vp], C.c_int32),
            "nic_ssim": ([vp, vp, vp, P(C.c_int32), P(C.c_double)], C.c_int32),
            "nic_set_channel_mask": ([vp, P(C.c_float), C.c_int32], C.c_int32),
            "nic_channel_spectrum": ([vp, C.c_int32, P(C.c_float)], C.c_int32),
            "nic_sync": ([vp], C.c_int32),
            "nic_psnr_noalloc": ([vp, vp, C.c_int64, vp, P(C.c_double)], C.c_int32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st: int):
    if st != NIC_OK:
        raise NicError(st, lib().nic_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


@dataclass
class Config:
    n_levels: int = 8
    feats_per_level: int = 2
    log2_table: int = 14
    base_res: int = 16
    max_res: int = 256
    mlp_depth: int = 3
    mlp_width: int = 32
    out_act: int = 0
    samples_per_ray: int = 64
    rays_per_step: int = 1024
    layernorm: int = 1
    precision: int = 0
    mu_max: float = 0.25
    ln_eps: float = 1e-5
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    seed: int = 0
    n_tables: int = 1

    def c(self) -> nic_config:
        return nic_config(self.n_levels, self.feats_per_level, self.log2_table, self.base_res,
                          self.max_res, self.mlp_depth, self.mlp_width, self.out_act,
                          self.samples_per_ray, self.rays_per_step, self.layernorm, self.precision,
                          self.n_tables, 0, self.mu_max, self.ln_eps, self.lr, self.beta1,
                          self.beta2, self.adam_eps, self.seed)


def config_for(w, **over) -> Config:
    """Config of a synthetic workload (paper_2506_19742_amd.synth.Workload)."""
    c = Config(w.n_levels, w.feats, w.log2_table, w.base_res, w.max_res, w.depth, w.width, 0,
               w.samples, w.rays, 1, w.precision)
    for k, v in over.items():
        setattr(c, k, v)
    return c


def geometry_struct(g):
    """nic_geometry from any object with dso, dsd, nu, nv, du, dv, off_u, off_v, vol, angles."""
    ang = np.ascontiguousarray(g.angles, dtype=np.float64)
    s = nic_geometry(g.dso, g.dsd, g.nu, g.nv, g.du, g.dv, g.off_u, g.off_v,
                     (C.c_double * 3)(*g.vol), len(ang), 0,
                     ang.ctypes.data_as(C.POINTER(C.c_double)))
    s._keep = ang
    return s


def nic_describe(cfg: Config) -> dict:
    out = nic_layout()
    _check(lib().nic_describe(C.byref(cfg.c()), C.byref(out)))
    L = out.n_levels
    return dict(res=list(out.res[:L]), dense=[bool(x) for x in out.dense[:L]],
                offset=list(out.offset[:L]), n_entries=out.n_entries, n_table=out.n_table,
                n_dense=out.n_dense, dense_offset=out.dense_offset,
                n_params_padded=out.n_params_padded, bin_shift=out.bin_shift, n_bins=out.n_bins)


def nic_workspace_size(cfg: Config, geom) -> int:
    n = lib().nic_workspace_size(C.byref(cfg.c()), C.byref(geometry_struct(geom)))
    if n == 0:
        raise NicError(NIC_EINVAL, lib().nic_last_error().decode())
    return int(n)


def psnr_noalloc(gt, pred, stream=None) -> float:
    """nic_psnr_noalloc: PSNR of two float32 device tensors of n <= 2^28 elements without a model
    (the library's static device scratch; allocates nothing)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(gt.device)
    out = C.c_double()
    _check(lib().nic_psnr_noalloc(_ptr(gt), _ptr(pred), gt.numel(), C.c_void_p(s.cuda_stream), C.byref(out)))
    return float(out.value)


class Model:
    """A model living in one torch uint8 workspace on cuda:0 (RAII around nic_create/destroy)."""

    def __init__(self, cfg: Config, geom, stream=None, device="cuda"):
        import torch
        self.cfg = cfg
        self.geom = geom
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws_bytes = nic_workspace_size(cfg, geom)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.layout = nic_describe(cfg)
        self.h = C.c_void_p()
        gs = geometry_struct(geom)
        _check(lib().nic_create(C.byref(cfg.c()), C.byref(gs), C.c_void_p(self.stream.cuda_stream),
                                _ptr(self.ws), self.ws_bytes, C.byref(self.h)))
        self.proj = None

    def close(self):
        if self.h:
            lib().nic_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- device views -------------------------------------------------------------------------
    def tensors(self):
        """(params, grads, adam_m, adam_v, table_f16 or None) as torch views of the workspace."""
        torch = self.torch
        arr = (nic_tensor * 8)()
        cnt = C.c_int32()
        _check(lib().nic_tensors(self.h, arr, C.byref(cnt)))
        base = self.ws.data_ptr()
        out = []
        for i in range(cnt.value):
            t = arr[i]
            if t.numel == 0:
                out.append(None)
                continue
            esz = 4 if t.dtype == 0 else 2
            off = t.ptr - base
            view = self.ws[off:off + t.numel * esz].view(torch.float32 if t.dtype == 0 else torch.float16)
            out.append(view)
        return tuple(out)

    def set_projections(self, proj):
        """Borrows proj (device float32 [n_views][nv][nu]); refused (NicError, NIC_ENONFINITE) when
        a value is not finite, and then the earlier projections stay in use."""
        _check(lib().nic_set_projections(self.h, _ptr(proj)))
        self.proj = proj

    def sync(self):
        """Synchronises the stream; raises NicError(NIC_ENONFINITE) when a training step since the
        last check met a non-finite value (the model was left as it was before that step)."""
        _check(lib().nic_sync(self.h))

    def sync_params(self):
        _check(lib().nic_sync_params(self.h))

    def init_params(self, seed: int):
        _check(lib().nic_init_params(self.h, seed))

    def step(self, view: int, pix=None, jitter=None, loss=None):
        _check(lib().nic_step(self.h, view, _ptr(pix), _ptr(jitter), _ptr(loss)))

    def train(self, n_steps: int, want_loss: bool = True):
        if want_loss:
            out = np.zeros(max(n_steps, 1), np.float32)
            st = lib().nic_train(self.h, n_steps, out.ctypes.data_as(C.POINTER(C.c_float)))
            _check(st)
            return out[:n_steps]
        _check(lib().nic_train(self.h, n_steps, None))
        return None

    def view_for_step(self, step: int) -> int:
        return int(lib().nic_view_for_step(self.h, step))

    def draw_rays(self, step: int):
        torch = self.torch
        R, N = self.cfg.rays_per_step, self.cfg.samples_per_ray
        pix = torch.empty(R, dtype=torch.int32, device=self.ws.device)
        jit = torch.empty((R, N), dtype=torch.float32, device=self.ws.device)
        _check(lib().nic_draw_rays(self.h, step, _ptr(pix), _ptr(jit)))
        return pix, jit

    def forward(self, view: int, pix, jitter):
        torch = self.torch
        a = torch.empty(pix.shape[0], dtype=torch.float32, device=self.ws.device)
        _check(lib().nic_forward(self.h, view, _ptr(pix), _ptr(jitter), pix.shape[0], _ptr(a)))
        return a

    def backward(self, view: int, pix, jitter, dA):
        _check(lib().nic_backward(self.h, view, _ptr(pix), _ptr(jitter), pix.shape[0], _ptr(dA)))

    def adam(self):
        _check(lib().nic_adam(self.h))

    def zero_grad(self):
        _check(lib().nic_zero_grad(self.h))

    def query(self, xn):
        torch = self.torch
        mu = torch.empty(xn.shape[0], dtype=torch.float32, device=self.ws.device)
        _check(lib().nic_query(self.h, _ptr(xn), xn.shape[0], _ptr(mu)))
        return mu

    def set_channel_mask(self, mask):
        """Channel mask before LayerNorm (sequence of n_levels * 2 floats), or None to remove it."""
        if mask is None:
            _check(lib().nic_set_channel_mask(self.h, None, 0))
            return
        arr = (C.c_float * len(mask))(*[float(v) for v in mask])
        _check(lib().nic_set_channel_mask(self.h, arr, len(mask)))

    def channel_spectrum(self, g_max: int = 64) -> np.ndarray:
        """High-band power fraction of every encoder channel (see nic_channel_spectrum)."""
        out = np.zeros(2 * self.cfg.n_levels, np.float32)
        _check(lib().nic_channel_spectrum(self.h, g_max, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def field_from_features(self, enc):
        """mu from given encoder outputs [n][2L] (LayerNorm + MLP + output activation only)."""
        torch = self.torch
        if enc.dim() != 2 or enc.shape[1] != 2 * self.cfg.n_levels or enc.dtype != torch.float32 \
                or not enc.is_contiguous():
            raise ValueError(f"enc must be contiguous float32 [n][{2 * self.cfg.n_levels}]")
        mu = torch.empty(enc.shape[0], dtype=torch.float32, device=self.ws.device)
        _check(lib().nic_field_from_features(self.h, _ptr(enc), enc.shape[0], _ptr(mu)))
        return mu

    def render_volume(self, nx: int, ny: int, nz: int):
        torch = self.torch
        vol = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.ws.device)
        dims = (C.c_int32 * 3)(nx, ny, nz)
        _check(lib().nic_render_volume(self.h, dims, _ptr(vol)))
        return vol

    def encode(self, xn, want_idx: bool = False):
        torch = self.torch
        n = xn.shape[0]
        L = self.cfg.n_levels
        enc = torch.empty((n, 2 * L), dtype=torch.float32, device=self.ws.device)
        idx = torch.empty((n, L, 8), dtype=torch.int32, device=self.ws.device) if want_idx else None
        _check(lib().nic_encode(self.h, _ptr(xn), n, _ptr(enc), _ptr(idx)))
        return (enc, idx) if want_idx else enc

    def get_step(self) -> int:
        return int(lib().nic_get_step(self.h))

    KERNEL_KINDS = ("rays", "forward", "backward", "encode", "adam", "bin_scan", "bin_reduce")

    ENCODER_PLACEMENTS = {"auto": 0, "level_major": 1, "in_forward": 2}

    def set_encoder_placement(self, placement: str):
        """Where ray training steps encode: "level_major" (a kernel of its own, one level per XCD at
        a time), "in_forward" (inside the forward kernel) or "auto" (the default: level-major when
        the table overflows an XCD's L2 and a level's table fits in about twice it).  The results
        are bitwise identical."""
        _check(lib().nic_set_encoder_placement(self.h, self.ENCODER_PLACEMENTS[placement]))

    def encoder_level_major(self) -> bool:
        return bool(lib().nic_encoder_level_major(self.h))

    def set_timing(self, enable: bool):
        _check(lib().nic_set_timing(self.h, 1 if enable else 0))

    def kernel_times(self):
        """{kind: (total_ms, launches)} since timing was enabled (synchronises the stream)."""
        ms = (C.c_double * 8)()
        calls = (C.c_int64 * 8)()
        cnt = C.c_int32()
        _check(lib().nic_kernel_times(self.h, ms, calls, C.byref(cnt)))
        return {self.KERNEL_KINDS[k]: (ms[k], int(calls[k])) for k in range(cnt.value)}

    # --- Mapping Consistency Initialization -----------------------------------------------------
    def set_volumes(self, vols):
        """Pre-training targets: device float32 [n_tables][n][n][n]."""
        self.vols = vols
        _check(lib().nic_set_volumes(self.h, _ptr(vols), int(vols.shape[-1])))

    def voxel_step(self, n_points: int, xn=None, loss=None):
        _check(lib().nic_voxel_step(self.h, _ptr(xn), n_points, _ptr(loss)))

    def voxel_train(self, n_steps: int, n_points: int, want_loss: bool = True):
        if want_loss:
            out = np.zeros(max(n_steps, 1), np.float32)
            _check(lib().nic_voxel_train(self.h, n_steps, n_points, out.ctypes.data_as(C.POINTER(C.c_float))))
            return out[:n_steps]
        _check(lib().nic_voxel_train(self.h, n_steps, n_points, None))
        return None

    def export_mlp(self) -> bytes:
        n = C.c_size_t()
        _check(lib().nic_export_mlp(self.h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(lib().nic_export_mlp(self.h, buf, C.byref(n)))
        return bytes(buf)

    def import_mlp(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        _check(lib().nic_import_mlp(self.h, buf, len(blob)))

    def save_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().nic_save_state(self.h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(lib().nic_save_state(self.h, buf, C.byref(n)))
        return bytes(buf)

    def load_state(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        _check(lib().nic_load_state(self.h, buf, len(blob)))

    def psnr(self, gt, pred) -> float:
        out = C.c_double()
        _check(lib().nic_psnr(self.h, _ptr(gt), _ptr(pred), gt.numel(), C.byref(out)))
        return float(out.value)

    def ssim(self, gt, pred) -> float:
        """3-D SSIM of two [nz][ny][nx] float32 device volumes (Gaussian window, see nic_ssim)."""
        torch = self.torch
        if gt.shape != pred.shape or gt.dim() != 3 or gt.dtype != torch.float32 or pred.dtype != torch.float32 \
                or not gt.is_contiguous() or not pred.is_contiguous():
            raise ValueError("gt and pred must be contiguous float32 volumes of the same [nz][ny][nx] shape")
        dims = (C.c_int32 * 3)(gt.shape[2], gt.shape[1], gt.shape[0])
        out = C.c_double()
        _check(lib().nic_ssim(self.h, _ptr(gt), _ptr(pred), dims, C.byref(out)))
        return float(out.value)

    # --- parameter helpers ------------------------------------------------------------------------
    def n_params(self):
        lay = self.layout
        return lay["n_table"], lay["n_dense"], lay["dense_offset"]

    def load_params(self, flat_params):
        """Sets parameters from a flat array in [table | dense] order (oracle layout)."""
        torch = self.torch
        p = self.tensors()[0]
        nt, nd, do = self.n_params()
        src = torch.as_tensor(np.asarray(flat_params, np.float32), device=p.device)
        p.zero_()
        p[:nt].copy_(src[:nt])
        p[do:do + nd].copy_(src[nt:nt + nd])
        self.sync_params()

    def flat(self, t):
        """[table | dense] view (oracle layout) of a params-shaped tensor, as float64 numpy."""
        nt, nd, do = self.n_params()
        a = t.detach().float().cpu().numpy()
        return np.concatenate([a[:nt], a[do:do + nd]]).astype(np.float64)
