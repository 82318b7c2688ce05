"""Seeded synthetic inputs: cone-beam geometry, ellipsoid phantoms, measured projections.

The paper measures on real CT datasets projected with TIGRE (Sec. 3.1, Data); none are available,
so random ellipsoid phantoms with closed-form line integrals stand in for them.  This module holds
none of the method's arithmetic: it produces the measurement (projections of an analytic phantom,
with optional Poisson noise), the ground-truth volume for PSNR, and the explicit random draws
(ray pixels, jitter, initial parameters) that parity tests hand to both the GPU path and the
oracle.  It is shared by both sides and by the benchmark.

Geometry convention (all lengths in mm, rotation about z):
  source s = DSO (cos a, sin a, 0); detector centre -(DSD - DSO)(cos a, sin a, 0);
  detector axes e_u = (-sin a, cos a, 0), e_v = (0, 0, 1);
  pixel (row r, column c) centre at u = ((c + 1/2) - nu/2) du + off_u, v = ((r + 1/2) - nv/2) dv + off_v;
  projection layout [view][row][column]; the reconstruction box [-vol/2, vol/2] is centred at 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ------------------------------------------------------------------------------------------------
# Geometry and configurations
# ------------------------------------------------------------------------------------------------


@dataclass
class Geometry:
    dso: float = 1000.0
    dsd: float = 1500.0
    nu: int = 64
    nv: int = 64
    du: float = 6.0
    dv: float = 6.0
    off_u: float = 0.0
    off_v: float = 0.0
    vol: tuple = (256.0, 256.0, 256.0)
    angles: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n_views(self) -> int:
        return int(len(self.angles))

    @property
    def n_pix(self) -> int:
        return self.nu * self.nv


def cone_geometry(n_det: int, n_views: int, box_mm: float = 256.0) -> Geometry:
    """Full 360-degree orbit, square detector whose pitch 384/n mm covers the box magnified 1.5x."""
    pitch = 384.0 / n_det
    ang = 2.0 * math.pi * np.arange(n_views, dtype=np.float64) / n_views
    return Geometry(1000.0, 1500.0, n_det, n_det, pitch, pitch, 0.0, 0.0,
                    (box_mm, box_mm, box_mm), ang)


@dataclass
class Workload:
    """One named workload: phantom, scan and encoder/network/batch sizes."""
    name: str
    grid: int              # ground-truth volume edge (voxels)
    n_ellipsoids: int
    seed: int
    n_views: int
    n_det: int
    noise_i0: float        # 0 = noiseless
    n_levels: int
    feats: int
    log2_table: int
    base_res: int
    max_res: int
    depth: int
    width: int
    samples: int           # N per ray
    rays: int              # R per step
    precision: int = 0     # 0 FP32, 1 BF16 MLP + FP16 table with FP32 master


WORKLOADS = {
    "tiny64": Workload("tiny64", 64, 6, 1, 50, 64, 0.0, 8, 2, 14, 16, 256, 3, 32, 64, 1024),
    "ct256": Workload("ct256", 256, 20, 2, 50, 256, 1e5, 16, 2, 19, 16, 2048, 4, 32, 192, 2048),
    "tiny64_mixed": Workload("tiny64_mixed", 64, 6, 1, 50, 64, 0.0, 8, 2, 14, 16, 256, 3, 32, 64,
                             1024, precision=1),
    "ct512": Workload("ct512", 512, 40, 5, 100, 512, 1e5, 16, 2, 21, 16, 2048, 4, 32, 320, 8192,
                      precision=1),
}

# ------------------------------------------------------------------------------------------------
# Ellipsoid phantoms
# ------------------------------------------------------------------------------------------------


@dataclass
class Phantom:
    centers: np.ndarray   # [K,3] mm
    axes: np.ndarray      # [K,3] semi-axes mm
    rot: np.ndarray       # [K,3,3] columns = ellipsoid axes in world frame
    mu: np.ndarray        # [K] attenuation 1/mm


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def make_phantom(seed: int, K: int, support: float = 120.0, mu_lo: float = 0.01,
                 mu_hi: float = 0.05) -> Phantom:
    """K random ellipsoids inside a support sphere; attenuations add where they overlap.

    Semi-axes U[0.05, 0.35]*support; centre uniform in the ball of radius support - max(axes);
    orientation uniform (random unit quaternion, Shoemake); mu U[mu_lo, mu_hi] per mm.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    C = np.zeros((K, 3)); A = np.zeros((K, 3)); Rm = np.zeros((K, 3, 3)); M = np.zeros(K)
    for k in range(K):
        a = rng.uniform(0.05, 0.35, 3) * support
        rad = support - a.max()
        while True:
            c = rng.uniform(-rad, rad, 3)
            if c @ c <= rad * rad:
                break
        u1, u2, u3 = rng.uniform(0.0, 1.0, 3)
        q = (math.sqrt(1 - u1) * math.sin(2 * math.pi * u2), math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
             math.sqrt(u1) * math.sin(2 * math.pi * u3), math.sqrt(u1) * math.cos(2 * math.pi * u3))
        C[k] = c; A[k] = a; Rm[k] = _quat_to_rot(q); M[k] = rng.uniform(mu_lo, mu_hi)
    return Phantom(C, A, Rm, M)


def phantom_mu(ph: Phantom, pts: np.ndarray) -> np.ndarray:
    """mu at world points [...,3] (a point on an ellipsoid surface counts as inside)."""
    shp = pts.shape[:-1]
    p = pts.reshape(-1, 3)
    out = np.zeros(p.shape[0])
    for k in range(len(ph.mu)):
        loc = (p - ph.centers[k]) @ ph.rot[k] / ph.axes[k]
        out += ph.mu[k] * (np.einsum("ij,ij->i", loc, loc) <= 1.0)
    return out.reshape(shp)


def voxelize(ph: Phantom, n: int, box_mm: float = 256.0) -> np.ndarray:
    """Ground-truth volume [z][y][x] of mu at voxel centres -box/2 + (i + 1/2) box/n."""
    vol = np.zeros((n, n, n), np.float64)
    h = box_mm / n
    coords = -box_mm / 2 + (np.arange(n) + 0.5) * h
    for k in range(len(ph.mu)):
        r = ph.axes[k].max()
        lo = np.searchsorted(coords, ph.centers[k] - r - h)
        hi = np.searchsorted(coords, ph.centers[k] + r + h)
        xs, ys, zs = coords[lo[0]:hi[0]], coords[lo[1]:hi[1]], coords[lo[2]:hi[2]]
        if len(xs) == 0 or len(ys) == 0 or len(zs) == 0:
            continue
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        pts = np.stack([X, Y, Z], -1) - ph.centers[k]
        loc = pts @ ph.rot[k] / ph.axes[k]
        inside = np.einsum("...i,...i->...", loc, loc) <= 1.0
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += ph.mu[k] * inside
    return vol


# ------------------------------------------------------------------------------------------------
# Closed-form projector (stand-in for TIGRE) and noise
# ------------------------------------------------------------------------------------------------


def source_and_pixels(g: Geometry, view: int):
    """Source position [3] and pixel centres [nv*nu, 3] (pixel index r*nu + c) of one view."""
    a = float(g.angles[view])
    ca, sa = math.cos(a), math.sin(a)
    s = np.array([g.dso * ca, g.dso * sa, 0.0])
    back = g.dsd - g.dso
    r, c = np.divmod(np.arange(g.n_pix), g.nu)
    u = ((c + 0.5) - 0.5 * g.nu) * g.du + g.off_u
    v = ((r + 0.5) - 0.5 * g.nv) * g.dv + g.off_v
    P = np.stack([-back * ca - u * sa, -back * sa + u * ca, v], -1)
    return s, P


def chord_lengths(ph: Phantom, s: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Line integral of the phantom along full lines s + l*d (d unit, [n,3]); source outside."""
    out = np.zeros(d.shape[0])
    for k in range(len(ph.mu)):
        Ainv = ph.rot[k] / ph.axes[k]          # world -> unit-sphere frame: (x - c) @ Ainv
        u = (s - ph.centers[k]) @ Ainv
        w = d @ Ainv
        al = np.einsum("ij,ij->i", w, w)
        be = 2.0 * (w @ u)
        ga = u @ u - 1.0
        D = be * be - 4.0 * al * ga
        out += ph.mu[k] * np.where(D > 0, np.sqrt(np.maximum(D, 0.0)) / al, 0.0)
    return out


def project(ph: Phantom, g: Geometry) -> np.ndarray:
    """Noiseless line integrals A = -ln(I/I0) = sum_k mu_k * chord_k, float64 [V][nv][nu]."""
    out = np.zeros((g.n_views, g.nv, g.nu))
    for v in range(g.n_views):
        s, P = source_and_pixels(g, v)
        d = P - s
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        out[v] = chord_lengths(ph, s, d).reshape(g.nv, g.nu)
    return out


def add_poisson(A: np.ndarray, i0: float, seed: int) -> np.ndarray:
    """Counts I ~ Poisson(I0 exp(-A)); measured A = -ln(max(I, 1)/I0)."""
    rng = np.random.default_rng(np.random.PCG64(seed + 7919))
    I = rng.poisson(i0 * np.exp(-A))
    return -np.log(np.maximum(I, 1) / i0)


# ------------------------------------------------------------------------------------------------
# Explicit random draws for parity (given to both the GPU path and the oracle as data)
# ------------------------------------------------------------------------------------------------


def ray_batch(seed: int, n_pix: int, R: int, N: int):
    """R distinct pixel indices (uniform without replacement) and jitter in [0,1) on a 2^-24 grid."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    pix = rng.choice(n_pix, size=R, replace=False).astype(np.int32)
    jit = (rng.integers(0, 1 << 24, size=(R, N)) * (1.0 / (1 << 24))).astype(np.float32)
    return pix, jit


def init_params(n_entries: int, feats: int, dense_layout: dict, depth: int, seed: int,
                table_scale: float = 1e-4):
    """Initial values as float32: table U(-s, s); linear layers U(+-1/sqrt(fan_in)); LN 1 / 0.

    dense_layout maps names (ln_g, ln_b, W0, b0, ..., w_out, b_out) to (offset, size) and 'n'.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    table = rng.uniform(-table_scale, table_scale, n_entries * feats)
    dense = np.zeros(dense_layout["n"])
    C = dense_layout["ln_g"][1]
    W = dense_layout["b0"][1]
    o, n = dense_layout["ln_g"]; dense[o:o + n] = 1.0
    for k in range(depth):
        fin = C if k == 0 else W
        for nm in (f"W{k}", f"b{k}"):
            o, n = dense_layout[nm]
            dense[o:o + n] = rng.uniform(-1, 1, n) / math.sqrt(fin)
    for nm in ("w_out", "b_out"):
        o, n = dense_layout[nm]
        dense[o:o + n] = rng.uniform(-1, 1, n) / math.sqrt(W)
    return np.concatenate([table, dense]).astype(np.float32)


def scan(w: Workload, seed_offset: int = 0):
    """Phantom, geometry, measured projections (float32) and ground-truth volume of a workload."""
    ph = make_phantom(w.seed + seed_offset, w.n_ellipsoids)
    g = cone_geometry(w.n_det, w.n_views)
    A = project(ph, g)
    if w.noise_i0 > 0:
        A = add_poisson(A, w.noise_i0, w.seed + seed_offset)
    return ph, g, A.astype(np.float32)
