"""Seeded synthetic inputs for the ProbeSDF per-ray render step.

This module only *generates inputs*: camera rigs, pixel rays, node values of
analytic SDFs, random feature / probe grids and MLP initialisations.  It holds
none of the render step's arithmetic (no interpolation, spherical harmonics,
compositing or MLP evaluation), so both the HIP path and the FP64 oracle can be
fed from it without sharing any of the method.

Stand-ins for the paper's data (Sec. 5, Protocol): the paper measures on
MVMannequins, ActorsHQ, DTU and BlendedMVS.  None of those are used; every
array here is synthetic and seeded (numpy PCG64).

Conventions shared by every array:
  * grids are align-corners over [-1, 1]^3 with R nodes per axis, node (i, j, k)
    at (-1 + i*h, -1 + j*h, -1 + k*h), h = 2/(R-1), stored x fastest:
    flat index (k*R + j)*R + i;
  * spatial features  feat[R][R][R][n_feat];
  * probes            probes[P][P][P][n_sh][n_ang];
  * MLP               per hidden layer W_l[hidden][n_prev] row-major and b_l[hidden],
                      then Wo[3][hidden], bo[3] (one hidden layer: W1, b1, W2, b2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_FEAT = 3
N_ANG = 4
HIDDEN = 16
N_OUT = 3
N_IN = N_FEAT + N_ANG + 3  # F_s, F_a, (c, c^2, c^4)


# the paper's own colour model (Sec. 3.1 Eq. newparametrization, Sec. 4): incidence
# inputs (1 - n.v)^0..5 and two hidden layers of 32
PAPER_N_IN = N_FEAT + N_ANG + 6
PAPER_HIDDEN = 32
PAPER_LAYERS = 2


def mlp_size(n_in: int = N_IN, hidden: int = HIDDEN, n_out: int = N_OUT, layers: int = 1) -> int:
    n = 0
    for l in range(layers):
        n += hidden * (n_in if l == 0 else hidden) + hidden
    return n + n_out * hidden + n_out


# ----------------------------------------------------------------------------
# cameras and rays
# ----------------------------------------------------------------------------
@dataclass
class Camera:
    """Pinhole camera.  c2w[:, :3] holds the camera axes (x right, y down,
    z forward) in world coordinates, c2w[:, 3] the centre.  Pixel (px, py)
    has its centre at (px + 0.5, py + 0.5); its direction in camera space is
    ((px + 0.5 - cx)/fx, (py + 0.5 - cy)/fy, 1)."""
    c2w: np.ndarray  # (3, 4) float64
    fx: float
    fy: float
    cx: float
    cy: float

    def as_array(self) -> np.ndarray:
        """16 float32: c2w row-major (12), fx, fy, cx, cy."""
        return np.concatenate([self.c2w.reshape(-1),
                               [self.fx, self.fy, self.cx, self.cy]]).astype(np.float32)


def fibonacci_cameras(V: int, W: int, H: int, radius: float = 3.0,
                      fov_y_deg: float = 30.0) -> list[Camera]:
    """V cameras on a Fibonacci sphere of the given radius, each aimed at the
    origin with world-up +z; vertical field of view fov_y_deg."""
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    fy = (H / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    for k in range(V):
        z = 1.0 - (2.0 * k + 1.0) / V
        rxy = math.sqrt(max(0.0, 1.0 - z * z))
        phi = k * golden
        c = radius * np.array([rxy * math.cos(phi), rxy * math.sin(phi), z])
        fwd = -c / np.linalg.norm(c)
        right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
        right /= np.linalg.norm(right)
        down = np.cross(fwd, right)
        c2w = np.stack([right, down, fwd, c], axis=1)
        cams.append(Camera(c2w=c2w, fx=fy, fy=fy, cx=W / 2.0, cy=H / 2.0))
    return cams


def _pixel_order(W: int, H: int, order: str) -> tuple[np.ndarray, np.ndarray]:
    py, px = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    px, py = px.reshape(-1), py.reshape(-1)
    if order == "image":
        return px, py
    if order.startswith("tile"):
        t = int(order[4:])
        # row-major over t x t tiles, row-major inside each tile
        key = ((py // t) * ((W + t - 1) // t) + (px // t)) * (t * t) + (py % t) * t + (px % t)
        idx = np.argsort(key, kind="stable")
        return px[idx], py[idx]
    raise ValueError(f"unknown ray order {order!r}")


def camera_rays(cams: list[Camera], W: int, H: int, order: str = "image"):
    """Pixel-centre rays of every camera, camera-major.  Computed in float64,
    returned as float32 (B, 3) origins and unit directions."""
    px, py = _pixel_order(W, H, order)
    os, ds = [], []
    for cam in cams:
        dc = np.stack([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy,
                       np.ones_like(px, dtype=np.float64)], axis=1)
        dw = dc @ cam.c2w[:, :3].T
        dw /= np.linalg.norm(dw, axis=1, keepdims=True)
        os.append(np.broadcast_to(cam.c2w[:, 3], dw.shape))
        ds.append(dw)
    o = np.ascontiguousarray(np.concatenate(os).astype(np.float32))
    d = np.ascontiguousarray(np.concatenate(ds).astype(np.float32))
    return o, d


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------
def grid_nodes(R: int) -> np.ndarray:
    """Node coordinates (R, R, R, 3) in float64, index [k, j, i] -> (x_i, y_j, z_k)."""
    a = -1.0 + 2.0 * np.arange(R, dtype=np.float64) / (R - 1)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([x, y, z], axis=-1)


def sphere_sdf_nodes(R: int, radius: float = 0.5) -> np.ndarray:
    """Node values |p| - radius, in float64 rounded to float32 (RNE)."""
    a = -1.0 + 2.0 * np.arange(R, dtype=np.float64) / (R - 1)
    out = np.empty((R, R, R), dtype=np.float32)
    for k in range(R):
        z2 = a[k] * a[k]
        r = np.sqrt(a[None, :] ** 2 + a[:, None] ** 2 + z2)  # [j, i]
        out[k] = (r - radius).astype(np.float32)
    return out


def torus_sdf_nodes(R: int, major: float = 0.5, minor: float = 0.2) -> np.ndarray:
    """Torus about the z axis: sqrt((sqrt(x^2+y^2) - major)^2 + z^2) - minor."""
    a = -1.0 + 2.0 * np.arange(R, dtype=np.float64) / (R - 1)
    out = np.empty((R, R, R), dtype=np.float32)
    rxy = np.sqrt(a[None, :] ** 2 + a[:, None] ** 2)  # [j, i]
    for k in range(R):
        out[k] = (np.sqrt((rxy - major) ** 2 + a[k] ** 2) - minor).astype(np.float32)
    return out


def xavier_uniform_mlp(rng: np.random.Generator, n_in: int = N_IN, hidden: int = HIDDEN,
                       n_out: int = N_OUT, layers: int = 1) -> np.ndarray:
    """Packed [W_1 (hidden x n_in), b_1, ..., W_L (hidden x hidden), b_L, Wo (n_out x
    hidden), bo], Xavier-uniform weights (bound sqrt(6/(fan_in+fan_out))), zero
    biases; the matrices are drawn in that order."""
    parts = []
    fan = n_in
    for _ in range(layers):
        a = math.sqrt(6.0 / (fan + hidden))
        parts += [rng.uniform(-a, a, size=(hidden, fan)).reshape(-1), np.zeros(hidden)]
        fan = hidden
    a = math.sqrt(6.0 / (hidden + n_out))
    parts += [rng.uniform(-a, a, size=(n_out, hidden)).reshape(-1), np.zeros(n_out)]
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Field:
    """One scene: SDF grid, spatial features, probe grid and MLP, all float32
    (float16 copies are made by `to_half`)."""
    R: int
    P: int
    n_sh: int
    sdf: np.ndarray      # (R, R, R)
    feat: np.ndarray     # (R, R, R, n_feat)
    probes: np.ndarray   # (P, P, P, n_sh, n_ang)
    mlp: np.ndarray      # (mlp_size,)
    extra: dict = field(default_factory=dict)
    hidden: int = HIDDEN
    layers: int = 1


def random_field(seed: int, R: int, P: int, n_sh: int = 9, shape: str = "sphere",
                 std: float = 0.1, model: str = "workload") -> Field:
    """Draw order (seed -> PCG64): features, probes, then the MLP matrices (biases
    are zero).  model "workload": 10 -> 16 -> 3 (inputs F_s, F_a, c, c^2, c^4);
    "paper": 13 -> 32 -> 32 -> 3 (inputs F_s, F_a, (1 - n.v)^0..5)."""
    rng = np.random.default_rng(seed)
    feat = (rng.standard_normal((R, R, R, N_FEAT), dtype=np.float32) * np.float32(std))
    probes = (rng.standard_normal((P, P, P, n_sh, N_ANG), dtype=np.float32) * np.float32(std))
    if model == "workload":
        hidden, layers = HIDDEN, 1
        mlp = xavier_uniform_mlp(rng)
    elif model == "paper":
        hidden, layers = PAPER_HIDDEN, PAPER_LAYERS
        mlp = xavier_uniform_mlp(rng, PAPER_N_IN, hidden, N_OUT, layers)
    else:
        raise ValueError(model)
    if shape == "sphere":
        sdf = sphere_sdf_nodes(R)
    elif shape == "torus":
        sdf = torus_sdf_nodes(R)
    else:
        raise ValueError(shape)
    return Field(R=R, P=P, n_sh=n_sh, sdf=sdf, feat=feat, probes=probes, mlp=mlp, hidden=hidden,
                 layers=layers)


@dataclass
class Tiles:
    """Sparse tiles of 16^3 cells with tri-plane spatial features: index [T, T, T]
    (slot of each allocated tile, -1 empty) and planes [slots, 3, 16, 16, n_feat]
    (F_x over (y, z), F_y over (x, z), F_z over (x, y), row-major [v][u])."""
    T: int
    index: np.ndarray
    planes: np.ndarray


TILE = 16  # cells per tile edge


def tiled_field(seed: int, T: int, n_sh: int = 9, shape: str = "sphere", margin_voxels: float = 8.0,
                plane_std: float = 0.1 ** (1.0 / 3.0), model: str = "workload") -> Field:
    """A field on R = 16 T + 1 nodes whose spatial features are tri-planes on the
    tiles that hold a node within margin_voxels voxels of the surface (others empty),
    probes at the tile corners (P = T + 1).  Planes ~ N(0, plane_std), so their
    channel product has std 0.1; draw order: planes, probes, MLP."""
    R, P = TILE * T + 1, T + 1
    rng = np.random.default_rng(seed)
    sdf = sphere_sdf_nodes(R) if shape == "sphere" else torus_sdf_nodes(R)
    h = 2.0 / (R - 1)
    near = np.abs(sdf) <= margin_voxels * h
    occ = np.zeros((T, T, T), bool)
    for k in range(T):
        for j in range(T):
            for i in range(T):
                occ[k, j, i] = near[TILE * k:TILE * k + TILE + 1, TILE * j:TILE * j + TILE + 1,
                                    TILE * i:TILE * i + TILE + 1].any()
    index = np.full((T, T, T), -1, np.int32)
    index[occ] = np.arange(int(occ.sum()), dtype=np.int32)
    planes = (rng.standard_normal((int(occ.sum()), 3, TILE, TILE, N_FEAT), dtype=np.float32)
              * np.float32(plane_std))
    probes = (rng.standard_normal((P, P, P, n_sh, N_ANG), dtype=np.float32) * np.float32(0.1))
    if model == "workload":
        hidden, layers, mlp = HIDDEN, 1, xavier_uniform_mlp(rng)
    else:
        hidden, layers = PAPER_HIDDEN, PAPER_LAYERS
        mlp = xavier_uniform_mlp(rng, PAPER_N_IN, hidden, N_OUT, layers)
    f = Field(R=R, P=P, n_sh=n_sh, sdf=sdf, feat=np.zeros((1, 1, 1, N_FEAT), np.float32),
              probes=probes, mlp=mlp, hidden=hidden, layers=layers)
    f.tiles = Tiles(T=T, index=index, planes=planes)
    return f


def round_half(a: np.ndarray) -> np.ndarray:
    """float32 -> float16, round to nearest even (numpy's cast)."""
    return a.astype(np.float16)


def round_bf16(a: np.ndarray) -> np.ndarray:
    """float32 -> the nearest bfloat16 value (ties to even), returned as float32:
    the upper 16 bits of the float32 pattern after adding half of the dropped part."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(np.shape(a))


def mlp_weight_mask(n_in: int, hidden: int = HIDDEN, layers: int = 1,
                    n_out: int = N_OUT) -> np.ndarray:
    """True at the weights (not the biases) of a packed MLP [W_1, b_1, ..., Wo, bo]."""
    parts, fan = [], n_in
    for _ in range(layers):
        parts += [np.ones(hidden * fan, bool), np.zeros(hidden, bool)]
        fan = hidden
    parts += [np.ones(n_out * hidden, bool), np.zeros(n_out, bool)]
    return np.concatenate(parts)


def round_mlp_weights(mlp: np.ndarray, n_in: int, hidden: int, layers: int,
                      kind: str) -> np.ndarray:
    """The packed MLP with its weights (not its biases) rounded to float16 ("f16") or
    bfloat16 ("bf16"), as float32: the values a reduced-precision MLP multiplies."""
    m = np.array(mlp, dtype=np.float32)
    w = mlp_weight_mask(n_in, hidden, layers)
    m[w] = (round_half(m[w]).astype(np.float32) if kind == "f16" else round_bf16(m[w]))
    return m


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    R: int
    P: int
    n_sh: int
    n_samples: int
    skip_voxels: float      # <= 0: every sample is active
    tau: float
    views: int
    W: int
    H: int
    feat_dtype: str         # "f32" | "f16"
    sdf_dtype: str          # "f32" | "f16"
    mlp_dtype: str          # "f32" | "f16" | "bf16"

    @property
    def rays(self) -> int:
        return self.views * self.W * self.H


WORKLOADS = {
    # plain FP32 forward, 64^3 / 16^3, 8 x 32x16 rays, 64 samples, no skip
    "fwd64": Workload("fwd64", 64, 16, 9, 64, 0.0, 64.0, 8, 32, 16, "f32", "f32", "f32"),
    # FP32 training step, 256^3 / 64^3, 2^18 rays (8 x 256x128), 128 samples, skip |s| > 4 voxels
    "train256": Workload("train256", 256, 64, 9, 128, 4.0, 64.0, 8, 256, 128, "f32", "f32", "f32"),
    # mixed precision, 512^3 / 128^3, 2^20 rays (8 x 512x256), 64 samples, no skip
    "mixed512": Workload("mixed512", 512, 128, 9, 64, 0.0, 64.0, 8, 512, 256, "f16", "f32", "f16"),
    # full iteration: train256 rules at 512^3 / 128^3, 2^20 rays
    "iter512": Workload("iter512", 512, 128, 9, 128, 4.0, 64.0, 8, 512, 256, "f32", "f32", "f32"),
    # inference: FP16 grids 512^3 / 128^3, 16 views at 1920x1080, sphere tracing
    "trace512": Workload("trace512", 512, 128, 9, 0, 0.0, 64.0, 16, 1920, 1080, "f16", "f16", "f32"),
    # real-time render: FP16 grids 512^3 / 128^3, one view at the paper's 1920x1163 window,
    # voxels shaded within RT_BAND_VOXELS of the surface, then volume rendered (128
    # samples, skip |s| > 4 voxels)
    "rt512": Workload("rt512", 512, 128, 9, 128, 4.0, 64.0, 1, 1920, 1163, "f16", "f16", "f32"),
}

# shading band of the real-time render, in voxels: the skip threshold plus the two
# voxels a trilinear corner can lie beyond an active sample (|grad s| ~ 1)
RT_BAND_VOXELS = 6.0


def workload_rays(wl: Workload, order: str = "image"):
    cams = fibonacci_cameras(wl.views, wl.W, wl.H)
    return camera_rays(cams, wl.W, wl.H, order)


def shuffled(rays_o: np.ndarray, rays_d: np.ndarray, seed: int = 2):
    perm = np.random.default_rng(seed).permutation(rays_o.shape[0])
    return np.ascontiguousarray(rays_o[perm]), np.ascontiguousarray(rays_d[perm])


def adam_state(seed: int, n: int, scale: float = 1e-3):
    """Random Adam moments (m ~ N(0, scale), v ~ |N(0, scale)|^2) for step tests."""
    rng = np.random.default_rng(seed)
    m = (rng.standard_normal(n, dtype=np.float32) * np.float32(scale))
    v = (rng.standard_normal(n, dtype=np.float32) * np.float32(scale)) ** 2
    return m, v.astype(np.float32)


def random_like(seed: int, shape, scale: float = 1e-3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape, dtype=np.float32) * np.float32(scale))
