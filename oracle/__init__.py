"""ctypes front-end of the FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports it.

Every function takes numpy arrays of any float dtype (float16 / float32 /
float64); they are up-cast exactly to float64 before the call, so the oracle
sees the same values the HIP path reads.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .build import build as _build, LIB_PATH

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class _Field(C.Structure):
    _fields_ = [("R", C.c_int32), ("P", C.c_int32), ("n_feat", C.c_int32), ("n_sh", C.c_int32),
                ("n_ang", C.c_int32), ("hidden", C.c_int32), ("mlp_layers", C.c_int32),
                ("sdf", _dp), ("feat", _dp),
                ("probes", _dp), ("mlp", _dp), ("tile_T", C.c_int32),
                ("tile_index", C.POINTER(C.c_int32)), ("tile_feat", _dp)]


class _Opts(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("tau", C.c_double), ("skip_voxels", C.c_double),
                ("flags", C.c_int32)]


class _StepOpts(C.Structure):
    _fields_ = [("lr_sdf", C.c_double), ("lr_feat", C.c_double), ("lr_probe", C.c_double),
                ("lr_mlp", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("lambda_eik", C.c_double), ("lambda_tv_feat", C.c_double),
                ("lambda_tv_probe", C.c_double)]


class _StepExt(C.Structure):
    _fields_ = [("base", _StepOpts), ("lambda_sdf", C.c_double), ("lambda_normal", C.c_double),
                ("sigma", C.c_double), ("smooth", C.c_int32), ("weighted", C.c_int32)]


NO_FS, NO_FA, NV_ONE = 1, 2, 4
SH_REFLECT, FRESNEL_PAPER = 8, 16
MAX_N = 1 << 20  # largest sample count the render calls accept


class OracleError(RuntimeError):
    pass


def _ok(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"oracle {what} rejected its arguments (rc={rc})")


def lib():
    """The oracle library: oracle/liboracle.so, or the build named by the
    PSDF_ORACLE_LIB environment variable (a sanitised build, say)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PSDF_ORACLE_LIB") or LIB_PATH
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            _build()
        _lib = C.CDLL(path)
        _lib.orc_logsigmoid.restype = C.c_double
        _lib.orc_composite.restype = C.c_double
        _lib.orc_l1_loss.restype = C.c_double
        _lib.orc_mlp_size.restype = C.c_int64
        _lib.orc_l2rel_loss.restype = C.c_double
        _lib.orc_max_threads.restype = C.c_int
        _lib.orc_plane_smooth.restype = C.c_double
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


@dataclass
class OField:
    """float64 copies of a field's arrays, kept alive with the C struct."""
    R: int
    P: int
    n_sh: int
    sdf: np.ndarray
    feat: np.ndarray
    probes: np.ndarray
    mlp: np.ndarray
    n_feat: int = 3
    n_ang: int = 4
    hidden: int = 16
    layers: int = 1
    tile_T: int = 0                      # > 0: tri-plane features on 16^3-cell tiles
    tile_index: np.ndarray = None        # int32 [T, T, T], -1 = empty tile
    tile_feat: np.ndarray = None         # [slots, 3, 16, 16, n_feat]

    def cstruct(self) -> _Field:
        ti = (self.tile_index.ctypes.data_as(C.POINTER(C.c_int32)) if self.tile_T
              else C.POINTER(C.c_int32)())
        tf = _p(self.tile_feat) if self.tile_T else _dp()
        return _Field(self.R, self.P, self.n_feat, self.n_sh, self.n_ang, self.hidden,
                      self.layers, _p(self.sdf), _p(self.feat), _p(self.probes), _p(self.mlp),
                      self.tile_T, ti, tf)

    def n_inputs(self, flags: int = 0) -> int:
        return self.n_feat + self.n_ang + (6 if flags & FRESNEL_PAPER else 3)


def make_field(sdf, feat, probes, mlp, n_sh=None, hidden=16, layers=1) -> OField:
    sdf, feat, probes, mlp = _d(sdf), _d(feat), _d(probes), _d(mlp)
    R = sdf.shape[0]
    P = probes.shape[0]
    n_feat = feat.shape[-1]
    if n_sh is None:
        n_sh = probes.shape[3]
    n_ang = probes.shape[-1]
    return OField(R=R, P=P, n_sh=n_sh, sdf=sdf, feat=feat, probes=probes, mlp=mlp,
                  n_feat=n_feat, n_ang=n_ang, hidden=hidden, layers=layers)


def field_from(fld, half: bool = False, half_sdf: bool = False, mlp_round: str = "",
               flags: int = 0) -> OField:
    """OField from a workloads.Field; `half` rounds features and probes to
    float16 first (the values an FP16-storage path reads); `mlp_round` ("f16" or
    "bf16") rounds the MLP weights (not the biases), the values a reduced-precision
    MLP multiplies (`flags` gives the MLP's input count)."""
    feat, probes, sdf, mlp = fld.feat, fld.probes, fld.sdf, fld.mlp
    if half:
        feat, probes = feat.astype(np.float16), probes.astype(np.float16)
    if half_sdf:
        sdf = sdf.astype(np.float16)
    if mlp_round:
        import workloads as wl
        n_in = fld.feat.shape[-1] + fld.probes.shape[-1] + (6 if flags & FRESNEL_PAPER else 3)
        mlp = wl.round_mlp_weights(mlp, n_in, fld.hidden, fld.layers, mlp_round)
    of = make_field(sdf, feat, probes, mlp, n_sh=fld.n_sh, hidden=fld.hidden,
                    layers=fld.layers)
    tiles = getattr(fld, "tiles", None)
    if tiles is not None:  # sparse tiles with tri-plane features
        planes = tiles.planes.astype(np.float16) if half else tiles.planes
        of.tile_T = tiles.T
        of.tile_index = np.ascontiguousarray(tiles.index, dtype=np.int32)
        of.tile_feat = _d(planes)
    return of


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------
def ray_box(o, d):
    o, d = _d(o), _d(d)
    tn, tf = C.c_double(), C.c_double()
    hit = lib().orc_ray_box(_p(o), _p(d), C.byref(tn), C.byref(tf))
    return bool(hit), tn.value, tf.value


def trilinear(grid, x):
    """grid (R,R,R) or (R,R,R,C...) ; x (3,) -> (C,)"""
    g = _d(grid)
    R = g.shape[0]
    Cc = int(np.prod(g.shape[3:])) if g.ndim > 3 else 1
    out = np.zeros(Cc)
    lib().orc_trilinear(_p(g), C.c_int(R), C.c_int(Cc), _p(_d(x)), _p(out))
    return out


def sdf_gradient(sdf, x):
    s = _d(sdf)
    g = np.zeros(3)
    lib().orc_sdf_gradient(_p(s), C.c_int(s.shape[0]), _p(_d(x)), _p(g))
    return g


def sh_basis(n_sh, v):
    Y = np.zeros(16)
    rc = lib().orc_sh_basis(C.c_int(n_sh), _p(_d(v)), _p(Y))
    if rc != 0:
        raise ValueError(n_sh)
    return Y[:n_sh]


def logsigmoid(x):
    return lib().orc_logsigmoid(C.c_double(x))


def sh_grad(n_sh, v):
    """(n_sh, 3): gradient of each SH polynomial at v"""
    dY = np.zeros(48)
    rc = lib().orc_sh_grad(C.c_int(n_sh), _p(_d(v)), _p(dY))
    if rc != 0:
        raise ValueError(n_sh)
    return dY[:3 * n_sh].reshape(n_sh, 3)


def mlp_size(n_in, hidden=16, layers=1) -> int:
    return int(lib().orc_mlp_size(C.c_int(n_in), C.c_int(hidden), C.c_int(layers)))


def mlp_forward(mlp, z, hidden=16, layers=1):
    """returns C, out, hid, pre; hid and pre are (layers, hidden) for layers > 1"""
    z = _d(z)
    n_in = z.shape[0]
    mlp = _d(mlp)
    if mlp.size != mlp_size(n_in, hidden, layers):
        raise ValueError(f"mlp has {mlp.size} values, expected {mlp_size(n_in, hidden, layers)}")
    pre, hid = np.zeros(layers * hidden), np.zeros(layers * hidden)
    out, Cc = np.zeros(3), np.zeros(3)
    lib().orc_mlp_forward(_p(mlp), C.c_int(n_in), C.c_int(hidden), C.c_int(layers), _p(z),
                          _p(pre), _p(hid), _p(out), _p(Cc))
    if layers > 1:
        hid, pre = hid.reshape(layers, hidden), pre.reshape(layers, hidden)
    return Cc, out, hid, pre


def composite(s, active, tau):
    s = _d(s)
    N = s.shape[0]
    act = np.ascontiguousarray(active, dtype=np.int32)
    alpha, T, w = np.zeros(N), np.zeros(N), np.zeros(N)
    logT = lib().orc_composite(C.c_int(N), _p(s), act.ctypes.data_as(_ip), C.c_double(tau),
                               _p(alpha), _p(T), _p(w))
    return alpha, T, w, logT


def _check_field(of: OField, flags: int):
    fs = of.cstruct()
    _ok(lib().orc_field_check(C.byref(fs), C.c_int32(flags)), "field")
    n = mlp_size(of.n_inputs(flags), of.hidden, of.layers)
    if of.mlp.size != n:
        raise OracleError(f"mlp has {of.mlp.size} values, the colour model needs {n}")


def shade(of: OField, x, v, flags=0):
    _check_field(of, flags)
    Cc = np.zeros(3)
    z = np.zeros(of.n_inputs(flags))
    fs = of.cstruct()
    lib().orc_shade(C.byref(fs), C.c_int32(flags), _p(_d(x)), _p(_d(v)), _p(Cc), _p(z))
    return Cc, z


# ---------------------------------------------------------------------------
# the render step
# ---------------------------------------------------------------------------
def render_forward(of: OField, rays_o, rays_d, n_samples, tau=64.0, skip_voxels=0.0, flags=0):
    o, d = _d(rays_o), _d(rays_d)
    B = o.shape[0]
    rgb, aux = np.zeros((B, 3)), np.zeros((B, 4))
    dw, margin = np.zeros((B, 2)), np.zeros(B)
    ns = np.zeros(B, dtype=np.int32)
    _check_field(of, flags)
    fs = of.cstruct()
    op = _Opts(n_samples, tau, skip_voxels, flags)
    _ok(lib().orc_render_forward(C.byref(fs), C.byref(op), C.c_int64(B), _p(o), _p(d), _p(rgb),
                                 _p(aux), _p(dw), _p(margin), ns.ctypes.data_as(_ip)),
        "render_forward")
    return dict(rgb=rgb, aux=aux, depth_wsum=dw, margin=margin, n_shaded=ns)


def render_backward(of: OField, rays_o, rays_d, dL_drgb, n_samples, tau=64.0, skip_voxels=0.0,
                    flags=0):
    o, d, dL = _d(rays_o), _d(rays_d), _d(dL_drgb)
    B = o.shape[0]
    g = dict(sdf=np.zeros_like(of.sdf),
             feat=np.zeros_like(of.tile_feat if of.tile_T else of.feat),  # tiles: plane layout
             probes=np.zeros_like(of.probes), mlp=np.zeros_like(of.mlp))
    _check_field(of, flags)
    fs = of.cstruct()
    op = _Opts(n_samples, tau, skip_voxels, flags)
    _ok(lib().orc_render_backward(C.byref(fs), C.byref(op), C.c_int64(B), _p(o), _p(d), _p(dL),
                                  _p(g["sdf"]), _p(g["feat"]), _p(g["probes"]), _p(g["mlp"])),
        "render_backward")
    return g


def l1_loss(rgb, target):
    rgb, target = _d(rgb), _d(target)
    B = rgb.shape[0]
    dL = np.zeros_like(rgb)
    loss = lib().orc_l1_loss(C.c_int64(B), _p(rgb), _p(target), _p(dL))
    return loss, dL


def regularizers(sdf, feat, probes, lambda_eik, lambda_tv_feat, lambda_tv_probe):
    sdf, feat, probes = _d(sdf), _d(feat), _d(probes)
    R, P = sdf.shape[0], probes.shape[0]
    n_feat = int(np.prod(feat.shape[3:]))
    n_pc = int(np.prod(probes.shape[3:]))
    gs, gf, gp = np.zeros_like(sdf), np.zeros_like(feat), np.zeros_like(probes)
    losses = np.zeros(3)
    lib().orc_regularizers(C.c_int(R), C.c_int(P), C.c_int(n_feat), C.c_int(n_pc), _p(sdf),
                           _p(feat), _p(probes), C.c_double(lambda_eik),
                           C.c_double(lambda_tv_feat), C.c_double(lambda_tv_probe), _p(gs),
                           _p(gf), _p(gp), _p(losses))
    return losses, gs, gf, gp


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.995, eps=1e-8):
    p, g, m, v = _d(p).copy(), _d(g), _d(m).copy(), _d(v).copy()
    lib().orc_adam(C.c_int64(p.size), _p(p), _p(g), _p(m), _p(v), C.c_int64(step),
                   C.c_double(lr), C.c_double(beta1), C.c_double(beta2), C.c_double(eps))
    return p, m, v


@dataclass
class StepOpts:
    lr_sdf: float = 0.01
    lr_feat: float = 0.01
    lr_probe: float = 0.001
    lr_mlp: float = 0.001
    beta1: float = 0.9
    beta2: float = 0.995
    eps: float = 1e-8
    lambda_eik: float = 0.1
    lambda_tv_feat: float = 0.05
    lambda_tv_probe: float = 0.2

    def cstruct(self) -> _StepOpts:
        return _StepOpts(self.lr_sdf, self.lr_feat, self.lr_probe, self.lr_mlp, self.beta1,
                         self.beta2, self.eps, self.lambda_eik, self.lambda_tv_feat,
                         self.lambda_tv_probe)


def grid_step(params: dict, grads: dict, m: np.ndarray, v: np.ndarray, step: int,
              opts: StepOpts):
    """params/grads: dict sdf, feat, probes, mlp.  m, v concatenated in that order.
    Returns (new params dict, m, v, losses)."""
    p = {k: _d(params[k]).copy() for k in ("sdf", "feat", "probes", "mlp")}
    g = {k: _d(grads[k]) for k in ("sdf", "feat", "probes", "mlp")}
    m, v = _d(m).copy(), _d(v).copy()
    R, P = p["sdf"].shape[0], p["probes"].shape[0]
    n_feat = int(np.prod(p["feat"].shape[3:]))
    n_pc = int(np.prod(p["probes"].shape[3:]))
    losses = np.zeros(3)
    so = opts.cstruct()
    lib().orc_grid_step(C.c_int(R), C.c_int(P), C.c_int(n_feat), C.c_int(n_pc),
                        C.c_int(p["mlp"].size), _p(p["sdf"]), _p(p["feat"]), _p(p["probes"]),
                        _p(p["mlp"]), _p(g["sdf"]), _p(g["feat"]), _p(g["probes"]),
                        _p(g["mlp"]), _p(m), _p(v), C.c_int64(step), C.byref(so), _p(losses))
    return p, m, v, losses


# ---------------------------------------------------------------------------
# smoothed SDF and the remaining regularisers (Sec. 3.3)
# ---------------------------------------------------------------------------
def gauss5(sigma=1.0):
    w = np.zeros(5)
    lib().orc_gauss5(C.c_double(sigma), _p(w))
    return w


def smooth(shat, sigma=1.0):
    """s = G(shat), the 5^3 Gaussian with replicated edges."""
    shat = _d(shat)
    s = np.zeros_like(shat)
    lib().orc_smooth(C.c_int(shat.shape[0]), C.c_double(sigma), _p(shat), _p(s))
    return s


def smooth_T(y, sigma=1.0):
    """G^T y."""
    y = _d(y)
    out = np.zeros_like(y)
    lib().orc_smooth_T(C.c_int(y.shape[0]), C.c_double(sigma), _p(y), _p(out))
    return out


def sdf_regs(shat, g_s=None, smooth=True, sigma=1.0, weighted=False, lambda_sdf=0.2,
             lambda_eik=0.1, lambda_normal=0.05):
    """(losses [L_sdf, L_Eik, L_normal], dL/dshat, s) with g_s the render gradient
    with respect to s (zero when None)."""
    shat = _d(shat)
    g_s = np.zeros_like(shat) if g_s is None else _d(g_s)
    g, s = np.zeros_like(shat), np.zeros_like(shat)
    losses = np.zeros(3)
    lib().orc_sdf_regs(C.c_int(shat.shape[0]), _p(shat), C.c_int(int(smooth)), C.c_double(sigma),
                       C.c_int(int(weighted)), C.c_double(lambda_sdf), C.c_double(lambda_eik),
                       C.c_double(lambda_normal), _p(g_s), _p(g), _p(s), _p(losses))
    return losses, g, s


@dataclass
class StepExt:
    base: StepOpts
    lambda_sdf: float = 0.2
    lambda_normal: float = 0.05
    sigma: float = 1.0
    smooth: bool = True
    weighted: bool = False

    def cstruct(self) -> _StepExt:
        return _StepExt(self.base.cstruct(), self.lambda_sdf, self.lambda_normal, self.sigma,
                        int(self.smooth), int(self.weighted))


def grid_step_ext(params: dict, grads: dict, m: np.ndarray, v: np.ndarray, step: int,
                  opts: StepExt):
    """params['sdf'] is shat; grads['sdf'] is the render gradient with respect to
    s = G(shat).  Returns (new params, m, v, losses[5], s of the new shat)."""
    p = {k: _d(params[k]).copy() for k in ("sdf", "feat", "probes", "mlp")}
    g = {k: _d(grads[k]) for k in ("sdf", "feat", "probes", "mlp")}
    m, v = _d(m).copy(), _d(v).copy()
    R, P = p["sdf"].shape[0], p["probes"].shape[0]
    n_feat = int(np.prod(p["feat"].shape[3:]))
    n_pc = int(np.prod(p["probes"].shape[3:]))
    losses = np.zeros(5)
    s_new = np.zeros_like(p["sdf"])
    so = opts.cstruct()
    lib().orc_grid_step_ext(C.c_int(R), C.c_int(P), C.c_int(n_feat), C.c_int(n_pc),
                            C.c_int(p["mlp"].size), _p(p["sdf"]), _p(p["feat"]), _p(p["probes"]),
                            _p(p["mlp"]), _p(g["sdf"]), _p(g["feat"]), _p(g["probes"]),
                            _p(g["mlp"]), _p(m), _p(v), C.c_int64(step), C.byref(so),
                            _p(losses), _p(s_new))
    return p, m, v, losses, s_new


def l2rel_loss(rgb, target, lam=40.0, eps=1e-3, n_images=1.0):
    """(L, dL/drgb) of the relatively weighted L2 photometric loss."""
    rgb, target = _d(rgb), _d(target)
    dL = np.zeros_like(rgb)
    L = lib().orc_l2rel_loss(C.c_int64(rgb.shape[0]), _p(rgb), _p(target), C.c_double(lam),
                             C.c_double(eps), C.c_double(n_images), _p(dL))
    return L, dL


# ---------------------------------------------------------------------------
# real-time path: per-voxel shading, then volume rendering of the colour field
# ---------------------------------------------------------------------------
def voxel_shade(of: OField, cam, band, flags=0):
    """Colours [R, R, R, 3] of the nodes with |s| <= band seen from the camera
    centre cam[3], 7, 11 (0 elsewhere)."""
    cam = _d(cam)
    centre = np.ascontiguousarray([cam[3], cam[7], cam[11]])
    _check_field(of, flags)
    col = np.zeros(of.sdf.shape + (3,))
    fs = of.cstruct()
    lib().orc_voxel_shade(C.byref(fs), C.c_int32(flags), _p(centre), C.c_double(band), _p(col))
    return col


def volume_render(of: OField, col, cam, W, H, n_samples, tau=64.0, skip_voxels=0.0,
                  pixel_ids=None):
    """Colours of pinhole pixels (ids py * W + px) volume-rendered through the colour
    field `col` [R, R, R, 3]; returns (rgb, margin)."""
    cam, col = _d(cam), _d(col)
    if pixel_ids is None:
        pixel_ids = np.arange(W * H, dtype=np.int64)
    ids = np.ascontiguousarray(pixel_ids, dtype=np.int64)
    out, mg = np.zeros((ids.size, 3)), np.zeros(ids.size)
    fs = of.cstruct()
    op = _Opts(n_samples, tau, skip_voxels, 0)
    _ok(lib().orc_volume_render(C.byref(fs), _p(col), C.byref(op), _p(cam), C.c_int32(W),
                                C.c_int32(H), ids.ctypes.data_as(_lp), C.c_int64(ids.size),
                                _p(out), _p(mg)), "volume_render")
    return out, mg


def triplane(of: OField, x):
    """(F_s at x, tile slot) of a tiled field."""
    x = _d(x)
    out = np.zeros(of.n_feat)
    slot = lib().orc_triplane(C.byref(of.cstruct()), _p(x), _p(out))
    return out, slot


def plane_smooth(planes, lam):
    """(loss, gradient) of the smoothness of the tri-plane features."""
    planes = _d(planes)
    g = np.zeros_like(planes)
    L = lib().orc_plane_smooth(C.c_int64(planes.shape[0]), C.c_int(planes.shape[-1]), _p(planes),
                               C.c_double(lam), _p(g))
    return L, g


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops."""
    lib().orc_set_threads(C.c_int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def sphere_trace(of: OField, cams: np.ndarray, W: int, H: int, pixel_ids=None, eps=1e-3,
                 max_steps=256, flags=0):
    """cams: (V, 16) float array (c2w row-major 12, fx, fy, cx, cy)."""
    cams = _d(cams)
    V = cams.shape[0]
    if pixel_ids is None:
        pixel_ids = np.arange(V * W * H, dtype=np.int64)
    ids = np.ascontiguousarray(pixel_ids, dtype=np.int64)
    n = ids.shape[0]
    out, th, mg = np.zeros((n, 3)), np.zeros(n), np.zeros(n)
    steps = np.zeros(n, dtype=np.int32)
    _check_field(of, flags)
    fs = of.cstruct()
    _ok(lib().orc_sphere_trace(C.byref(fs), C.c_int32(flags), C.c_double(eps),
                               C.c_int32(max_steps), C.c_int32(V), _p(cams), C.c_int32(W),
                               C.c_int32(H), ids.ctypes.data_as(_lp), C.c_int64(n), _p(out),
                               _p(th), steps.ctypes.data_as(_ip), _p(mg)),
        "sphere_trace")
    return dict(rgb=out, t_hit=th, steps=steps, margin=mg)
