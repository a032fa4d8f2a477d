"""Python binding of libprobesdf.so, the MI355X (gfx950) ProbeSDF render step.

Argument marshalling only: every step of the render path runs in the HIP
kernels behind the C ABI declared in include/probesdf.h.  PyTorch supplies
device memory (tensors) and the stream (torch's current HIP stream).  If the
library is not built, every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field as dc_field
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprobesdf.so")

F32, F16, BF16 = 0, 1, 2
FLAG_NO_FS, FLAG_NO_FA, FLAG_NV_ONE = 1, 2, 4
FLAG_SH_REFLECT, FLAG_FRESNEL_PAPER = 8, 16
MODEL_MAX_SAMPLES = 513
OK, EINVAL, EALIGN, EUNSUPPORTED, EHIP = 0, -1, -2, -3, -4
ABI_VERSION = 5
BWD_FROM_TAPE = 1
BRICK = 8

N_FEAT, N_ANG, HIDDEN, N_MLP = 3, 4, 16, 227


def mlp_size(flags: int = 0, hidden: int = HIDDEN, layers: int = 1) -> int:
    """Parameters of the packed colour MLP (227 for the workload model)."""
    n_in = N_FEAT + N_ANG + (6 if flags & FLAG_FRESNEL_PAPER else 3)
    return hidden * n_in + hidden + (layers - 1) * (hidden * hidden + hidden) + 3 * hidden + 3

EXPORTS = ("psdf_render_forward", "psdf_render_backward", "psdf_render_backward_noalloc",
           "psdf_l1_loss", "psdf_l2rel_loss", "psdf_grid_step", "psdf_step_work_bytes",
           "psdf_smooth_sdf", "psdf_render_sphere_trace", "psdf_sdf_bounds",
           "psdf_voxel_list", "psdf_voxel_shade", "psdf_volume_render", "psdf_plane_step",
           "psdf_backward_workspace_bytes", "psdf_last_error", "psdf_abi_version")
STEP_SMOOTH, STEP_REG_WEIGHT = 1, 2
NOALLOC_SCRATCH_BYTES = 134217728


class PsdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"probesdf error {code}: {msg}")
        self.code = code


class _Field(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("R", C.c_int32), ("P", C.c_int32),
                ("n_feat", C.c_int32), ("sh_coeffs", C.c_int32), ("n_ang", C.c_int32),
                ("mlp_hidden", C.c_int32), ("sdf_dtype", C.c_int32), ("feat_dtype", C.c_int32),
                ("mlp_dtype", C.c_int32), ("sdf", C.c_void_p), ("feat", C.c_void_p),
                ("probes", C.c_void_p), ("mlp", C.c_void_p), ("sdf_bounds", C.c_void_p),
                ("mlp_layers", C.c_int32), ("tile_T", C.c_int32), ("tile_index", C.c_void_p),
                ("n_tiles", C.c_int64)]


class _RenderOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_samples", C.c_int32), ("tau", C.c_float),
                ("skip_voxels", C.c_float), ("flags", C.c_int32)]


class _Grads(C.Structure):
    _fields_ = [("sdf", C.c_void_p), ("feat", C.c_void_p), ("probes", C.c_void_p),
                ("mlp", C.c_void_p)]


class _StepArgs(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("R", C.c_int32), ("P", C.c_int32),
                ("n_feat", C.c_int32), ("n_pc", C.c_int32), ("n_mlp", C.c_int32),
                ("step", C.c_int64),
                ("lr_sdf", C.c_float), ("lr_feat", C.c_float), ("lr_probe", C.c_float),
                ("lr_mlp", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("lambda_eik", C.c_float), ("lambda_tv_feat", C.c_float),
                ("lambda_tv_probe", C.c_float)] + [
        (n, C.c_void_p) for n in (
            "sdf_in", "sdf_out", "feat_in", "feat_out", "probes_in", "probes_out", "mlp",
            "g_sdf", "g_feat", "g_probes", "g_mlp", "m_sdf", "v_sdf", "m_feat", "v_feat",
            "m_probes", "v_probes", "m_mlp", "v_mlp", "sdf_half_out", "feat_half_out",
            "probes_half_out", "losses", "sdf_bounds_out")] + [
        ("sdf_reg_flags", C.c_int32), ("lambda_sdf", C.c_float), ("lambda_normal", C.c_float),
        ("smooth_sigma", C.c_float), ("s_in", C.c_void_p), ("s_out", C.c_void_p),
        ("work", C.c_void_p), ("work_bytes", C.c_int64), ("losses_ext", C.c_void_p)]


class _TraceOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("eps", C.c_float), ("max_steps", C.c_int32),
                ("flags", C.c_int32)]


_lib = None


def lib():
    """Load libprobesdf.so (built in tree by paper_2412_10084_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2412_10084_amd.build`"
                               " (the HIP library is required; there is no fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.psdf_render_forward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, i64, vp]
        L.psdf_render_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, i64, i32, vp]
        L.psdf_render_backward_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.psdf_backward_workspace_bytes.argtypes = [i64, i32, i64]
        L.psdf_l1_loss.argtypes = [i64, vp, vp, vp, vp, vp]
        f32 = C.c_float
        L.psdf_l2rel_loss.argtypes = [i64, vp, vp, vp, vp, f32, f32, f32, vp]
        L.psdf_step_work_bytes.argtypes = [i32]
        L.psdf_smooth_sdf.argtypes = [i32, f32, vp, vp, vp, vp]
        L.psdf_voxel_list.argtypes = [i32, i32, vp, f32, vp, i64, vp, vp]
        L.psdf_voxel_shade.argtypes = [vp, i32, vp, vp, vp, i64, vp, i32, vp]
        L.psdf_volume_render.argtypes = [vp, vp, vp, i32, vp, i32, i32, vp, vp]
        L.psdf_plane_step.argtypes = [i64, i32, vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, f32,
                                      vp, vp, vp]
        L.psdf_grid_step.argtypes = [vp, vp]
        L.psdf_render_sphere_trace.argtypes = [vp, vp, i32, vp, i32, i32, vp, vp]
        L.psdf_sdf_bounds.argtypes = [i32, i32, vp, vp, vp]
        L.psdf_last_error.restype = C.c_char_p
        L.psdf_last_error.argtypes = []
        L.psdf_abi_version.restype = C.c_int
        for n in EXPORTS:
            if n not in ("psdf_last_error", "psdf_abi_version", "psdf_backward_workspace_bytes",
                         "psdf_step_work_bytes"):
                getattr(L, n).restype = C.c_int
        L.psdf_backward_workspace_bytes.restype = C.c_int64
        L.psdf_step_work_bytes.restype = C.c_int64
        if L.psdf_abi_version() != ABI_VERSION:
            raise RuntimeError("libprobesdf ABI version mismatch")
        _lib = L
    return _lib


def last_error() -> str:
    return lib().psdf_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise PsdfError(rc, last_error())


def _ptr(t) -> Optional[int]:
    """Device address of a tensor argument (or a raw pointer passed as an int).
    Tensors must be dense and on the GPU: a strided view or a host tensor would
    be read as packed device memory, so both raise instead."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise PsdfError(EINVAL, f"tensor of shape {tuple(t.shape)} is not on the GPU")
    if not t.is_contiguous():
        raise PsdfError(EINVAL, f"tensor of shape {tuple(t.shape)} is not contiguous")
    return t.data_ptr()


def _f32(t, name: str):
    """A float32 tensor argument (rays, colours, gradients, MLP weights)."""
    if t is not None and not isinstance(t, int):
        import torch
        if t.dtype != torch.float32:
            raise PsdfError(EINVAL, f"{name} must be float32, got {t.dtype}")
    return t


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
@dataclass
class Field:
    """Device tensors of one scene.  sdf (R,R,R) f32|f16; feat (R,R,R,3) f32|f16;
    probes (P,P,P,sh,4) same dtype as feat; mlp (227,) f32; bounds: optional brick
    bounds of exactly this sdf (sdf_bounds() or grid_step(bounds_out=...)) that let
    the march skip samples the skip rule leaves inactive."""
    sdf: object
    feat: object
    probes: object
    mlp: object
    mlp_dtype: int = F32
    bounds: object = None
    hidden: int = HIDDEN
    layers: int = 1
    tiles: object = None  # int32 (T, T, T) tile index: feat holds tri-planes (n_tiles,3,16,16,3)

    @staticmethod
    def _dt(t) -> int:
        import torch
        return {torch.float32: F32, torch.float16: F16}[t.dtype]

    def cstruct(self) -> _Field:
        _f32(self.mlp, "mlp")
        if not isinstance(self.probes, int) and self._dt(self.probes) != self._dt(self.feat):
            raise PsdfError(EINVAL, "probes and feat must have the same dtype")
        R = self.sdf.shape[0]
        P = self.probes.shape[0]
        sh = self.probes.shape[3]
        return _Field(C.sizeof(_Field), R, P, self.feat.shape[-1], sh, self.probes.shape[-1],
                      self.hidden, self._dt(self.sdf), self._dt(self.feat), self.mlp_dtype,
                      _ptr(self.sdf), _ptr(self.feat), _ptr(self.probes), _ptr(self.mlp),
                      _ptr(self.bounds), self.layers,
                      0 if self.tiles is None else self.tiles.shape[0], _ptr(self.tiles),
                      0 if self.tiles is None else self.feat.shape[0])


@dataclass
class RenderOpts:
    n_samples: int = 64
    tau: float = 64.0
    skip_voxels: float = 0.0
    flags: int = 0

    def cstruct(self) -> _RenderOpts:
        return _RenderOpts(C.sizeof(_RenderOpts), self.n_samples, self.tau, self.skip_voxels,
                           self.flags)


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
    # Sec. 3.3's smoothed SDF and remaining regularisers (off by default)
    smooth: bool = False        # the sdf parameters are raw values; rendering reads G(shat)
    reg_weight: bool = False    # (1 + 5 |s|)^-1 on the SDF regularisers' gradients
    lambda_sdf: float = 0.0
    lambda_normal: float = 0.0
    sigma: float = 1.0

    def extended(self) -> bool:
        return self.smooth or self.reg_weight or self.lambda_sdf != 0 or self.lambda_normal != 0


# ---------------------------------------------------------------------------
# entry points (raw calls: every tensor argument is a device tensor or a pointer)
# ---------------------------------------------------------------------------
def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


def render_forward(field: Field, opts: RenderOpts, rays_o, rays_d, rgb, aux=None,
                   depth_wsum=None, stream=None, tape=None) -> None:
    """tape: optional workspace (backward_workspace) in which the forward records its
    shaded samples for render_backward(..., from_tape=True)."""
    for t, n in ((rays_o, "rays_o"), (rays_d, "rays_d"), (rgb, "rgb"), (aux, "aux"),
                 (depth_wsum, "depth_wsum")):
        _f32(t, n)
    fs, op = field.cstruct(), opts.cstruct()
    B = rays_o.shape[0] if not isinstance(rays_o, int) else None
    _check(lib().psdf_render_forward(C.byref(fs), C.byref(op), B, _ptr(rays_o), _ptr(rays_d),
                                     _ptr(rgb), _ptr(aux), _ptr(depth_wsum), _ptr(tape),
                                     _nbytes(tape), _stream(stream)))


def backward_workspace_bytes(B: int, P: int, max_samples: int) -> int:
    n = lib().psdf_backward_workspace_bytes(B, P, max_samples)
    if n < 0:
        raise PsdfError(EINVAL, f"workspace size out of range (B={B}, P={P}, "
                                f"max_samples={max_samples})")
    return n


def backward_workspace(B: int, P: int, max_samples: int, device="cuda"):
    """A device buffer for the entry-parallel backward of B rays over a P^3 probe grid
    with room for `max_samples` shaded samples (any size gives the same gradients;
    waves that do not fit take the fused schedule)."""
    import torch
    n = backward_workspace_bytes(B, P, max_samples)
    return torch.empty(n, dtype=torch.uint8, device=device)


def render_backward(field: Field, opts: RenderOpts, rays_o, rays_d, aux, dL_drgb, grads: dict,
                    stream=None, workspace=None, from_tape: bool = False) -> None:
    """workspace: optional scratch for the entry-parallel schedule, or (from_tape) the
    tape the forward recorded for the same field, opts and rays."""
    for t, n in ((rays_o, "rays_o"), (rays_d, "rays_d"), (aux, "aux"), (dL_drgb, "dL_drgb"),
                 *((grads.get(k), "grads." + k) for k in ("sdf", "feat", "probes", "mlp"))):
        _f32(t, n)
    fs, op = field.cstruct(), opts.cstruct()
    g = _Grads(_ptr(grads.get("sdf")), _ptr(grads.get("feat")), _ptr(grads.get("probes")),
               _ptr(grads.get("mlp")))
    _check(lib().psdf_render_backward(C.byref(fs), C.byref(op), rays_o.shape[0], _ptr(rays_o),
                                      _ptr(rays_d), _ptr(aux), _ptr(dL_drgb), C.byref(g),
                                      _ptr(workspace), _nbytes(workspace),
                                      BWD_FROM_TAPE if from_tape else 0, _stream(stream)))


def render_backward_noalloc(field: Field, opts: RenderOpts, rays_o, rays_d, aux, dL_drgb,
                            grads: dict, stream=None) -> None:
    """render_backward with the entry-parallel schedule over the library's static
    device scratch (NOALLOC_SCRATCH_BYTES): no workspace argument, no allocation.
    Calls on one GPU share the scratch and must not overlap."""
    fs, op = field.cstruct(), opts.cstruct()
    g = _Grads(_ptr(grads.get("sdf")), _ptr(grads.get("feat")), _ptr(grads.get("probes")),
               _ptr(grads.get("mlp")))
    _check(lib().psdf_render_backward_noalloc(C.byref(fs), C.byref(op), rays_o.shape[0],
                                              _ptr(rays_o), _ptr(rays_d), _ptr(aux),
                                              _ptr(dL_drgb), C.byref(g), _stream(stream)))


def l1_loss(rgb, target, dL_drgb, loss=None, stream=None) -> None:
    for t, n in ((rgb, "rgb"), (target, "target"), (dL_drgb, "dL_drgb"), (loss, "loss")):
        _f32(t, n)
    _check(lib().psdf_l1_loss(rgb.shape[0], _ptr(rgb), _ptr(target), _ptr(dL_drgb), _ptr(loss),
                              _stream(stream)))


def n_bricks(R: int) -> int:
    """Bricks per axis of the sdf bounds of an R^3 grid."""
    return (R - 2) // BRICK + 1


def sdf_bounds(sdf, out=None, stream=None):
    """Brick bounds (nb, nb, nb, 2) FP32 of an (R, R, R) sdf tensor; returns `out`."""
    import torch
    R = sdf.shape[0]
    if out is None:
        nb = n_bricks(R)
        out = torch.empty((nb, nb, nb, 2), device=sdf.device, dtype=torch.float32)
    dt = Field._dt(sdf)
    _check(lib().psdf_sdf_bounds(R, dt, _ptr(sdf), _ptr(out), _stream(stream)))
    return out


def plane_step(planes_in, planes_out, grad, m, v, step: int, lr: float = 0.01,
               beta1: float = 0.9, beta2: float = 0.995, eps: float = 1e-8,
               lam: float = 0.05, half_out=None, loss=None, stream=None) -> None:
    """Smoothness of the tri-plane features of sparse tiles + Adam (out of place)."""
    for t, n in ((planes_in, "planes_in"), (planes_out, "planes_out"), (grad, "grad"), (m, "m"),
                 (v, "v"), (loss, "loss")):
        _f32(t, n)
    _check(lib().psdf_plane_step(planes_in.shape[0], planes_in.shape[-1], _ptr(planes_in),
                                 _ptr(planes_out), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1,
                                 beta2, eps, lam, _ptr(half_out), _ptr(loss), _stream(stream)))


def step_work_bytes(R: int) -> int:
    return int(lib().psdf_step_work_bytes(R))


def smooth_sdf(shat, s, sigma: float = 1.0, s_half=None, stream=None) -> None:
    """s = G(shat), the 5^3 Gaussian of the raw SDF (the field the renderer reads)."""
    _check(lib().psdf_smooth_sdf(shat.shape[0], sigma, _ptr(_f32(shat, "shat")),
                                 _ptr(_f32(s, "s")), _ptr(s_half), _stream(stream)))


def l2rel_loss(rgb, target, dL_drgb, loss=None, lam: float = 40.0, eps: float = 1e-3,
               n_images: float = 1.0, stream=None) -> None:
    """The paper's relatively weighted L2 photometric loss and its gradient."""
    for t, n in ((rgb, "rgb"), (target, "target"), (dL_drgb, "dL_drgb"), (loss, "loss")):
        _f32(t, n)
    _check(lib().psdf_l2rel_loss(rgb.shape[0], _ptr(rgb), _ptr(target), _ptr(dL_drgb), _ptr(loss),
                                 lam, eps, n_images, _stream(stream)))


def grid_step(params_in: dict, params_out: dict, grads: dict, m: dict, v: dict, step: int,
              opts: StepOpts, half_out: Optional[dict] = None, losses=None, stream=None,
              bounds_out=None, s_in=None, s_out=None, work=None, losses_ext=None) -> None:
    """params_*: dict sdf, feat, probes (grids, out of place) and mlp (in place, taken from
    params_in); grads/m/v: dicts with the same keys; half_out: optional FP16 copies;
    bounds_out: optional brick bounds of the new sdf (of its FP16 copy when given).
    With opts.extended(): `work` (step_work_bytes(R) bytes; allocated when None), and
    with opts.smooth the smoothed fields s_in = G(params_in["sdf"]) (what the renderer
    read) and s_out (receives G(params_out["sdf"]))."""
    half_out = half_out or {}
    if opts.extended() and work is None:
        import torch
        work = torch.empty(step_work_bytes(params_in["sdf"].shape[0]), dtype=torch.uint8,
                           device=params_in["sdf"].device)
    R = params_in["sdf"].shape[0]
    P = params_in["probes"].shape[0]
    n_feat = params_in["feat"].shape[-1]
    n_pc = params_in["probes"][0, 0, 0].numel()
    a = _StepArgs(C.sizeof(_StepArgs), R, P, n_feat, n_pc, params_in["mlp"].numel(), step,
                  opts.lr_sdf, opts.lr_feat, opts.lr_probe, opts.lr_mlp, opts.beta1, opts.beta2,
                  opts.eps, opts.lambda_eik, opts.lambda_tv_feat, opts.lambda_tv_probe,
                  _ptr(params_in["sdf"]), _ptr(params_out["sdf"]), _ptr(params_in["feat"]),
                  _ptr(params_out["feat"]), _ptr(params_in["probes"]), _ptr(params_out["probes"]),
                  _ptr(params_in["mlp"]), _ptr(grads["sdf"]), _ptr(grads["feat"]),
                  _ptr(grads["probes"]), _ptr(grads["mlp"]), _ptr(m["sdf"]), _ptr(v["sdf"]),
                  _ptr(m["feat"]), _ptr(v["feat"]), _ptr(m["probes"]), _ptr(v["probes"]),
                  _ptr(m["mlp"]), _ptr(v["mlp"]), _ptr(half_out.get("sdf")),
                  _ptr(half_out.get("feat")), _ptr(half_out.get("probes")), _ptr(losses),
                  _ptr(bounds_out),
                  (STEP_SMOOTH if opts.smooth else 0) | (STEP_REG_WEIGHT if opts.reg_weight else 0),
                  opts.lambda_sdf, opts.lambda_normal, opts.sigma, _ptr(s_in), _ptr(s_out),
                  _ptr(work), _nbytes(work), _ptr(losses_ext))
    _check(lib().psdf_grid_step(C.byref(a), _stream(stream)))


def sphere_trace(field: Field, cams, W: int, H: int, out, eps: float = 1e-3,
                 max_steps: int = 256, flags: int = 0, stream=None) -> None:
    fs = field.cstruct()
    to = _TraceOpts(C.sizeof(_TraceOpts), eps, max_steps, flags)
    _check(lib().psdf_render_sphere_trace(C.byref(fs), C.byref(to), cams.shape[0], _ptr(cams), W, H,
                                          _ptr(out), _stream(stream)))


# ---------------------------------------------------------------------------
# real-time render: per-voxel shading, then volume rendering of the colour field
# ---------------------------------------------------------------------------
def voxel_list(sdf, band: float, list_out, count_out, stream=None) -> None:
    """Flat indices of the nodes with |sdf| <= band into list_out (int32), their
    number into count_out (int32 [1])."""
    import torch
    if list_out.dtype != torch.int32 or count_out.dtype != torch.int32:
        raise PsdfError(EINVAL, "list and count must be int32")
    _check(lib().psdf_voxel_list(sdf.shape[0], Field._dt(sdf), _ptr(sdf), band, _ptr(list_out),
                                 list_out.numel(), _ptr(count_out), _stream(stream)))


def voxel_shade(field: Field, cam, list_in, count, colour, flags: int = 0, stream=None) -> None:
    """Colours (R, R, R, 4) float32 or float16 of the listed nodes seen from the
    camera centre of cam (16,)."""
    fs = field.cstruct()
    _check(lib().psdf_voxel_shade(C.byref(fs), flags, _ptr(_f32(cam, "cam")), _ptr(list_in),
                                  _ptr(count), list_in.numel(), _ptr(colour),
                                  Field._dt(colour), _stream(stream)))


def volume_render(field: Field, opts: RenderOpts, colour, cam, W: int, H: int, out,
                  stream=None) -> None:
    """One W x H view volume-rendered through the colour grid; out (H, W, 3)."""
    fs, op = field.cstruct(), opts.cstruct()
    _check(lib().psdf_volume_render(C.byref(fs), C.byref(op), _ptr(colour), Field._dt(colour),
                                    _ptr(_f32(cam, "cam")), W, H, _ptr(_f32(out, "out")),
                                    _stream(stream)))


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
def render(field: Field, opts: RenderOpts, rays_o, rays_d, tape_samples: Optional[int] = None):
    """Differentiable render: returns rgb (B, 3); gradients flow to field.sdf,
    field.feat, field.probes and field.mlp through the HIP backward kernels.

    The forward records its shaded samples into a tape (a backward workspace with
    room for `tape_samples` samples; default 8 per ray, or N - 1 per ray without
    the skip rule, capped at 2^24) that the backward reads (PSDF_BWD_FROM_TAPE).
    Waves whose samples do not fit the tape are re-marched, so any size gives the
    same gradients.  Gradients take the dtype of their parameter: FP16 feature or
    probe tensors receive FP16 gradients (one rounding of the FP32 sums, coarse
    below 6e-5 where FP16 is subnormal); keep FP32 masters for training (grid_step
    writes FP16 render copies of them)."""
    return _RenderFn.apply(field.sdf, field.feat, field.probes, field.mlp, field.mlp_dtype, opts,
                           rays_o, rays_d, field.bounds, tape_samples, (field.hidden, field.layers))


def is_paper_model(field: Field, flags: int) -> bool:
    """True when the render runs the paper colour model's kernels (no tape)."""
    return (field.hidden, field.layers) != (HIDDEN, 1) or field.tiles is not None or bool(
        flags & (FLAG_SH_REFLECT | FLAG_FRESNEL_PAPER))


def _default_tape_samples(B: int, opts: RenderOpts) -> int:
    per_ray = 8 if opts.skip_voxels > 0 else max(opts.n_samples - 1, 1)
    return min(B * per_ray, 1 << 24)


def _make_autograd():
    import torch

    class RenderFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sdf, feat, probes, mlp, mlp_dtype, opts, rays_o, rays_d, bounds,
                    tape_samples, shape):
            B = rays_o.shape[0]
            rgb = torch.empty((B, 3), device=rays_o.device, dtype=torch.float32)
            aux = torch.empty((B, 4), device=rays_o.device, dtype=torch.float32)
            fld = Field(sdf, feat, probes, mlp, mlp_dtype, bounds, *shape)
            tape = None
            if not is_paper_model(fld, opts.flags):  # the paper model's backward re-marches
                cap = _default_tape_samples(B, opts) if tape_samples is None else int(tape_samples)
                tape = backward_workspace(max(B, 1), probes.shape[0], cap, device=rays_o.device)
            render_forward(fld, opts, rays_o, rays_d, rgb, aux, tape=tape)
            ctx.save_for_backward(sdf, feat, probes, mlp, rays_o, rays_d, aux)
            ctx.tape = tape
            ctx.bounds, ctx.shape = bounds, shape
            ctx.mlp_dtype, ctx.opts = mlp_dtype, opts
            return rgb

        @staticmethod
        def backward(ctx, g_rgb):
            sdf, feat, probes, mlp, rays_o, rays_d, aux = ctx.saved_tensors
            fld = Field(sdf, feat, probes, mlp, ctx.mlp_dtype, ctx.bounds, *ctx.shape)
            gs = torch.zeros(sdf.shape, device=sdf.device, dtype=torch.float32)
            gf = torch.zeros(feat.shape, device=sdf.device, dtype=torch.float32)
            gp = torch.zeros(probes.shape, device=sdf.device, dtype=torch.float32)
            gm = torch.zeros(mlp.shape, device=sdf.device, dtype=torch.float32)
            # the tape is read once: a second backward through the same graph (retain_graph)
            # re-marches with the tape as scratch
            tape = ctx.tape
            from_tape = tape is not None and not getattr(ctx, "tape_used", False)
            render_backward(fld, ctx.opts, rays_o, rays_d, aux, g_rgb.float().contiguous(),
                            dict(sdf=gs, feat=gf, probes=gp, mlp=gm), workspace=tape,
                            from_tape=from_tape)
            ctx.tape_used = True
            return (gs.to(sdf.dtype), gf.to(feat.dtype), gp.to(probes.dtype), gm, None, None,
                    None, None, None, None, None)

    return RenderFn


class _Lazy:
    def __init__(self):
        self._fn = None

    def apply(self, *a):
        if self._fn is None:
            self._fn = _make_autograd()
        return self._fn.apply(*a)


_RenderFn = _Lazy()
