"""Shared helpers of the GPU parity tests: device copies of seeded scenes and
the comparison rules.  Inputs come from workloads; expected values from the
oracle only."""
from __future__ import annotations

import functools

import numpy as np

import oracle
import workloads as wl

# FP32 colour: |d| <= REL * |c_ref| + ABS  (derivation: see the design notes)
FP32_COLOR_REL = 1e-5
FP32_COLOR_ABS = 1e-6
FP32_GRAD_REL = 1e-5     # norm-relative, grids
FP32_MLP_GRAD_REL = 1e-4  # norm-relative, MLP (sums over many samples)
F16_COLOR_ABS = 2e-3
BF16_COLOR_ABS = 5e-3
F16_GRAD_REL = 1e-2
BF16_GRAD_REL = 3e-2
SKIP_MARGIN = 1e-5        # rays whose |s| passes this close to the skip threshold are excluded


def torch():
    import torch as _t
    return _t


def dev(a, dtype=None):
    t = torch()
    x = t.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        x = x.to(dtype)
    return x.cuda()


def device_field(f: wl.Field, feat_half=False, sdf_half=False, mlp_dtype=0):
    import paper_2412_10084_amd as ps
    t = torch()
    fdt = t.float16 if feat_half else t.float32
    sdt = t.float16 if sdf_half else t.float32
    return ps.Field(sdf=dev(f.sdf, sdt), feat=dev(f.feat, fdt), probes=dev(f.probes, fdt),
                    mlp=dev(f.mlp), mlp_dtype=mlp_dtype)


@functools.lru_cache(maxsize=None)
def scene(seed: int, R: int, P: int, n_sh: int = 9, shape: str = "sphere") -> wl.Field:
    return wl.random_field(seed, R, P, n_sh=n_sh, shape=shape)


@functools.lru_cache(maxsize=None)
def rays(views: int, W: int, H: int, order: str = "image"):
    cams = wl.fibonacci_cameras(views, W, H)
    return wl.camera_rays(cams, W, H, order)


def gpu_forward(fld, o, d, N, tau=64.0, skip=0.0, flags=0, tape=None):
    import paper_2412_10084_amd as ps
    t = torch()
    B = o.shape[0]
    do, dd = dev(o), dev(d)
    rgb = t.empty((B, 3), device="cuda")
    aux = t.empty((B, 4), device="cuda")
    dw = t.empty((B, 2), device="cuda")
    ps.render_forward(fld, ps.RenderOpts(N, tau, skip, flags), do, dd, rgb, aux, dw, tape=tape)
    t.cuda.synchronize()
    return dict(rgb=rgb.cpu().numpy(), aux=aux.cpu().numpy(), depth_wsum=dw.cpu().numpy(),
                dev=(do, dd, rgb, aux))


def gpu_backward(fld, o_dev, d_dev, aux_dev, dL, N, tau=64.0, skip=0.0, flags=0, workspace=None,
                 groups=("sdf", "feat", "probes", "mlp"), from_tape=False):
    """workspace: None (fused schedule), an int (entry-parallel schedule with room for that
    many shaded samples) or a device buffer (with from_tape: the forward's tape)."""
    import paper_2412_10084_amd as ps
    t = torch()
    g = dict(sdf=t.zeros(fld.sdf.shape, device="cuda"), feat=t.zeros(fld.feat.shape, device="cuda"),
             probes=t.zeros(fld.probes.shape, device="cuda"), mlp=t.zeros(227, device="cuda"))
    if isinstance(workspace, int):
        workspace = ps.backward_workspace(o_dev.shape[0], fld.probes.shape[0], workspace)
    ps.render_backward(fld, ps.RenderOpts(N, tau, skip, flags), o_dev, d_dev, aux_dev,
                       dev(dL.astype(np.float32)), {k: g[k] for k in groups}, workspace=workspace,
                       from_tape=from_tape)
    t.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}


def color_check(got, ref, rel, abs_, mask=None):
    err = np.abs(got - ref)
    bound = rel * np.abs(ref) + abs_
    bad = err > bound
    if mask is not None:
        bad &= mask[:, None]
    return int(bad.sum()), float(err.max(initial=0.0))


def norm_rel(got, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / max(den, 1e-30))
