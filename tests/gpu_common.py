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
# rays whose |s| passes this close to the skip threshold are excluded: the FP32 trilinear
# value near the threshold (4 voxels, node values below ~0.05) errs by a few 1e-8, so a
# decision within 1e-6 of the threshold is the only one FP32 and FP64 can take differently
SKIP_MARGIN = 1e-6

# Element-wise gradient bound, beside the norm bound: |d_k| <= rtol |ref_k| + atol max|ref|.
# FP32 sums of many contributions in an arbitrary order (FP32 atomics, or the taped box
# pass's 32-bit fixed point with error below B / 2^25 per add, B the batch's largest
# contribution) carry errors relative to the largest gradient, hence the atol term; the
# mixed paths round the MLP's operands to FP16 / BF16, which no FP64 reference reproduces.
GRAD_TOL = {
    # prec: (norm grids, norm mlp, (rtol, atol) grids, (rtol, atol) mlp)
    "fp32": (FP32_GRAD_REL, FP32_MLP_GRAD_REL, (1e-3, 1e-6), (1e-3, 1e-5)),
    "f16": (F16_GRAD_REL, F16_GRAD_REL, (5e-2, 3e-2), (5e-2, 3e-2)),
    "bf16": (BF16_GRAD_REL, BF16_GRAD_REL, (2e-1, 1.5e-1), (2e-1, 1.5e-1)),
    # the paper's MLP (two ReLU layers of 32): operand rounding flips the ReLU mask of
    # more units, and a flipped unit changes a sample's gradient by its whole term, so
    # these errors grow like sqrt(u) (BF16 / FP16 measured ~3 = sqrt(8)), not like u
    "f16_paper": (2e-2, 2e-2, (1e-1, 1e-1), (1e-1, 1e-1)),
    "bf16_paper": (6e-2, 6e-2, (3e-1, 3e-1), (3e-1, 3e-1)),
}


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


def elem_check(got, ref, rtol, atol):
    """(number of entries outside rtol |ref| + atol max|ref|, worst err / bound)"""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    bound = rtol * np.abs(ref) + atol * max(float(np.abs(ref).max(initial=0.0)), 1e-30)
    err = np.abs(got - ref)
    return int((err > bound).sum()), float((err / bound).max(initial=0.0))


def grad_errors(g, g_ref, keys=("sdf", "feat", "probes", "mlp")):
    """Per group: (norm-relative error, max |d| / max |ref|)."""
    out = {}
    for k in keys:
        d = np.abs(np.asarray(g[k], np.float64) - np.asarray(g_ref[k], np.float64))
        out[k] = (norm_rel(g[k], g_ref[k]),
                  float(d.max(initial=0.0) / max(float(np.abs(g_ref[k]).max(initial=0.0)), 1e-30)))
    return out


def grad_check(g, g_ref, prec="fp32", keys=("sdf", "feat", "probes", "mlp")):
    """Norm-relative and element-wise bounds of gradient groups against a reference
    (every group is checked before the first failure is reported)."""
    n_grid, n_mlp, e_grid, e_mlp = GRAD_TOL[prec]
    fails = []
    for k in keys:
        nt, (rt, at) = (n_mlp, e_mlp) if k == "mlp" else (n_grid, e_grid)
        e = norm_rel(g[k], g_ref[k])
        if not e <= nt:
            fails.append(f"{k}: norm-relative {e:.3g} > {nt}")
        nbad, worst = elem_check(g[k], g_ref[k], rt, at)
        if nbad:
            fails.append(f"{k}: {nbad} entries outside {rt:g} |ref| + {at:g} max|ref| "
                         f"(worst {worst:.3g} x bound)")
    assert not fails, "; ".join(fails) + f" [all groups: {grad_errors(g, g_ref, keys)}]"
