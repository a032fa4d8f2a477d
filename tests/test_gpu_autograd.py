"""The torch.autograd path (paper_2412_10084_amd.render): its forward against the
FP64 oracle, its backward (taped schedule) against the oracle's analytic gradient
and against render_backward called directly, a second backward through the same
graph (re-marched), and the binding's refusal of strided or host tensors."""
import numpy as np
import pytest

import oracle
from gpu_common import (FP32_COLOR_ABS, FP32_COLOR_REL, SKIP_MARGIN, color_check, dev,
                        device_field, gpu_backward, grad_check, rays, scene, torch)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("skip,N", [(0.0, 64), (4.0, 96)])
def test_autograd_matches_oracle_and_direct_backward(skip, N):
    import paper_2412_10084_amd as ps
    t = torch()
    f = scene(0, 64, 16)
    ft = scene(1, 64, 16, shape="torus")
    o, d = rays(8, 32, 16)
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o, d, N, skip_voxels=skip)
    keep = ref["margin"] > SKIP_MARGIN
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N, skip_voxels=skip)["rgb"]
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    dL[~keep] = 0.0
    g_ref = oracle.render_backward(of, o, d, dL, N, skip_voxels=skip)

    fld = device_field(f)
    if skip > 0:
        fld.bounds = ps.sdf_bounds(fld.sdf)
    for k in ("sdf", "feat", "probes", "mlp"):
        getattr(fld, k).requires_grad_(True)
    opts = ps.RenderOpts(N, 64.0, skip, 0)
    do, dd = dev(o), dev(d)
    print(f"autograd case: B={o.shape[0]} N={N} skip={skip}", flush=True)
    rgb = ps.render(fld, opts, do, dd)
    w = dev(dL.astype(np.float32))
    (rgb * w).sum().backward(retain_graph=True)
    t.cuda.synchronize()
    nbad, emax = color_check(rgb.detach().cpu().numpy(), ref["rgb"], FP32_COLOR_REL,
                             FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    g = {k: getattr(fld, k).grad.cpu().numpy().astype(np.float64)
         for k in ("sdf", "feat", "probes", "mlp")}
    grad_check(g, g_ref, "fp32")

    # the same gradients from the raw entry points (taped forward + backward)
    raw = ps.Field(*(getattr(fld, k).detach() for k in ("sdf", "feat", "probes", "mlp")),
                   bounds=fld.bounds)
    tape = ps.backward_workspace(o.shape[0], f.P, o.shape[0] * (N - 1))
    rgb2 = t.empty_like(rgb)
    aux = t.empty((o.shape[0], 4), device="cuda")
    ps.render_forward(raw, opts, do, dd, rgb2, aux, tape=tape)
    g_direct = gpu_backward(raw, do, dd, aux, dL, N, skip=skip, workspace=tape, from_tape=True)
    np.testing.assert_array_equal(rgb2.cpu().numpy(), rgb.detach().cpu().numpy())
    grad_check(g, g_direct, "fp32")

    # a second backward through the same graph re-marches (the tape was consumed)
    for k in ("sdf", "feat", "probes", "mlp"):
        getattr(fld, k).grad = None
    (rgb * w).sum().backward()
    t.cuda.synchronize()
    g2 = {k: getattr(fld, k).grad.cpu().numpy().astype(np.float64)
          for k in ("sdf", "feat", "probes", "mlp")}
    grad_check(g2, g_ref, "fp32")


def test_autograd_small_tape_and_fp16_storage():
    """A tape too small for the batch (overflowing waves re-march) and FP16 features:
    gradients flow back as FP16 tensors of the parameters' dtype and match the
    direct entry points' FP32 gradients to one FP16 rounding (those are held to the
    oracle)."""
    import paper_2412_10084_amd as ps
    t = torch()
    f = scene(0, 64, 16)
    ft = scene(1, 64, 16, shape="torus")
    o, d = rays(8, 32, 16)
    N = 64
    of_h = oracle.field_from(f, half=True, mlp_round="f16")
    ref = oracle.render_forward(of_h, o, d, N)
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N)["rgb"]
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    g_ref = oracle.render_backward(of_h, o, d, dL, N)
    fld = device_field(f, feat_half=True, mlp_dtype=ps.F16)
    for k in ("sdf", "feat", "probes", "mlp"):
        getattr(fld, k).requires_grad_(True)
    opts = ps.RenderOpts(N, 64.0, 0.0, 0)
    do, dd = dev(o), dev(d)
    rgb = ps.render(fld, opts, do, dd, tape_samples=500)
    (rgb * dev(dL.astype(np.float32))).sum().backward()
    t.cuda.synchronize()
    assert np.abs(rgb.detach().cpu().numpy() - ref["rgb"]).max() <= 2e-3
    assert fld.feat.grad.dtype == t.float16
    g = {k: getattr(fld, k).grad.float().cpu().numpy().astype(np.float64)
         for k in ("sdf", "feat", "probes", "mlp")}
    raw = ps.Field(*(getattr(fld, k).detach() for k in ("sdf", "feat", "probes", "mlp")),
                   mlp_dtype=ps.F16)
    aux = t.empty((o.shape[0], 4), device="cuda")
    ps.render_forward(raw, opts, do, dd, t.empty_like(rgb), aux)
    g_direct = gpu_backward(raw, do, dd, aux, dL, N)
    grad_check(g_direct, g_ref, "f16")
    # FP16 parameters receive FP16 gradients: one rounding of the FP32 gradient (half an
    # ulp, 2^-11 relative, 2^-25 absolute in the subnormal range) beside the summation order
    for k in ("feat", "probes"):
        err = np.abs(g[k] - g_direct[k])
        bound = 2.0 ** -11 * np.abs(g_direct[k]) + 2.0 ** -25 + 1e-6 * np.abs(g_direct[k]).max()
        assert np.all(err <= bound), k
    grad_check({k: g[k] for k in ("sdf", "mlp")}, g_direct, "fp32", keys=("sdf", "mlp"))


def test_binding_rejects_strided_device_tensors():
    import paper_2412_10084_amd as ps
    t = torch()
    f = scene(0, 16, 4)
    fld = device_field(f)
    o, d = rays(1, 8, 4)
    do = dev(np.concatenate([o, o], axis=1))[:, ::2]  # a strided view of the right shape
    assert not do.is_contiguous()
    rgb = t.empty((o.shape[0], 3), device="cuda")
    with pytest.raises(ps.PsdfError, match="contiguous"):
        ps.render_forward(fld, ps.RenderOpts(16, 64.0, 0.0, 0), do, dev(d), rgb)
