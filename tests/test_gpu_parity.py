"""GPU parity: the HIP render step (through the C ABI) against the FP64 oracle.

Inputs are the seeded synthetic scenes of `workloads`; expected values come
only from the oracle.  FP32 paths use the tolerances in gpu_common; rays whose
SDF passes within SKIP_MARGIN of the skip threshold are excluded (a decision
that FP32 and FP64 may legitimately take differently) and counted.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_common import (FP32_COLOR_ABS, FP32_COLOR_REL, FP32_GRAD_REL, FP32_MLP_GRAD_REL,
                        SKIP_MARGIN, color_check, dev, device_field, gpu_backward, gpu_forward,
                        grad_check, norm_rel, rays, scene, torch)

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------------------
# forward, small workload (64^3 / 16^3, 8 x 32x16 rays, N = 64, no skip)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("flags", [0, 1, 2, 4])
def test_forward_fwd64(flags):
    f = scene(0, 64, 16)
    o, d = rays(8, 32, 16)
    ref = oracle.render_forward(oracle.field_from(f), o, d, 64, tau=64.0, flags=flags)
    got = gpu_forward(device_field(f), o, d, 64, flags=flags)
    nbad, emax = color_check(got["rgb"], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} colour values out of tolerance, max err {emax:.3g}"
    np.testing.assert_allclose(got["aux"][:, 3], ref["aux"][:, 3], rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(got["depth_wsum"], ref["depth_wsum"], rtol=1e-5, atol=1e-5)
    assert np.count_nonzero(ref["rgb"].sum(1)) > 1000


@pytest.mark.parametrize("n_sh", [1, 4, 16])
def test_forward_sh_orders(n_sh):
    f = scene(3, 32, 8, n_sh=n_sh)
    o, d = rays(4, 16, 8)
    ref = oracle.render_forward(oracle.field_from(f), o, d, 48, tau=32.0)
    got = gpu_forward(device_field(f), o, d, 48, tau=32.0)
    nbad, emax = color_check(got["rgb"], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} bad, max err {emax:.3g}"


def test_forward_skip_rule_and_ragged_batch():
    f = scene(0, 64, 16)
    o, d = rays(8, 32, 16)
    o, d = o[:4093], d[:4093]  # not a multiple of the wave or block size
    ref = oracle.render_forward(oracle.field_from(f), o, d, 96, tau=64.0, skip_voxels=4.0)
    got = gpu_forward(device_field(f), o, d, 96, skip=4.0)
    keep = ref["margin"] > SKIP_MARGIN
    assert keep.mean() > 0.99
    nbad, emax = color_check(got["rgb"], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} bad, max err {emax:.3g}"


def test_forward_edge_rays():
    f = scene(0, 64, 16)
    o = np.array([[3, 3, 0], [0, 0, 0], [0.2, -0.1, 0.95], [1.0, 0.3, 0.2], [3, 0, 0],
                  [-0.999, -0.999, -0.999], [0, 0, 5]], dtype=np.float32)
    d = np.array([[-1, 0, 0], [0.3, 0.2, 0.9], [0, 0, -1], [-1, 0, 0], [-1, 1e-4, 0],
                  [1, 1, 1], [0, 0, -2]], dtype=np.float32)
    ref = oracle.render_forward(oracle.field_from(f), o, d, 64)
    got = gpu_forward(device_field(f), o, d, 64)
    nbad, emax = color_check(got["rgb"], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} bad, max err {emax:.3g}"
    assert np.all(got["rgb"][0] == 0)  # misses the cube
    # one ray, B = 1
    got1 = gpu_forward(device_field(f), o[1:2], d[1:2], 64)
    np.testing.assert_array_equal(got1["rgb"], got["rgb"][1:2])


def test_forward_deterministic():
    f = scene(0, 64, 16)
    o, d = rays(8, 32, 16)
    fld = device_field(f)
    a = gpu_forward(fld, o, d, 64)
    b = gpu_forward(fld, o, d, 64)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])


def test_empty_batch_is_noop():
    import paper_2412_10084_amd as ps
    t = torch()
    f = scene(0, 16, 4)
    fld = device_field(f)
    e = t.empty((0, 3), device="cuda")
    ps.render_forward(fld, ps.RenderOpts(16), e, e, e)
    t.cuda.synchronize()


# ---------------------------------------------------------------------------
# backward, small: 64^3 / 16^3, L1 loss against the torus target
# ---------------------------------------------------------------------------
def _loss_grad(rgb_ref, tgt):
    _, dL = oracle.l1_loss(rgb_ref, tgt)
    return dL


@pytest.mark.parametrize("skip,N", [(0.0, 64), (4.0, 128)])
def test_backward_small(skip, N):
    f = scene(0, 64, 16)
    ft = scene(1, 64, 16, shape="torus")
    o, d = rays(8, 32, 16)
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o, d, N, skip_voxels=skip)
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N, skip_voxels=skip)["rgb"]
    dL = _loss_grad(ref["rgb"], tgt)
    if skip > 0:
        dL[ref["margin"] <= SKIP_MARGIN] = 0.0
    g_ref = oracle.render_backward(of, o, d, dL, N, skip_voxels=skip)
    fld = device_field(f)
    fw = gpu_forward(fld, o, d, N, skip=skip)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N, skip=skip)
    grad_check(g, g_ref, "fp32")
    for k in g_ref:
        assert np.linalg.norm(g_ref[k]) > 0


def test_backward_accumulates_and_null_groups():
    f = scene(0, 32, 8)
    o, d = rays(4, 16, 8)
    fld = device_field(f)
    fw = gpu_forward(fld, o, d, 32)
    do, dd, _, aux = fw["dev"]
    dL = np.random.default_rng(5).standard_normal((o.shape[0], 3)) * 1e-3
    g1 = gpu_backward(fld, do, dd, aux, dL, 32)
    import paper_2412_10084_amd as ps
    t = torch()
    g = dict(sdf=t.zeros(fld.sdf.shape, device="cuda"), feat=None, probes=None,
             mlp=t.zeros(227, device="cuda"))
    ps.render_backward(fld, ps.RenderOpts(32), do, dd, aux, dev(dL.astype(np.float32)), g)
    ps.render_backward(fld, ps.RenderOpts(32), do, dd, aux, dev(dL.astype(np.float32)), g)
    t.cuda.synchronize()
    assert norm_rel(g["sdf"].cpu().numpy() / 2, g1["sdf"]) < 1e-6
    assert norm_rel(g["mlp"].cpu().numpy() / 2, g1["mlp"]) < 1e-6


# ---------------------------------------------------------------------------
# L1 loss kernel
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B", [5000, 5001, 262144])  # float4 path, scalar path, train256 batch
def test_l1_loss_kernel(B):
    import paper_2412_10084_amd as ps
    t = torch()
    rng = np.random.default_rng(3)
    rgb = rng.uniform(size=(B, 3)).astype(np.float32)
    tgt = rng.uniform(size=(B, 3)).astype(np.float32)
    tgt[:7] = rgb[:7]
    loss_ref, dL_ref = oracle.l1_loss(rgb, tgt)
    dL = t.empty((B, 3), device="cuda")
    loss = t.empty(1, device="cuda")
    ps.l1_loss(dev(rgb), dev(tgt), dL, loss)
    t.cuda.synchronize()
    np.testing.assert_array_equal(dL.cpu().numpy(), dL_ref.astype(np.float32))
    assert abs(loss.item() - loss_ref) <= 1e-6 * loss_ref
