"""GPU parity of the entry-parallel backward schedule (march -> per-entry
shading reverse mode -> per-ray opacity walk) against the FP64 oracle, and
against the fused schedule, including workspaces too small for the batch (the
waves that do not fit fall back to the fused kernel)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_common import (BF16_GRAD_REL, F16_GRAD_REL, FP32_GRAD_REL, FP32_MLP_GRAD_REL,
                        SKIP_MARGIN, device_field, gpu_backward, gpu_forward, grad_check, rays,
                        scene, torch)

pytestmark = pytest.mark.gpu

TOL = (("sdf", FP32_GRAD_REL), ("feat", FP32_GRAD_REL), ("probes", FP32_GRAD_REL),
       ("mlp", FP32_MLP_GRAD_REL))


def _case(N=96, skip=4.0, B=4093, flags=0, seed=0, shape="sphere", R=64, P=16):
    f = scene(seed, R, P, shape=shape)
    ft = scene(seed + 1, R, P, shape="torus")
    o, d = rays(8, 32, 16)
    o, d = o[:B], d[:B]
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o, d, N, skip_voxels=skip, flags=flags)
    keep = ref["margin"] > SKIP_MARGIN
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N, skip_voxels=skip, flags=flags)["rgb"]
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    dL[~keep] = 0.0
    g_ref = oracle.render_backward(of, o, d, dL, N, skip_voxels=skip, flags=flags)
    return f, o, d, dL, g_ref


def _check(g, g_ref, tol=TOL):
    grad_check(g, g_ref, "fp32", keys=tuple(k for k, _ in tol))


@pytest.mark.parametrize("cap", [1 << 20, 1000, 64, 0])
def test_split_backward_matches_oracle(cap):
    import paper_2412_10084_amd as ps
    N, skip = 96, 4.0
    f, o, d, dL, g_ref = _case(N, skip)
    fld = device_field(f)
    fld.bounds = ps.sdf_bounds(fld.sdf)
    fw = gpu_forward(fld, o, d, N, skip=skip)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N, skip=skip, workspace=cap)
    _check(g, g_ref)
    g_fused = gpu_backward(fld, do, dd, aux, dL, N, skip=skip)
    grad_check(g, g_fused, "fp32")


@pytest.mark.parametrize("flags", [1, 2, 4])
def test_split_backward_flags(flags):
    N, skip = 64, 2.0
    f, o, d, dL, g_ref = _case(N, skip, B=2048, flags=flags, shape="torus")
    fld = device_field(f)
    fw = gpu_forward(fld, o, d, N, skip=skip, flags=flags)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N, skip=skip, flags=flags, workspace=1 << 16)
    _check(g, g_ref)


def test_split_backward_no_skip_and_partial_groups():
    N = 64
    f, o, d, dL, g_ref = _case(N, 0.0, B=1500)
    fld = device_field(f)
    fw = gpu_forward(fld, o, d, N)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N, workspace=1 << 18, groups=("sdf", "probes"))
    _check(g, g_ref, (("sdf", FP32_GRAD_REL), ("probes", FP32_GRAD_REL)))
    assert not g["feat"].any() and not g["mlp"].any()
    g = gpu_backward(fld, do, dd, aux, dL, N, workspace=1 << 18, groups=("feat", "mlp"))
    _check(g, g_ref, (("feat", FP32_GRAD_REL), ("mlp", FP32_MLP_GRAD_REL)))
    assert not g["sdf"].any()


@pytest.mark.parametrize("mlp_dt,gtol", [(1, F16_GRAD_REL), (2, BF16_GRAD_REL)])
def test_split_backward_mixed(mlp_dt, gtol):
    f = scene(0, 64, 16)
    ft = scene(1, 64, 16, shape="torus")
    o, d = rays(8, 32, 16)
    N = 64
    of_h = oracle.field_from(f, half=True, mlp_round=("f16", "bf16")[mlp_dt - 1])
    ref = oracle.render_forward(of_h, o, d, N)
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N)["rgb"]
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    g_ref = oracle.render_backward(of_h, o, d, dL, N)
    fld = device_field(f, feat_half=True, mlp_dtype=mlp_dt)
    fw = gpu_forward(fld, o, d, N)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N, workspace=1 << 18)
    grad_check(g, g_ref, ("f16", "bf16")[mlp_dt - 1])


def test_split_backward_empty_loss():
    f = scene(0, 64, 16)
    o, d = rays(2, 32, 16)
    fld = device_field(f)
    fw = gpu_forward(fld, o, d, 64)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, np.zeros((o.shape[0], 3)), 64, workspace=1 << 12)
    for k in g:
        assert not g[k].any(), k


def test_split_backward_train256_full_size_sampled():
    """The benchmark's launch: full train256 batch, brick bounds, workspace for
    4 shaded samples per ray; loss gradient on a sample of rays checked against
    the oracle."""
    import paper_2412_10084_amd as ps
    w = wl.WORKLOADS["train256"]
    f = scene(0, w.R, w.P)
    o, d = rays(w.views, w.W, w.H)
    fld = device_field(f)
    fld.bounds = ps.sdf_bounds(fld.sdf)
    got = gpu_forward(fld, o, d, w.n_samples, skip=w.skip_voxels)
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(o.shape[0], 3000, replace=False))
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o[idx], d[idx], w.n_samples, skip_voxels=w.skip_voxels)
    keep = ref["margin"] > SKIP_MARGIN
    sel = idx[keep][:1500]
    dL = np.zeros((o.shape[0], 3))
    dL[sel] = rng.choice([-1.0, 1.0], size=(sel.size, 3)) / (3.0 * o.shape[0])
    do, dd, _, aux = got["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, w.n_samples, skip=w.skip_voxels,
                     workspace=4 * o.shape[0])
    g_ref = oracle.render_backward(of, o[sel], d[sel], dL[sel], w.n_samples,
                                   skip_voxels=w.skip_voxels)
    _check(g, g_ref)


# ---------------------------------------------------------------------------
# taped schedule: the forward records its shaded samples, the backward reads them
# ---------------------------------------------------------------------------
def _tape_run(f, o, d, dL, N, skip, cap, flags=0, groups=("sdf", "feat", "probes", "mlp"),
              feat_half=False, mlp_dtype=0, bounds=True):
    import paper_2412_10084_amd as ps
    fld = device_field(f, feat_half=feat_half, mlp_dtype=mlp_dtype)
    if bounds:
        fld.bounds = ps.sdf_bounds(fld.sdf)
    tape = ps.backward_workspace(o.shape[0], fld.probes.shape[0], cap)
    plain = gpu_forward(fld, o, d, N, skip=skip, flags=flags)
    fw = gpu_forward(fld, o, d, N, skip=skip, flags=flags, tape=tape)
    for k in ("rgb", "aux", "depth_wsum"):  # recording changes no output
        np.testing.assert_array_equal(fw[k], plain[k], err_msg=k)
    do, dd, _, aux = fw["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N, skip=skip, flags=flags, workspace=tape,
                     groups=groups, from_tape=True)
    return fld, fw, g


@pytest.mark.parametrize("cap", [1 << 20, 1000, 64, 0])
def test_tape_backward_matches_oracle(cap):
    N, skip = 96, 4.0
    f, o, d, dL, g_ref = _case(N, skip)
    fld, fw, g = _tape_run(f, o, d, dL, N, skip, cap)
    _check(g, g_ref)
    do, dd, _, aux = fw["dev"]
    g_fused = gpu_backward(fld, do, dd, aux, dL, N, skip=skip)
    grad_check(g, g_fused, "fp32")


@pytest.mark.parametrize("flags", [1, 2, 4])
def test_tape_backward_flags(flags):
    N, skip = 64, 2.0
    f, o, d, dL, g_ref = _case(N, skip, B=2048, flags=flags, shape="torus")
    _, _, g = _tape_run(f, o, d, dL, N, skip, 1 << 16, flags=flags)
    _check(g, g_ref)


def test_tape_backward_no_skip_and_partial_groups():
    N = 64
    f, o, d, dL, g_ref = _case(N, 0.0, B=1500)
    _, _, g = _tape_run(f, o, d, dL, N, 0.0, 1 << 18, groups=("sdf", "probes"), bounds=False)
    _check(g, g_ref, (("sdf", FP32_GRAD_REL), ("probes", FP32_GRAD_REL)))
    assert not g["feat"].any() and not g["mlp"].any()
    _, _, g = _tape_run(f, o, d, dL, N, 0.0, 1 << 18, groups=("feat", "mlp"), bounds=False)
    _check(g, g_ref, (("feat", FP32_GRAD_REL), ("mlp", FP32_MLP_GRAD_REL)))
    assert not g["sdf"].any()


@pytest.mark.parametrize("skip", [0.0, 4.0])
def test_tape_backward_far_successors(skip):
    """Samples about ten cells apart (R = 96, N = 16) with a dense loss gradient: in a
    batch of one block of probe cells, the next-sample corners of the batch's last
    shaded samples no longer fit the LDS box with the samples' own patches, so the
    box holds the patches and those corners go to the grid directly."""
    N = 16
    f, o, d, dL, g_ref = _case(N, skip, B=4096, R=96, P=24)
    assert np.count_nonzero(dL.any(axis=1)) > 1000
    fld, fw, g = _tape_run(f, o, d, dL, N, skip, 1 << 18)
    _check(g, g_ref)
    do, dd, _, aux = fw["dev"]
    g_fused = gpu_backward(fld, do, dd, aux, dL, N, skip=skip)
    grad_check(g, g_fused, "fp32")


@pytest.mark.parametrize("mlp_dt,gtol", [(1, F16_GRAD_REL), (2, BF16_GRAD_REL)])
def test_tape_backward_mixed(mlp_dt, gtol):
    f = scene(0, 64, 16)
    ft = scene(1, 64, 16, shape="torus")
    o, d = rays(8, 32, 16)
    N = 64
    of_h = oracle.field_from(f, half=True, mlp_round=("f16", "bf16")[mlp_dt - 1])
    ref = oracle.render_forward(of_h, o, d, N)
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N)["rgb"]
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    g_ref = oracle.render_backward(of_h, o, d, dL, N)
    _, _, g = _tape_run(f, o, d, dL, N, 0.0, 1 << 18, feat_half=True, mlp_dtype=mlp_dt,
                        bounds=False)
    grad_check(g, g_ref, ("f16", "bf16")[mlp_dt - 1])


def test_tape_backward_train256_full_size_sampled():
    """The benchmark's launch: full train256 batch, brick bounds, forward tape with
    room for 8 shaded samples per ray, backward from the tape."""
    w = wl.WORKLOADS["train256"]
    f = scene(0, w.R, w.P)
    o, d = rays(w.views, w.W, w.H)
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(o.shape[0], 3000, replace=False))
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o[idx], d[idx], w.n_samples, skip_voxels=w.skip_voxels)
    keep = ref["margin"] > SKIP_MARGIN
    sel = idx[keep][:1500]
    dL = np.zeros((o.shape[0], 3))
    dL[sel] = rng.choice([-1.0, 1.0], size=(sel.size, 3)) / (3.0 * o.shape[0])
    _, _, g = _tape_run(f, o, d, dL, w.n_samples, w.skip_voxels, 8 * o.shape[0])
    g_ref = oracle.render_backward(of, o[sel], d[sel], dL[sel], w.n_samples,
                                   skip_voxels=w.skip_voxels)
    _check(g, g_ref)
