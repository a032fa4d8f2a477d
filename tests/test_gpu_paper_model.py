"""GPU parity of the paper's own colour model (Sec. 3.1 Eq. newparametrization:
SH at the reflected vector r, incidence inputs (1 - n.v)^0..5; Sec. 4: two hidden
layers of 32, up to 16 SH coefficients) against the FP64 oracle: forward colour,
log-transmittance, depth and weight sum, and every gradient group, with and
without the skip rule, the ablation flags, FP16 / BF16 arithmetic, the full-size
train256 launch on sampled rays, and the autograd path."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_common import (BF16_COLOR_ABS, F16_COLOR_ABS, FP32_COLOR_ABS, FP32_COLOR_REL,
                        SKIP_MARGIN, color_check, dev, grad_check, rays, torch)

pytestmark = pytest.mark.gpu

REFLECT, FRESNEL = 8, 16
PAPER = REFLECT | FRESNEL


def model_field(seed, R, P, n_sh, hidden, layers, flags, shape="sphere"):
    """Seeded scene whose MLP matches the colour model (Xavier, inputs by flags)."""
    f = wl.random_field(seed, R, P, n_sh=n_sh, shape=shape)
    n_in = wl.N_FEAT + wl.N_ANG + (6 if flags & FRESNEL else 3)
    f.mlp = wl.xavier_uniform_mlp(np.random.default_rng(seed + 100), n_in, hidden, wl.N_OUT, layers)
    f.hidden, f.layers = hidden, layers
    return f


def gpu_field(f, half=False, mlp_dtype=0, bounds=False):
    import paper_2412_10084_amd as ps
    t = torch()
    fdt = t.float16 if half else t.float32
    sdf = dev(f.sdf)
    return ps.Field(sdf=sdf, feat=dev(f.feat, fdt), probes=dev(f.probes, fdt),
                    mlp=dev(f.mlp), mlp_dtype=mlp_dtype, hidden=f.hidden, layers=f.layers,
                    bounds=ps.sdf_bounds(sdf) if bounds else None)


def run(fld, o, d, N, skip, flags, dL=None):
    import paper_2412_10084_amd as ps
    t = torch()
    B = o.shape[0]
    do, dd = dev(o), dev(d)
    rgb = t.empty((B, 3), device="cuda")
    aux = t.empty((B, 4), device="cuda")
    dw = t.empty((B, 2), device="cuda")
    opts = ps.RenderOpts(N, 64.0, skip, flags)
    ps.render_forward(fld, opts, do, dd, rgb, aux, dw)
    out = dict(rgb=rgb, aux=aux, depth_wsum=dw)
    if dL is not None:
        g = dict(sdf=t.zeros(fld.sdf.shape, device="cuda"),
                 feat=t.zeros(fld.feat.shape, device="cuda"),
                 probes=t.zeros(fld.probes.shape, device="cuda"),
                 mlp=t.zeros(fld.mlp.shape, device="cuda"))
        ps.render_backward(fld, opts, do, dd, aux, dev(dL.astype(np.float32)), g)
        out["grads"] = g
    t.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "grads"}
    if dL is not None:
        res["grads"] = {k: v.cpu().numpy().astype(np.float64) for k, v in out["grads"].items()}
    return res


def target_rgb(f, o, d, N, skip, flags, seed=1):
    """colours of a torus field with the same colour model, rendered by the oracle"""
    ft = model_field(seed, f.R, f.P, f.n_sh, f.hidden, f.layers, flags, shape="torus")
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N, skip_voxels=skip, flags=flags)
    return tgt["rgb"]


CASES = [  # (n_sh, hidden, layers, flags)
    (16, 32, 2, PAPER),  # the paper's model
    (9, 32, 2, 0),       # two layers of 32 with the workload inputs
    (9, 16, 1, REFLECT),
    (16, 16, 1, FRESNEL),
]


@pytest.mark.parametrize("n_sh,hidden,layers,flags", CASES)
@pytest.mark.parametrize("skip,N", [(0.0, 64), (4.0, 96)])
def test_paper_model_matches_oracle(n_sh, hidden, layers, flags, skip, N):
    f = model_field(0, 64, 16, n_sh, hidden, layers, flags)
    o, d = rays(8, 32, 16)
    of = oracle.field_from(f)
    print(f"paper model case: sh={n_sh} mlp={layers}x{hidden} flags={flags} skip={skip} N={N}",
          flush=True)
    ref = oracle.render_forward(of, o, d, N, skip_voxels=skip, flags=flags)
    keep = ref["margin"] > SKIP_MARGIN
    tgt = target_rgb(f, o, d, N, skip, flags)
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    dL[~keep] = 0.0
    g_ref = oracle.render_backward(of, o, d, dL, N, skip_voxels=skip, flags=flags)
    got = run(gpu_field(f), o, d, N, skip, flags, dL)
    nbad, emax = color_check(got["rgb"], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    assert np.count_nonzero(ref["rgb"].sum(1)) > 300
    k = keep
    np.testing.assert_allclose(got["aux"][k, 3], ref["aux"][k, 3], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(got["depth_wsum"][k], ref["depth_wsum"][k], rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(got["aux"][:, :3], got["rgb"])
    grad_check(got["grads"], g_ref, "fp32")


@pytest.mark.parametrize("abl", [1, 2, 4, 1 | 4])
def test_paper_model_ablations(abl):
    flags = PAPER | abl
    f = model_field(2, 48, 12, 16, 32, 2, flags)
    o, d = rays(8, 32, 16)
    o, d = o[:2000], d[:2000]
    N = 64
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o, d, N, flags=flags)
    rng = np.random.default_rng(5)
    dL = rng.choice([-1.0, 1.0], size=(o.shape[0], 3)) / (3.0 * o.shape[0])
    g_ref = oracle.render_backward(of, o, d, dL, N, flags=flags)
    got = run(gpu_field(f), o, d, N, 0.0, flags, dL)
    nbad, emax = color_check(got["rgb"], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    keys = [k for k in ("sdf", "feat", "probes", "mlp") if np.abs(g_ref[k]).max() > 0]
    if abl & 1:
        assert "feat" not in keys and not got["grads"]["feat"].any()
    grad_check(got["grads"], g_ref, "fp32", keys=tuple(keys))


@pytest.mark.parametrize("mlp_dt,prec,ctol", [(1, "f16", F16_COLOR_ABS), (2, "bf16", BF16_COLOR_ABS)])
def test_paper_model_mixed(mlp_dt, prec, ctol):
    f = model_field(0, 64, 16, 16, 32, 2, PAPER)
    o, d = rays(8, 32, 16)
    N = 64
    of_h = oracle.field_from(f, half=True, mlp_round=prec, flags=PAPER)
    ref = oracle.render_forward(of_h, o, d, N, flags=PAPER)
    tgt = target_rgb(f, o, d, N, 0.0, PAPER)
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    g_ref = oracle.render_backward(of_h, o, d, dL, N, flags=PAPER)
    got = run(gpu_field(f, half=True, mlp_dtype=mlp_dt), o, d, N, 0.0, PAPER, dL)
    err = np.abs(got["rgb"] - ref["rgb"]).max()
    assert err <= ctol, f"colour error {err:.3g} > {ctol}"
    grad_check(got["grads"], g_ref, prec + "_paper")


@pytest.mark.parametrize("n_sh,hidden,layers,flags", [CASES[0], CASES[2]])
def test_paper_model_brick_skipping_changes_nothing(n_sh, hidden, layers, flags):
    """With the SDF's brick bounds the march skips chunks that cannot be active: the
    forward is bit-identical to the march without them, and the gradients match the
    oracle (and the unbounded run up to the FP32 atomics' order)."""
    f = model_field(3, 64, 16, n_sh, hidden, layers, flags)
    o, d = rays(8, 32, 16)
    N, skip = 96, 4.0
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o, d, N, skip_voxels=skip, flags=flags)
    keep = ref["margin"] > SKIP_MARGIN
    rng = np.random.default_rng(4)
    dL = rng.choice([-1.0, 1.0], size=(o.shape[0], 3)) / (3.0 * o.shape[0])
    dL[~keep] = 0.0
    plain = run(gpu_field(f), o, d, N, skip, flags, dL)
    fast = run(gpu_field(f, bounds=True), o, d, N, skip, flags, dL)
    for k in ("rgb", "aux", "depth_wsum"):
        np.testing.assert_array_equal(fast[k], plain[k])
    assert np.count_nonzero(plain["rgb"].sum(1)) > 300
    g_ref = oracle.render_backward(of, o, d, dL, N, skip_voxels=skip, flags=flags)
    grad_check(fast["grads"], g_ref, "fp32")
    grad_check(fast["grads"], plain["grads"], "fp32")


@pytest.mark.parametrize("bounds", [False, True])
def test_paper_model_train256_full_size_sampled(bounds):
    """train256's launch (256^3 / 64^3, 2^18 rays, N = 128, skip 4 voxels) with the
    paper's model (16 SH coefficients), with and without the brick bounds the
    benchmark passes: the oracle evaluates 1500 sampled rays."""
    w = wl.WORKLOADS["train256"]
    f = model_field(0, w.R, w.P, 16, 32, 2, PAPER)
    o, d = rays(w.views, w.W, w.H)
    rng = np.random.default_rng(17)
    idx = np.sort(rng.choice(o.shape[0], 3000, replace=False))
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o[idx], d[idx], w.n_samples, skip_voxels=w.skip_voxels,
                                flags=PAPER)
    keep = ref["margin"] > SKIP_MARGIN
    sel = idx[keep][:1500]
    dL = np.zeros((o.shape[0], 3))
    dL[sel] = rng.choice([-1.0, 1.0], size=(sel.size, 3)) / (3.0 * o.shape[0])
    print(f"paper model train256 launch, bounds={bounds}", flush=True)
    got = run(gpu_field(f, bounds=bounds), o, d, w.n_samples, w.skip_voxels, PAPER, dL)
    nbad, emax = color_check(got["rgb"][idx], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    assert np.count_nonzero(ref["rgb"].sum(1)) > 200
    g_ref = oracle.render_backward(of, o[sel], d[sel], dL[sel], w.n_samples,
                                   skip_voxels=w.skip_voxels, flags=PAPER)
    grad_check(got["grads"], g_ref, "fp32")


def test_paper_model_autograd():
    import paper_2412_10084_amd as ps
    t = torch()
    f = model_field(0, 48, 12, 16, 32, 2, PAPER)
    o, d = rays(4, 32, 16)
    N = 64
    of = oracle.field_from(f)
    rng = np.random.default_rng(9)
    dL = rng.choice([-1.0, 1.0], size=(o.shape[0], 3)) / (3.0 * o.shape[0])
    g_ref = oracle.render_backward(of, o, d, dL, N, flags=PAPER)
    fld = gpu_field(f)
    for k in ("sdf", "feat", "probes", "mlp"):
        getattr(fld, k).requires_grad_(True)
    rgb = ps.render(fld, ps.RenderOpts(N, 64.0, 0.0, PAPER), dev(o), dev(d))
    (rgb * dev(dL.astype(np.float32))).sum().backward()
    t.cuda.synchronize()
    ref = oracle.render_forward(of, o, d, N, flags=PAPER)
    nbad, emax = color_check(rgb.detach().cpu().numpy(), ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    g = {k: getattr(fld, k).grad.cpu().numpy().astype(np.float64)
         for k in ("sdf", "feat", "probes", "mlp")}
    grad_check(g, g_ref, "fp32")
