"""GPU parity, continued: full-size workloads on sampled outputs, the FP16 /
BF16 mixed-precision paths, the optimiser step and the sphere tracer."""
import json

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_common import (BF16_COLOR_ABS, BF16_GRAD_REL, F16_COLOR_ABS, F16_GRAD_REL,
                        FP32_COLOR_ABS, FP32_COLOR_REL, FP32_GRAD_REL, FP32_MLP_GRAD_REL,
                        SKIP_MARGIN, color_check, dev, device_field, gpu_backward, gpu_forward,
                        grad_check, grad_errors, norm_rel, rays, scene, torch)

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------------------
# full size, FP32 training workload: 256^3 / 64^3, 2^18 rays, N = 128, skip 4 voxels.
# The GPU runs the whole batch (the benchmark's launch); the oracle evaluates a
# sample of rays, and the backward carries loss gradient on that sample only.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("bounds", [True, False])
def test_train256_full_size_sampled(bounds):
    import paper_2412_10084_amd as ps
    w = wl.WORKLOADS["train256"]
    f = scene(0, w.R, w.P)
    o, d = rays(w.views, w.W, w.H)
    assert o.shape[0] == 1 << 18
    fld = device_field(f)
    if bounds:  # empty-space skipping, as the benchmark runs it
        fld.bounds = ps.sdf_bounds(fld.sdf)
    got = gpu_forward(fld, o, d, w.n_samples, skip=w.skip_voxels)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(o.shape[0], 3000, replace=False))
    of = oracle.field_from(f)
    ref = oracle.render_forward(of, o[idx], d[idx], w.n_samples, skip_voxels=w.skip_voxels)
    keep = ref["margin"] > SKIP_MARGIN
    nbad, emax = color_check(got["rgb"][idx], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} bad, max err {emax:.3g}"
    assert np.count_nonzero(ref["rgb"].sum(1)) > 200
    # backward with the loss gradient on the sampled rays only
    sel = idx[keep][:1500]
    dL = np.zeros((o.shape[0], 3))
    dL[sel] = rng.choice([-1.0, 1.0], size=(sel.size, 3)) / (3.0 * o.shape[0])
    do, dd, _, aux = got["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, w.n_samples, skip=w.skip_voxels)
    g_ref = oracle.render_backward(of, o[sel], d[sel], dL[sel], w.n_samples,
                                   skip_voxels=w.skip_voxels)
    grad_check(g, g_ref, "fp32")


# ---------------------------------------------------------------------------
# mixed precision: FP16 features and probes, MLP on FP16 / BF16 MFMA
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mlp_dt,ctol,gtol", [(1, F16_COLOR_ABS, F16_GRAD_REL),
                                              (2, BF16_COLOR_ABS, BF16_GRAD_REL)])
def test_mixed_forward_backward_small(mlp_dt, ctol, gtol):
    f = scene(0, 64, 16)
    ft = scene(1, 64, 16, shape="torus")
    o, d = rays(8, 32, 16)
    N = 64
    of_h = oracle.field_from(f, half=True, mlp_round=("f16", "bf16")[mlp_dt - 1])  # the values the GPU reads
    ref = oracle.render_forward(of_h, o, d, N)
    fld = device_field(f, feat_half=True, mlp_dtype=mlp_dt)
    got = gpu_forward(fld, o, d, N)
    err = np.abs(got["rgb"] - ref["rgb"]).max()
    assert err <= ctol, f"colour error {err:.3g} > {ctol}"
    # total error against the FP32 parameters is reported, and stays small
    ref32 = oracle.render_forward(oracle.field_from(f), o, d, N)
    assert np.abs(got["rgb"] - ref32["rgb"]).max() <= 2 * ctol
    tgt = oracle.render_forward(oracle.field_from(ft), o, d, N)["rgb"]
    _, dL = oracle.l1_loss(ref["rgb"], tgt)
    g_ref = oracle.render_backward(of_h, o, d, dL, N)
    do, dd, _, aux = got["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, N)
    grad_check(g, g_ref, ("f16", "bf16")[mlp_dt - 1])


@pytest.mark.parametrize("prec", ["fp32", "f16", "bf16"])
def test_mixed512_full_size_sampled(prec):
    """The benchmark's mixed512 launch (512^3 / 128^3, 2^20 rays, N = 64, no skip),
    forward with a tape and backward from it, in FP32 and with FP16 storage and the
    MLP on FP16 / BF16 MFMA.  The oracle evaluates 600 sampled rays, fed the same
    FP16-rounded values the GPU reads; the loss gradient sits on those rays only."""
    import paper_2412_10084_amd as ps
    w = wl.WORKLOADS["mixed512"]
    f = scene(0, w.R, w.P)
    o, d = rays(w.views, w.W, w.H)
    B = o.shape[0]
    assert B == 1 << 20
    half = prec != "fp32"
    mdt = {"fp32": 0, "f16": 1, "bf16": 2}[prec]
    print(f"mixed512 case: {prec}", flush=True)
    fld = device_field(f, feat_half=half, mlp_dtype=mdt)
    tape = ps.backward_workspace(B, w.P, B * (w.n_samples - 1))
    got = gpu_forward(fld, o, d, w.n_samples, tape=tape)
    rng = np.random.default_rng(8)
    idx = np.sort(rng.choice(B, 600, replace=False))
    of = oracle.field_from(f, half=half, mlp_round=prec if half else "")
    ref = oracle.render_forward(of, o[idx], d[idx], w.n_samples)
    if half:
        ctol = F16_COLOR_ABS if prec == "f16" else BF16_COLOR_ABS
        nbad, emax = color_check(got["rgb"][idx], ref["rgb"], 0.0, ctol)
    else:
        nbad, emax = color_check(got["rgb"][idx], ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    dL = np.zeros((B, 3))
    dL[idx] = rng.choice([-1.0, 1.0], size=(idx.size, 3)) / (3.0 * B)
    do, dd, _, aux = got["dev"]
    g = gpu_backward(fld, do, dd, aux, dL, w.n_samples, workspace=tape, from_tape=True)
    g_ref = oracle.render_backward(of, o[idx], d[idx], dL[idx], w.n_samples)
    # the per-result error table against FP64: arithmetic error (oracle fed the values
    # the GPU reads) and, for the mixed paths, total error (oracle fed the FP32 values)
    table = {"prec": prec, "rays": int(idx.size),
             "colour_max_abs": float(np.abs(got["rgb"][idx] - ref["rgb"]).max()),
             "grads": grad_errors(g, g_ref)}
    if half:
        of32 = oracle.field_from(f)
        ref32 = oracle.render_forward(of32, o[idx], d[idx], w.n_samples)
        g32 = oracle.render_backward(of32, o[idx], d[idx], dL[idx], w.n_samples)
        table["total_colour_max_abs"] = float(np.abs(got["rgb"][idx] - ref32["rgb"]).max())
        table["total_grads"] = grad_errors(g, g32)
    print("ERRTABLE " + json.dumps(table), flush=True)
    grad_check(g, g_ref, prec)


# ---------------------------------------------------------------------------
# optimiser step: regulariser gradients + Adam, against the oracle
# ---------------------------------------------------------------------------
def _step_inputs(R=24, P=8, seed=21):
    rng = np.random.default_rng(seed)
    p = dict(sdf=(rng.standard_normal((R, R, R)) * 0.3).astype(np.float32),
             feat=(rng.standard_normal((R, R, R, 3)) * 0.1).astype(np.float32),
             probes=(rng.standard_normal((P, P, P, 9, 4)) * 0.1).astype(np.float32),
             mlp=(rng.standard_normal(227) * 0.3).astype(np.float32))
    g = {k: (rng.standard_normal(v.shape) * 1e-3).astype(np.float32) for k, v in p.items()}
    m = {k: (rng.standard_normal(v.shape) * 1e-3).astype(np.float32) for k, v in p.items()}
    v = {k: ((rng.standard_normal(v.shape) * 1e-3) ** 2).astype(np.float32) for k, v in p.items()}
    return p, g, m, v


# R = 70: several x tiles and z chunks of the tiled SDF pass, ragged at the ends.
# R = 344, P = 128: the launch geometry of the 512^3 / 128^3 step (feature rows of
# 3R/4 > 256 float4 span two blocks, probe rows of 128 x 36 floats five).
@pytest.mark.parametrize("step,R,P", [(1, 24, 8), (7, 24, 8), (3, 70, 8), (2, 344, 128)])
def test_grid_step_matches_oracle(step, R, P):
    import paper_2412_10084_amd as ps
    t = torch()
    print(f"grid step case: R={R} P={P} step={step}", flush=True)
    p, g, m, v = _step_inputs(R=R, P=P)
    opts = ps.StepOpts()
    keys = ("sdf", "feat", "probes", "mlp")
    dp = {k: dev(p[k]) for k in keys}
    dout = {k: t.empty_like(dp[k]) for k in keys}
    dg = {k: dev(g[k]) for k in keys}
    dm_ = {k: dev(m[k]) for k in keys}
    dv_ = {k: dev(v[k]) for k in keys}
    half = {k: t.empty(dp[k].shape, dtype=t.float16, device="cuda") for k in ("sdf", "feat", "probes")}
    losses = t.empty(3, device="cuda")
    ps.grid_step(dp, dout, dg, dm_, dv_, step, opts, half_out=half, losses=losses)
    t.cuda.synchronize()
    o_opts = oracle.StepOpts(**{k: getattr(opts, k) for k in vars(oracle.StepOpts())})
    mcat = np.concatenate([m[k].reshape(-1) for k in keys])
    vcat = np.concatenate([v[k].reshape(-1) for k in keys])
    newp, m2, v2, L = oracle.grid_step(p, g, mcat, vcat, step, o_opts)
    lr = dict(sdf=opts.lr_sdf, feat=opts.lr_feat, probes=opts.lr_probe, mlp=opts.lr_mlp)
    _, rs, rf, rp = oracle.regularizers(p["sdf"], p["feat"], p["probes"], opts.lambda_eik,
                                        opts.lambda_tv_feat, opts.lambda_tv_probe)
    reg = dict(sdf=rs, feat=rf, probes=rp, mlp=np.zeros(227))
    b1, b2 = opts.beta1, opts.beta2
    bc1, bc2 = 1 - b1 ** step, 1 - b2 ** step
    off = 0
    for k in keys:
        n = p[k].size
        # moments: relative to the magnitudes of the terms that form them (they can
        # cancel); the FP32 regulariser gradient carries a few ulps of its own scale
        gk, rk = g[k].astype(np.float64).reshape(-1), reg[k].reshape(-1)
        G = gk + rk
        eG = 1e-6 * (np.abs(gk) + np.abs(rk)) + 1e-6 * np.abs(rk).max()
        m0, v0 = m[k].astype(np.float64).reshape(-1), v[k].astype(np.float64).reshape(-1)
        dm = 1e-6 * (b1 * np.abs(m0) + (1 - b1) * np.abs(G)) + (1 - b1) * eG + 1e-30
        dv = 1e-6 * (b2 * v0 + (1 - b2) * G * G) + (1 - b2) * 2 * np.abs(G) * eG + 1e-30
        gm, gv = dm_[k].cpu().numpy().reshape(-1), dv_[k].cpu().numpy().reshape(-1)
        em = np.abs(gm - m2[off:off + n]) / dm
        ev = np.abs(gv - v2[off:off + n]) / dv
        assert em.max() <= 1.0 and ev.max() <= 1.0, f"{k}: moments {em.max():.3g} {ev.max():.3g}"
        # parameters: one FP32 ulp of the result, a few ulps of the update, and the
        # moment bounds carried through m_hat / (sqrt(v_hat) + eps)
        got = (dp[k] if k == "mlp" else dout[k]).cpu().numpy().astype(np.float64).reshape(-1)
        ref = newp[k].reshape(-1)
        upd = p[k].astype(np.float64).reshape(-1) - ref
        sv = np.sqrt(v2[off:off + n] / bc2)
        mh = np.abs(m2[off:off + n]) / bc1
        bound = (2.0 ** -23 * np.abs(ref) + 2e-6 * np.abs(upd)
                 + lr[k] * (dm / bc1) / (sv + opts.eps)
                 + lr[k] * mh * (dv / bc2) / (2 * np.maximum(sv, 1e-30) * (sv + opts.eps) ** 2)
                 + 1e-30)
        ex = np.abs(got - ref) / bound
        assert ex.max() <= 1.0, f"{k}: worst |d|/bound {ex.max():.3g} at {ex.argmax()}"
        off += n
        assert float(dg[k].abs().max()) == 0.0, f"{k} gradient not zeroed"
        if k != "mlp":
            h = half[k].cpu().numpy().astype(np.float64).reshape(-1)
            # FP16 copy of the FP32 result: one FP16 rounding (half ulp, 2^-11 relative;
            # 2^-25 absolute in the subnormal range) plus the FP32 error above
            eh = np.abs(h - ref) / (np.abs(ref) * 2.0 ** -11 + 2.0 ** -25 + bound)
            assert eh.max() <= 1.0, f"{k}: fp16 copy {eh.max():.3g}"
    # the losses are FP32 sums of up to 1.2e8 non-negative terms: per-thread sums, block
    # trees and one atomic add per block, so the error grows with the count of block
    # partials added in sequence (about 1e-4 of the sum at R = 344)
    np.testing.assert_allclose(losses.cpu().numpy(), L, rtol=1e-4 if R < 100 else 1e-3)


# ---------------------------------------------------------------------------
# sphere tracing
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("half,mlp_dt", [(False, 0), (True, 0), (True, 1)])
def test_sphere_trace(half, mlp_dt):
    import paper_2412_10084_amd as ps
    t = torch()
    f = scene(0, 64, 16)
    V, W, H = 2, 64, 32
    cams = np.stack([c.as_array() for c in wl.fibonacci_cameras(V, W, H)]).astype(np.float32)
    fld = device_field(f, feat_half=half, sdf_half=half, mlp_dtype=mlp_dt)
    out = t.empty((V, H, W, 3), device="cuda")
    ps.sphere_trace(fld, dev(cams), W, H, out, eps=1e-3, max_steps=256)
    t.cuda.synchronize()
    of = oracle.field_from(f, half=half, half_sdf=half)
    ref = oracle.sphere_trace(of, cams, W, H, eps=1e-3, max_steps=256)
    got = out.cpu().numpy().reshape(-1, 3)
    _trace_check(got, ref, mlp_dt)


def _trace_check(got, ref, mlp_dt):
    # the trace runs in FP64 on both sides, so only a step whose s lands within
    # 1e-6 of eps (or t of t_f) may decide differently
    keep = (ref["margin"] > 1e-6) & (ref["steps"] < 250)
    assert keep.mean() > 0.99, f"only {keep.mean():.4f} of rays away from thresholds"
    hit = ref["t_hit"] >= 0
    assert hit.sum() > 300
    if mlp_dt:
        nbad, emax = color_check(got, ref["rgb"], 0.0, F16_COLOR_ABS, keep)
    else:
        nbad, emax = color_check(got, ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    assert np.all(got[keep & ~hit] == 0)


def test_trace512_full_size_sampled():
    """The benchmark's inference launch: FP16 grids 512^3 / 128^3, 16 views at
    1920x1080 in one launch; the oracle traces 2000 sampled pixels."""
    import paper_2412_10084_amd as ps
    t = torch()
    w = wl.WORKLOADS["trace512"]
    f = scene(0, w.R, w.P)
    cams = np.stack([c.as_array() for c in wl.fibonacci_cameras(w.views, w.W, w.H)])
    cams = cams.astype(np.float32)
    fld = device_field(f, feat_half=True, sdf_half=True)
    out = t.empty((w.views, w.H, w.W, 3), device="cuda")
    print("trace512 launch: 16 x 1920 x 1080", flush=True)
    ps.sphere_trace(fld, dev(cams), w.W, w.H, out, eps=1e-3, max_steps=256)
    t.cuda.synchronize()
    rng = np.random.default_rng(31)
    n_pix = w.views * w.W * w.H
    ids = np.sort(rng.choice(n_pix, 2000, replace=False))
    of = oracle.field_from(f, half=True, half_sdf=True)
    ref = oracle.sphere_trace(of, cams, w.W, w.H, pixel_ids=ids, eps=1e-3, max_steps=256)
    got = out.reshape(-1, 3)[t.from_numpy(ids).cuda()].cpu().numpy()
    keep = (ref["margin"] > 1e-6) & (ref["steps"] < 250)
    assert keep.mean() > 0.99
    nbad, emax = color_check(got, ref["rgb"], FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"
    assert (ref["t_hit"] >= 0).sum() > 100
