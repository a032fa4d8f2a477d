"""Pins of the oracle's reverse mode, regularisers, Adam and sphere tracer.

P10  analytic backward vs central finite differences of the FP64 forward;
P11  Adam vs closed forms of Kingma & Ba's bias-corrected moments;
P12  regularisers vs closed forms and finite differences;
P13  sphere tracing vs the analytic ray-sphere intersection.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

RNG = np.random.default_rng(77)


def _bias_slices(n_in, hidden, layers):
    """index ranges of the biases in the packed MLP"""
    out, off = [], 0
    for l in range(layers):
        off += hidden * (n_in if l == 0 else hidden)
        out.append((off, off + hidden))
        off += hidden
    off += 3 * hidden
    out.append((off, off + 3))
    return out


def _tiny_scene(seed=11, R=6, P=3, n_sh=9, model="workload"):
    f = wl.random_field(seed, R, P, n_sh=n_sh, model=model)
    rng = np.random.default_rng(seed + 1)
    sdf = f.sdf.astype(np.float64) + 0.05 * rng.standard_normal(f.sdf.shape)
    mlp = f.mlp.astype(np.float64)
    n_in = wl.N_IN if model == "workload" else wl.PAPER_N_IN
    for lo, hi in _bias_slices(n_in, f.hidden, f.layers):
        mlp[lo:hi] = 0.05 * rng.standard_normal(hi - lo)
    cams = wl.fibonacci_cameras(8, 4, 2)
    o, d = wl.camera_rays(cams, 4, 2)
    sel = rng.choice(o.shape[0], 8, replace=False)
    return (sdf, f.feat.astype(np.float64), f.probes.astype(np.float64), mlp,
            o[sel].astype(np.float64), d[sel].astype(np.float64), f.hidden, f.layers)


def _objective(params, o, d, r, N, tau, skip, flags=0, hidden=16, layers=1):
    of = oracle.make_field(*params, hidden=hidden, layers=layers)
    out = oracle.render_forward(of, o, d, N, tau=tau, skip_voxels=skip, flags=flags)
    return float(np.sum(out["rgb"] * r))


P10_CASES = [
    (0.0, 0, 8.0, "workload", 9),
    (3.0, 0, 8.0, "workload", 9),
    (0.0, oracle.NV_ONE, 5.0, "workload", 9),
    # reflected-vector SH (Sec. 3.1-3.2), alone and with the incidence input ablated
    (0.0, oracle.SH_REFLECT, 8.0, "workload", 9),
    (0.0, oracle.SH_REFLECT | oracle.NV_ONE, 8.0, "workload", 16),
    # the paper's colour model: r, (1 - n.v)^0..5, two hidden layers of 32 (Sec. 4)
    (0.0, oracle.SH_REFLECT | oracle.FRESNEL_PAPER, 8.0, "paper", 16),
    (3.0, oracle.FRESNEL_PAPER, 8.0, "paper", 4),
]


@pytest.mark.parametrize("skip,flags,tau,model,n_sh", P10_CASES)
def test_p10_backward_matches_finite_differences(skip, flags, tau, model, n_sh):
    sdf, feat, probes, mlp, o, d, hidden, layers = _tiny_scene(n_sh=n_sh, model=model)
    N = 8
    r = RNG.standard_normal((o.shape[0], 3))
    params = [sdf, feat, probes, mlp]
    of = oracle.make_field(*params, hidden=hidden, layers=layers)
    fwd = oracle.render_forward(of, o, d, N, tau=tau, skip_voxels=skip, flags=flags)
    assert np.count_nonzero(fwd["n_shaded"]) >= 4
    g = oracle.render_backward(of, o, d, r, N, tau=tau, skip_voxels=skip, flags=flags)
    names = ["sdf", "feat", "probes", "mlp"]
    eps = 1e-6
    worst = 0.0
    for pi, name in enumerate(names):
        flat = params[pi].reshape(-1)
        gflat = g[name].reshape(-1)
        scale = max(np.abs(gflat).max(), 1e-12)
        for q in range(flat.size):
            keep = flat[q]
            flat[q] = keep + eps
            jp = _objective(params, o, d, r, N, tau, skip, flags, hidden, layers)
            flat[q] = keep - eps
            jm = _objective(params, o, d, r, N, tau, skip, flags, hidden, layers)
            flat[q] = keep
            fd = (jp - jm) / (2 * eps)
            err = abs(fd - gflat[q]) / scale
            worst = max(worst, err)
            assert err < 1e-6, (name, q, fd, gflat[q])
    assert worst < 1e-6


def test_p10_gradients_accumulate():
    sdf, feat, probes, mlp, o, d, _, _ = _tiny_scene(seed=3)
    of = oracle.make_field(sdf, feat, probes, mlp)
    r = RNG.standard_normal((o.shape[0], 3))
    g1 = oracle.render_backward(of, o, d, r, 8, tau=8.0)
    g2 = oracle.render_backward(of, o[:4], d[:4], r[:4], 8, tau=8.0)
    g3 = oracle.render_backward(of, o[4:], d[4:], r[4:], 8, tau=8.0)
    for k in g1:
        np.testing.assert_allclose(g1[k], g2[k] + g3[k], atol=1e-14)


# --------------------------------------------------------------------------
# L1 loss gradient
# --------------------------------------------------------------------------
def test_l1_loss():
    rgb = RNG.uniform(size=(10, 3))
    tgt = rgb.copy()
    tgt[:5] += 0.1
    tgt[5:8] -= 0.2
    loss, dL = oracle.l1_loss(rgb, tgt)
    assert loss == pytest.approx((5 * 3 * 0.1 + 3 * 3 * 0.2) / 30)
    assert np.all(dL[:5] == -1 / 30) and np.all(dL[5:8] == 1 / 30) and np.all(dL[8:] == 0)


# --------------------------------------------------------------------------
# P11  Adam (Kingma & Ba, Algorithm 1) closed forms
# --------------------------------------------------------------------------
def test_p11_adam_constant_gradient():
    n = 7
    p0 = RNG.standard_normal(n)
    g = RNG.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    p = p0.copy()
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        p, m, v = oracle.adam(p, g, m, v, t, lr, 0.9, 0.995, eps)
        # bias-corrected moments of a constant gradient are g and g^2 exactly
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=1e-13, atol=1e-15)


def test_p11_adam_geometric_gradient():
    a, r, b1, b2, lr, eps = 0.3, 0.8, 0.9, 0.995, 0.05, 1e-8
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    expect = 1.0
    for t in range(1, 9):
        g = np.array([a * r ** t])
        p, m, v = oracle.adam(p, g, m, v, t, lr, b1, b2, eps)
        # sum_{j<=t} (1-b) b^{t-j} q^j = (1-b) q (q^t - b^t) / (q - b)
        mt = (1 - b1) * a * r * (r ** t - b1 ** t) / (r - b1)
        vt = (1 - b2) * a * a * r * r * (r ** (2 * t) - b2 ** t) / (r * r - b2)
        expect -= lr * (mt / (1 - b1 ** t)) / (math.sqrt(vt / (1 - b2 ** t)) + eps)
        assert m[0] == pytest.approx(mt, rel=1e-12)
        assert v[0] == pytest.approx(vt, rel=1e-12)
        assert p[0] == pytest.approx(expect, rel=1e-12)


# --------------------------------------------------------------------------
# P12  regularisers
# --------------------------------------------------------------------------
def test_p12_eikonal_affine():
    R = 9
    nodes = wl.grid_nodes(R)
    a = np.array([0.6, -0.48, 0.64])  # |a| = 1
    for c in (1.0, 1.7):
        sdf = c * (nodes @ a) + 0.1
        feat = np.zeros((R, R, R, 3))
        probes = np.zeros((3, 3, 3, 9, 4))
        losses, gs, gf, gp = oracle.regularizers(sdf, feat, probes, 0.1, 0.05, 0.2)
        assert losses[0] == pytest.approx(0.1 * (c - 1) ** 2, abs=1e-14)
        assert losses[1] == 0 and losses[2] == 0
        if c == 1.0:
            assert np.abs(gs).max() < 1e-12
        # interior nodes whose 6 neighbours are all interior see zero gradient
        np.testing.assert_allclose(gs[2:-2, 2:-2, 2:-2], 0, atol=1e-12)


def test_p12_tv_closed_forms():
    R, C = 6, 3
    feat = np.full((R, R, R, C), 0.37)
    probes = np.full((4, 4, 4, 9, 4), -1.2)
    sdf = np.zeros((R, R, R))
    losses, gs, gf, gp = oracle.regularizers(sdf, feat, probes, 0.0, 0.05, 0.2)
    assert losses[1] == 0 and losses[2] == 0 and np.all(gf == 0) and np.all(gp == 0)
    # ramp along x: every x-pair differs by a, y/z pairs by 0 -> lambda a^2 / 3
    a = 0.25
    ramp = a * np.arange(R, dtype=np.float64)[None, None, :, None] * np.ones((R, R, R, C))
    losses, gs, gf, gp = oracle.regularizers(sdf, ramp, probes, 0.0, 0.05, 0.2)
    assert losses[1] == pytest.approx(0.05 * a * a / 3, rel=1e-13)
    np.testing.assert_allclose(gf[:, :, 1:-1], 0, atol=1e-15)  # interior of a ramp is stationary


def test_p12_regularizer_gradients_fd():
    R, P = 5, 3
    rng = np.random.default_rng(9)
    sdf = rng.standard_normal((R, R, R)) * 0.3
    feat = rng.standard_normal((R, R, R, 3))
    probes = rng.standard_normal((P, P, P, 4, 4))
    lam = (0.1, 0.05, 0.2)
    _, gs, gf, gp = oracle.regularizers(sdf, feat, probes, *lam)
    eps = 1e-6
    for arr, g, li in ((sdf, gs, 0), (feat, gf, 1), (probes, gp, 2)):
        flat, gfl = arr.reshape(-1), g.reshape(-1)
        for q in range(0, flat.size, 3):
            keep = flat[q]
            flat[q] = keep + eps
            lp = oracle.regularizers(sdf, feat, probes, *lam)[0][li]
            flat[q] = keep - eps
            lm = oracle.regularizers(sdf, feat, probes, *lam)[0][li]
            flat[q] = keep
            assert (lp - lm) / (2 * eps) == pytest.approx(gfl[q], abs=1e-8)


def test_grid_step_composes_regularizers_and_adam():
    R, P = 5, 3
    rng = np.random.default_rng(4)
    params = dict(sdf=rng.standard_normal((R, R, R)), feat=rng.standard_normal((R, R, R, 3)),
                  probes=rng.standard_normal((P, P, P, 9, 4)), mlp=rng.standard_normal(227))
    grads = {k: rng.standard_normal(v.shape) * 1e-3 for k, v in params.items()}
    n = sum(v.size for v in params.values())
    m, v = rng.standard_normal(n) * 1e-3, rng.standard_normal(n) ** 2 * 1e-6
    opts = oracle.StepOpts()
    newp, m2, v2, losses = oracle.grid_step(params, grads, m, v, 3, opts)
    L, gs, gf, gp = oracle.regularizers(params["sdf"], params["feat"], params["probes"],
                                        opts.lambda_eik, opts.lambda_tv_feat, opts.lambda_tv_probe)
    np.testing.assert_allclose(losses, L)
    off = 0
    for k, greg, lr in (("sdf", gs, opts.lr_sdf), ("feat", gf, opts.lr_feat),
                        ("probes", gp, opts.lr_probe), ("mlp", 0.0, opts.lr_mlp)):
        sz = params[k].size
        p1, mm, vv = oracle.adam(params[k].reshape(-1), (grads[k] + greg).reshape(-1),
                                 m[off:off + sz], v[off:off + sz], 3, lr)
        np.testing.assert_allclose(newp[k].reshape(-1), p1, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(m2[off:off + sz], mm, rtol=1e-12, atol=1e-18)
        off += sz


# --------------------------------------------------------------------------
# P13  sphere tracing on the sphere grid vs the analytic intersection
# --------------------------------------------------------------------------
def test_p13_sphere_trace_analytic():
    R, W, H = 64, 48, 24
    f = wl.random_field(0, R, 16)
    of = oracle.field_from(f)
    cams = wl.fibonacci_cameras(2, W, H)
    cam_arr = np.stack([c.as_array() for c in cams]).astype(np.float64)
    out = oracle.sphere_trace(of, cam_arr, W, H, eps=1e-3)
    o, d = wl.camera_rays(cams, W, H)
    o, d = o.astype(np.float64), d.astype(np.float64)
    b = -(o * d).sum(1)
    c = (o * o).sum(1) - 0.25
    disc = b * b - c
    hit_true = disc > 0
    tstar = np.where(hit_true, b - np.sqrt(np.maximum(disc, 0)), -1)
    hit = out["t_hit"] >= 0
    # impact-parameter band around the silhouette where the grid SDF may decide differently
    imp = np.sqrt(np.maximum(c + 0.25 - b * b, 0))
    safe = np.abs(imp - 0.5) > 0.01
    assert np.all(hit[safe] == hit_true[safe])
    both = hit & hit_true
    xh = o + tstar[:, None] * d
    cosang = np.abs((xh / 0.5 * d).sum(1))
    ok = both & (cosang > 0.3)
    err = np.abs(out["t_hit"] - tstar)
    assert np.all(err[ok] <= (1e-3 + 1e-3) / cosang[ok])
    assert np.all(out["rgb"][~hit] == 0)
    assert ok.sum() > 50
