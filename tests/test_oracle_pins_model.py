"""Closed-form pins of the oracle's colour-model inputs and its sample rules.

Each render here is built so that its output has a closed form that does not
come from the oracle's own code:

* The MLP inputs z are decoded from a render.  The SDF is affine, so the normal
  is the constant unit gradient (P2).  Features and probes are constant over
  space, so F_s and F_a are constant along a ray.  The MLP passes three chosen
  slots of z straight to the three outputs (C_c = sigmoid(z[j_c])).  So
  rgb_c = wsum * sigmoid(z[j_c]), and z[j_c] = logit(rgb_c / wsum).  The decoded
  values are compared with:
  - F_s, the constant feature vector;
  - F_a, from the addition theorem.  With probe coefficients b_jk = Y_j(u_k),
    F_a,k = sum_l (2l+1)/(4 pi) P_l(u_k . a), where a is the SH argument.  This
    value depends only on a, not on how the basis is written;
  - the incidence inputs, from c = n . v, with v = -d/|d| and n = grad s/|grad s|
    (Sec. 3.1, Eq. newparametrization; the reflected vector r = 2 (n.v) n - v).
* On an axis ray through an affine SDF, the samples, the skip rule
  |s_i| <= skip * 2/(R-1) and the telescoping NeuS weights are known exactly:
  which samples are shaded, the weight sum, and the margin to the threshold.
  The last sample never has an opacity (Eq. neus needs s_{i+1}).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

# slots of z = [F_s (3), F_a (4), incidence inputs]
FS, FA, INC = (0, 1, 2), (3, 4, 5, 6), 7
OFFSET = 8.0  # every decoded value is above -OFFSET, so the pass-through ReLU is linear


def _legendre(l, x):
    return [1.0, x, 0.5 * (3 * x * x - 1), 0.5 * (5 * x ** 3 - 3 * x)][l]


def _fa_closed_form(us, a, n_sh):
    """F_a,k for probe coefficients b_jk = Y_j(u_k): addition theorem"""
    bands = int(round(math.sqrt(n_sh)))
    return np.array([sum((2 * l + 1) / (4 * math.pi) * _legendre(l, float(np.dot(u, a)))
                          for l in range(bands)) for u in us])


def _passthrough_mlp(n_in, slots):
    """10 -> 16 -> 3 (or n_in -> 16 -> 3): out_c = z[slots[c]]"""
    W1 = np.zeros((16, n_in))
    b1 = np.zeros(16)
    W2 = np.zeros((3, 16))
    b2 = np.full(3, -OFFSET)
    for c, j in enumerate(slots):
        W1[c, j] = 1.0
        b1[c] = OFFSET
        W2[c, c] = 1.0
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2])


def _scene(R, a, s0, fs, us, n_sh, P=3):
    nodes = wl.grid_nodes(R)
    sdf = nodes @ np.asarray(a) + s0
    feat = np.broadcast_to(np.asarray(fs, dtype=np.float64), (R, R, R, 3)).copy()
    coef = np.stack([oracle.sh_basis(n_sh, u) for u in us], axis=-1)  # (n_sh, n_ang)
    probes = np.broadcast_to(coef, (P, P, P, n_sh, len(us))).copy()
    return sdf, feat, probes


def _decode(sdf, feat, probes, n_sh, o, d, flags, slots, n_in):
    of = oracle.make_field(sdf, feat, probes, _passthrough_mlp(n_in, slots), n_sh=n_sh)
    out = oracle.render_forward(of, o, d, 48, tau=16.0, flags=flags)
    wsum = out["depth_wsum"][:, 1]
    assert np.all(wsum > 0.05)
    p = out["rgb"] / wsum[:, None]
    return np.log(p / (1.0 - p)) , out


def _rays():
    # directions with a . d < 0 (the SDF falls along every ray), from outside the cube
    d = np.array([[1.0, 0.3, -0.2], [0.6, 0.7, 0.2], [0.9, -0.4, 0.5], [0.2, 0.1, 1.0]])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = -2.5 * d + np.array([[0.05, -0.1, 0.02]])
    return o, d * np.array([[1.7], [0.6], [2.3], [1.0]])  # rays need not be unit


A = np.array([-0.6, -0.5, -0.62])   # affine SDF gradient, a . d < 0 for the rays above
FSV = (0.11, -0.23, 0.37)
US = [np.array(u) / np.linalg.norm(u) for u in
      ([1.0, 0.2, -0.3], [-0.4, 0.9, 0.1], [0.3, -0.2, 1.0], [-0.7, -0.6, -0.4])]


def _expected(o, d, flags, n_sh):
    """closed-form z of every ray (constant along it)"""
    v = -d / np.linalg.norm(d, axis=1, keepdims=True)
    n = A / np.linalg.norm(A)
    rows = []
    for vv in v:
        c = float(np.dot(n, vv))
        arg = 2 * c * n - vv if flags & oracle.SH_REFLECT else vv
        ci = 1.0 if flags & oracle.NV_ONE else c
        if flags & oracle.FRESNEL_PAPER:
            inc = [(1.0 - ci) ** m for m in range(6)]
        else:
            inc = [ci, ci ** 2, ci ** 4]
        rows.append(np.concatenate([FSV, _fa_closed_form(US, arg, n_sh), inc]))
    return np.array(rows)


@pytest.mark.parametrize("flags,n_sh", [
    (0, 9), (0, 16), (oracle.NV_ONE, 9), (oracle.SH_REFLECT, 9), (oracle.SH_REFLECT, 16),
    (oracle.FRESNEL_PAPER, 9), (oracle.SH_REFLECT | oracle.FRESNEL_PAPER, 16),
    (oracle.SH_REFLECT | oracle.FRESNEL_PAPER | oracle.NV_ONE, 4)])
def test_mlp_inputs_decoded_from_render(flags, n_sh):
    """Every slot of z, decoded from rendered colours, equals its closed form.  A
    flipped view direction, a swapped F_s / F_a slot, c^3 in place of c^4, a wrong
    power (1 - c)^m or a wrong reflection changes some decoded slot by far more
    than the tolerance."""
    sdf, feat, probes = _scene(9, A, 0.05, FSV, US, n_sh)
    o, d = _rays()
    n_in = 3 + 4 + (6 if flags & oracle.FRESNEL_PAPER else 3)
    exp = _expected(o, d, flags, n_sh)
    for start in range(0, n_in, 3):
        slots = [min(j, n_in - 1) for j in range(start, start + 3)]
        got, _ = _decode(sdf, feat, probes, n_sh, o, d, flags, slots, n_in)
        np.testing.assert_allclose(got, exp[:, slots], atol=1e-9, err_msg=f"slots {slots}")


def test_incidence_inputs_distinguish_the_plausible_mistakes():
    """The chosen rays keep c away from the values where the mistakes coincide."""
    o, d = _rays()
    v = -d / np.linalg.norm(d, axis=1, keepdims=True)
    c = v @ (A / np.linalg.norm(A))
    assert np.all(c > 0.2) and np.all(c < 0.95)
    assert np.min(np.abs(c ** 4 - c ** 3)) > 1e-2          # c^4 vs c^3
    assert np.min(np.abs(c - (-c))) > 0.4                   # v vs -v on the c slot
    fa_v = np.array([_fa_closed_form(US, vv, 9) for vv in v])
    fa_mv = np.array([_fa_closed_form(US, -vv, 9) for vv in v])
    assert np.min(np.max(np.abs(fa_v - fa_mv), axis=1)) > 1e-2  # v vs -v on F_a


def test_reflection_is_the_view_at_normal_incidence():
    """r = v when the ray meets the surface head on, so REFLECT changes nothing."""
    R = 9
    nodes = wl.grid_nodes(R)
    sdf = 0.1 - nodes[..., 0]            # n = (-1, 0, 0) = v for a +x ray
    f = wl.random_field(4, R, 3, n_sh=16)
    of = oracle.make_field(sdf, f.feat, f.probes, f.mlp, n_sh=16)
    o = np.array([[-3.0, 0.13, -0.21], [-3.0, -0.4, 0.33]])
    d = np.array([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    a = oracle.render_forward(of, o, d, 40, tau=16.0)
    b = oracle.render_forward(of, o, d, 40, tau=16.0, flags=oracle.SH_REFLECT)
    assert np.all(a["n_shaded"] > 0)
    np.testing.assert_allclose(b["rgb"], a["rgb"], atol=1e-15)


def test_reflection_changes_oblique_colour():
    sdf, feat, probes = _scene(9, A, 0.05, FSV, US, 9)
    o, d = _rays()
    f = wl.random_field(5, 9, 3)
    of = oracle.make_field(sdf, feat, probes, f.mlp)
    a = oracle.render_forward(of, o, d, 48, tau=16.0)
    b = oracle.render_forward(of, o, d, 48, tau=16.0, flags=oracle.SH_REFLECT)
    assert np.max(np.abs(a["rgb"] - b["rgb"])) > 1e-4


# --------------------------------------------------------------------------
# skip rule, last sample and weights on an axis ray through an affine SDF
# --------------------------------------------------------------------------
def _axis_case(R, N, skip, x0, tau=16.0):
    """s(x) = x0 - x (falls along +x); one +x ray through the cube."""
    nodes = wl.grid_nodes(R)
    sdf = x0 - nodes[..., 0]
    f = wl.random_field(2, R, 3)
    of = oracle.make_field(sdf, f.feat, f.probes, f.mlp)
    o = np.array([[-3.0, 0.17, -0.08]])
    d = np.array([[1.0, 0.0, 0.0]])
    out = oracle.render_forward(of, o, d, N, tau=tau, skip_voxels=skip)
    # closed form: t in [2, 4], x_i = -1 + (i + 1/2) 2/N, s_i = x0 - x_i, h = 2/(R-1)
    X = -1.0 + (np.arange(N) + 0.5) * 2.0 / N
    s = x0 - X
    thr = skip * 2.0 / (R - 1)
    active = (np.abs(s) <= thr) if skip > 0 else np.ones(N, bool)
    active[N - 1] = False
    return out, s, thr, active


def _log_phi(x):
    return min(x, 0.0) - math.log1p(math.exp(-abs(x)))


@pytest.mark.parametrize("R,N,skip,x0", [
    (17, 64, 2.0, 0.013),     # h = 2/(R-1) = 0.125 and 2/R = 0.1176 shade 16 vs 15 samples
    (17, 64, 2.0, 0.93),      # the band reaches the last sample, which never shades
    (33, 1500, 3.0, -0.2),    # N above any fixed per-ray buffer of 1024
    (9, 40, 0.0, 0.87),       # no skip rule: every sample but the last
])
def test_skip_rule_last_sample_and_weights_closed_form(R, N, skip, x0):
    tau = 16.0
    out, s, thr, active = _axis_case(R, N, skip, x0, tau)
    idx = np.flatnonzero(active)
    assert out["n_shaded"][0] == idx.size
    # the active samples are consecutive; telescoping (Eq. neus): T after them is
    # Phi(s_{last+1}) / Phi(s_first)
    assert np.all(np.diff(idx) == 1)
    i0, i1 = idx[0], idx[-1]
    wsum = 1.0 - math.exp(_log_phi(tau * s[i1 + 1]) - _log_phi(tau * s[i0]))
    assert out["depth_wsum"][0, 1] == pytest.approx(wsum, rel=1e-12)
    assert out["aux"][0, 3] == pytest.approx(math.log1p(-wsum), rel=1e-10)
    if skip > 0:
        margin = np.min(np.abs(np.abs(s[:-1]) - thr))
        assert out["margin"][0] == pytest.approx(margin, abs=1e-12)


def test_threshold_in_voxels_of_two_over_r_minus_one():
    """The first case above separates h = 2/(R-1) from h = 2/R."""
    R, N, x0 = 17, 64, 0.013
    X = -1.0 + (np.arange(N - 1) + 0.5) * 2.0 / N
    n_h = np.count_nonzero(np.abs(x0 - X) <= 2.0 * 2.0 / (R - 1))
    n_r = np.count_nonzero(np.abs(x0 - X) <= 2.0 * 2.0 / R)
    assert n_h != n_r
    out, *_ = _axis_case(R, N, 2.0, x0)
    assert out["n_shaded"][0] == n_h


def test_sample_count_limits():
    f = wl.random_field(0, 8, 3)
    of = oracle.field_from(f)
    o, d = np.array([[0.0, 0.0, -3.0]]), np.array([[0.0, 0.0, 1.0]])
    for bad in (1, oracle.MAX_N + 1):
        with pytest.raises(oracle.OracleError):
            oracle.render_forward(of, o, d, bad)
        with pytest.raises(oracle.OracleError):
            oracle.render_backward(of, o, d, np.ones((1, 3)), bad)


def test_mlp_size_mismatch_is_rejected():
    f = wl.random_field(0, 8, 3)
    of = oracle.field_from(f)
    o, d = np.array([[0.0, 0.0, -3.0]]), np.array([[0.0, 0.0, 1.0]])
    with pytest.raises(oracle.OracleError):
        oracle.render_forward(of, o, d, 16, flags=oracle.FRESNEL_PAPER)  # needs 13 inputs


# --------------------------------------------------------------------------
# SH gradient (used by the reflected argument's reverse mode) and the 2-layer MLP
# --------------------------------------------------------------------------
def test_sh_grad_matches_finite_differences():
    rng = np.random.default_rng(9)
    for v in rng.standard_normal((12, 3)):
        J = oracle.sh_grad(16, v)
        eps = 1e-6
        for a in range(3):
            vp, vm = v.copy(), v.copy()
            vp[a] += eps
            vm[a] -= eps
            fd = (oracle.sh_basis(16, vp) - oracle.sh_basis(16, vm)) / (2 * eps)
            np.testing.assert_allclose(J[:, a], fd, atol=1e-8)


def test_two_layer_mlp_against_matmul_chain():
    rng = np.random.default_rng(10)
    n_in, H = 13, 32
    mlp = wl.xavier_uniform_mlp(rng, n_in, H, 3, 2).astype(np.float64)
    mlp += 0.01 * rng.standard_normal(mlp.size)
    W1 = mlp[:H * n_in].reshape(H, n_in)
    b1 = mlp[H * n_in:H * n_in + H]
    o2 = H * n_in + H
    W2 = mlp[o2:o2 + H * H].reshape(H, H)
    b2 = mlp[o2 + H * H:o2 + H * H + H]
    o3 = o2 + H * H + H
    Wo = mlp[o3:o3 + 3 * H].reshape(3, H)
    bo = mlp[o3 + 3 * H:]
    assert bo.size == 3
    for z in rng.standard_normal((10, n_in)):
        h1 = np.maximum(W1 @ z + b1, 0.0)
        h2 = np.maximum(W2 @ h1 + b2, 0.0)
        ref = 1.0 / (1.0 + np.exp(-(Wo @ h2 + bo)))
        C, out, hid, pre = oracle.mlp_forward(mlp, z, hidden=H, layers=2)
        np.testing.assert_allclose(C, ref, rtol=1e-14)
        np.testing.assert_allclose(hid[1], h2, atol=1e-14)
