"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Each test checks an oracle building block against something independent of the
oracle's own code: exact reproduction of closed forms, invariants, special
cases that reduce to textbook results, brute force and finite differences.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

RNG = np.random.default_rng(1234)


def _affine_grid(R, a, b, C=1):
    nodes = wl.grid_nodes(R)  # [k, j, i, 3]
    vals = nodes @ np.asarray(a, dtype=np.float64).T + b  # (..., C)
    return vals if C > 1 else vals[..., 0]


# --------------------------------------------------------------------------
# P1  trilinear: exact on affine fields (the operator is exact on multilinear
#     functions), node values reproduced at nodes.  Sec. 3.2 (trilinear probes)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("R", [2, 5, 17])
def test_p1_trilinear_affine_exact(R):
    A = RNG.standard_normal((3, 3))
    b = RNG.standard_normal(3)
    grid = _affine_grid(R, A, b, C=3)
    xs = RNG.uniform(-1, 1, size=(200, 3))
    xs[:10] = np.sign(xs[:10])  # domain corners
    xs[10:20, 0] = 1.0           # faces
    xs[20:30, 1] = -1.0
    for x in xs:
        np.testing.assert_allclose(oracle.trilinear(grid, x), A @ x + b, atol=1e-12)


def test_p1_trilinear_nodes_and_bilinear_term():
    R = 7
    g = RNG.standard_normal((R, R, R))
    nodes = wl.grid_nodes(R)
    for (k, j, i) in [(0, 0, 0), (6, 6, 6), (3, 2, 5), (0, 6, 1)]:
        assert oracle.trilinear(g, nodes[k, j, i]) == pytest.approx(g[k, j, i], abs=1e-13)
    # x*y*z is trilinear, so it is reproduced exactly too
    xyz = nodes[..., 0] * nodes[..., 1] * nodes[..., 2]
    for x in RNG.uniform(-1, 1, size=(50, 3)):
        assert oracle.trilinear(xyz, x)[0] == pytest.approx(x[0] * x[1] * x[2], abs=1e-13)


# --------------------------------------------------------------------------
# P2  normal: an affine SDF gives n = a/|a| exactly everywhere (including
#     clamped stencils at the faces); the exact sphere SDF gives the radial
#     normal with O(h^2) error.  Sec. 3.3 (n = grad s / |grad s|)
# --------------------------------------------------------------------------
def test_p2_affine_normal_exact():
    a = np.array([0.3, -0.8, 0.52])
    s = _affine_grid(9, a[None, :], 0.1)
    xs = RNG.uniform(-1, 1, size=(100, 3))
    xs[:8] = np.sign(RNG.uniform(-1, 1, size=(8, 3)))
    for x in xs:
        np.testing.assert_allclose(oracle.sdf_gradient(s, x), a, atol=1e-12)


def test_p2_sphere_normal_second_order():
    errs = []
    for R in (33, 65):
        s = wl.sphere_sdf_nodes(R).astype(np.float64)
        # use exact node values (not float32-rounded) for a clean convergence rate
        n = wl.grid_nodes(R)
        s = np.linalg.norm(n, axis=-1) - 0.5
        e = 0.0
        for x in RNG.uniform(-1, 1, size=(60, 3)):
            x = 0.5 * x / np.linalg.norm(x)
            g = oracle.sdf_gradient(s, x)
            e = max(e, np.linalg.norm(g / np.linalg.norm(g) - x / np.linalg.norm(x)))
        errs.append(e)
    h = 2.0 / 64
    assert errs[1] < 2.0 * h * h * 4  # O(h^2) bound
    assert errs[0] / errs[1] > 2.5    # second order convergence (ratio ~4)


# --------------------------------------------------------------------------
# P3  SH: orthonormality by exact quadrature, addition theorem, ordering and
#     sign convention.  Sec. 3.2 Eq. spherical_harmonics (l^2 coefficients)
# --------------------------------------------------------------------------
def _sphere_quadrature(nt=24, nphi=48):
    x, w = np.polynomial.legendre.leggauss(nt)  # cos(theta)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return dirs, wts


def test_p3_sh_orthonormal():
    dirs, wts = _sphere_quadrature()
    Y = np.stack([oracle.sh_basis(16, d) for d in dirs])  # (Q, 16)
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_p3_sh_addition_theorem():
    for v in RNG.standard_normal((20, 3)):
        v /= np.linalg.norm(v)
        Y = oracle.sh_basis(16, v)
        for l, (lo, hi) in enumerate([(0, 1), (1, 4), (4, 9), (9, 16)]):
            assert np.sum(Y[lo:hi] ** 2) == pytest.approx((2 * l + 1) / (4 * np.pi), rel=1e-13)


def test_p3_sh_order_and_sign():
    # band 1 is (y, z, x) with a positive constant; band 2 (2,0) peaks on +z
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(oracle.sh_basis(4, [1, 0, 0]), [0.5 / math.sqrt(math.pi), 0, 0, c1],
                               atol=1e-15)
    np.testing.assert_allclose(oracle.sh_basis(4, [0, 1, 0])[1:], [c1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(oracle.sh_basis(4, [0, 0, 1])[1:], [0, c1, 0], atol=1e-15)
    Y = oracle.sh_basis(9, [0, 0, 1])
    assert Y[6] == pytest.approx(0.5 * math.sqrt(5 / math.pi))
    s = 1 / math.sqrt(2)
    Y = oracle.sh_basis(9, [s, s, 0])
    assert Y[4] == pytest.approx(0.5 * math.sqrt(15 / math.pi) * 0.5)  # xy term
    # a sub-basis is a prefix of the larger one
    v = np.array([0.2, -0.4, 0.7]) / np.linalg.norm([0.2, -0.4, 0.7])
    np.testing.assert_array_equal(oracle.sh_basis(9, v), oracle.sh_basis(16, v)[:9])
    with pytest.raises(ValueError):
        oracle.sh_basis(5, v)


# --------------------------------------------------------------------------
# P4  Eq. sh_eval1 == Eq. sh_eval2: evaluating each corner probe's SH and
#     interpolating equals interpolating the coefficients and evaluating once.
# P5  only the constant coefficient non-zero => F_a independent of the view;
#     with zero cosine columns the colour is view independent too.
# --------------------------------------------------------------------------
def _small_field(R=6, P=3, n_sh=9, seed=5, sdf_noise=0.05):
    f = wl.random_field(seed, R, P, n_sh=n_sh)
    rng = np.random.default_rng(seed + 100)
    sdf = f.sdf.astype(np.float64) + sdf_noise * rng.standard_normal(f.sdf.shape)
    return oracle.make_field(sdf, f.feat, f.probes, f.mlp, n_sh=n_sh)


def test_p4_interpolate_then_evaluate():
    of = _small_field(R=7, P=4, n_sh=16)
    for _ in range(20):
        x = RNG.uniform(-1, 1, 3)
        v = RNG.standard_normal(3)
        v /= np.linalg.norm(v)
        Y = oracle.sh_basis(16, v)
        per_probe = np.einsum("kjisa,s->kjia", of.probes, Y)  # SH evaluated at every probe
        fa1 = oracle.trilinear(per_probe, x)                  # then interpolated (sh_eval1)
        _, z = oracle.shade(of, x, v)                          # oracle: sh_eval2
        np.testing.assert_allclose(z[3:7], fa1, atol=1e-13)


def test_p5_view_invariance():
    of = _small_field(R=6, P=3, n_sh=9)
    probes = of.probes.copy()
    probes[..., 1:, :] = 0.0
    mlp = of.mlp.copy()
    W1 = mlp[:160].reshape(16, 10)
    W1[:, 7:] = 0.0
    mlp[:160] = W1.reshape(-1)
    of2 = oracle.make_field(of.sdf, of.feat, probes, mlp)
    x = np.array([0.11, -0.23, 0.31])
    ref_c, ref_z = None, None
    for v in RNG.standard_normal((10, 3)):
        v /= np.linalg.norm(v)
        c, z = oracle.shade(of2, x, v)
        if ref_c is None:
            ref_c, ref_z = c, z
        np.testing.assert_allclose(z[3:7], ref_z[3:7], atol=1e-15)
        np.testing.assert_allclose(c, ref_c, atol=1e-15)
    # and F_a = b_0 * Y_0 exactly
    b0 = oracle.trilinear(probes[..., 0, :], x)
    np.testing.assert_allclose(ref_z[3:7], b0 * 0.5 / math.sqrt(math.pi), atol=1e-15)


# --------------------------------------------------------------------------
# P6  MLP: numpy matmul chain on the packed layout; closed-form special cases
# --------------------------------------------------------------------------
def test_p6_mlp():
    mlp = wl.xavier_uniform_mlp(np.random.default_rng(3)).astype(np.float64)
    mlp[160:176] = RNG.standard_normal(16) * 0.1
    mlp[224:227] = RNG.standard_normal(3) * 0.1
    W1, b1 = mlp[:160].reshape(16, 10), mlp[160:176]
    W2, b2 = mlp[176:224].reshape(3, 16), mlp[224:227]
    for z in RNG.standard_normal((20, 10)):
        C, out, hid, pre = oracle.mlp_forward(mlp, z)
        ref = 1 / (1 + np.exp(-(W2 @ np.maximum(W1 @ z + b1, 0) + b2)))
        np.testing.assert_allclose(C, ref, atol=1e-15)
    # zero weights: C = sigmoid(b2)
    m0 = np.zeros(227)
    m0[224:227] = [0.0, 1.0, -2.0]
    C, *_ = oracle.mlp_forward(m0, RNG.standard_normal(10))
    np.testing.assert_allclose(C, 1 / (1 + np.exp(-np.array([0.0, 1.0, -2.0]))), atol=1e-15)
    # single path z_3 -> hidden 5 -> output 1
    m1 = np.zeros(227)
    m1[5 * 10 + 3] = 2.0
    m1[176 + 16 + 5] = 1.5
    z = np.zeros(10)
    z[3] = 0.7
    C, *_ = oracle.mlp_forward(m1, z)
    assert C[1] == pytest.approx(1 / (1 + math.exp(-2.1)))
    z[3] = -0.7  # ReLU cuts it
    C, *_ = oracle.mlp_forward(m1, z)
    assert C[1] == pytest.approx(0.5)


# --------------------------------------------------------------------------
# P7  alpha / T: on a decreasing SDF the NeuS weights telescope,
#     T_i = Phi_i/Phi_0 and w_i = (Phi_i - Phi_{i+1})/Phi_0; an increasing SDF
#     is transparent; weights are >= 0 and sum with T_final to 1.  Eq. neus
# --------------------------------------------------------------------------
def _phi(x):
    return 1.0 / (1.0 + np.exp(-x))


def test_p7_telescoping():
    tau = 64.0
    s = np.sort(RNG.uniform(-0.1, 0.1, 40))[::-1].copy()
    alpha, T, w, logT = oracle.composite(s, np.ones(40), tau)
    Phi = _phi(tau * s)
    np.testing.assert_allclose(T, Phi / Phi[0], rtol=1e-12)
    np.testing.assert_allclose(w[:-1], (Phi[:-1] - Phi[1:]) / Phi[0], rtol=1e-10, atol=1e-300)
    assert w[-1] == 0.0
    assert math.exp(logT) == pytest.approx(Phi[-1] / Phi[0], rel=1e-12)


def test_p7_increasing_is_transparent_and_partition_of_unity():
    s = np.sort(RNG.uniform(-0.3, 0.3, 30))
    alpha, T, w, logT = oracle.composite(s, np.ones(30), 64.0)
    assert np.all(alpha == 0) and logT == 0.0
    for _ in range(20):
        s = np.cumsum(RNG.standard_normal(50) * 0.03)
        act = RNG.uniform(size=50) < 0.8
        alpha, T, w, logT = oracle.composite(s, act, 64.0)
        assert np.all(w >= 0) and np.all(alpha[~act] == 0)
        assert w.sum() + math.exp(logT) == pytest.approx(1.0, abs=1e-13)


def test_p7_extreme_sdf_no_nan():
    s = np.array([-50.0, -60.0, 50.0, 60.0, -80.0])
    alpha, T, w, logT = oracle.composite(s, np.ones(5), 64.0)
    assert np.all(np.isfinite(alpha)) and np.all(np.isfinite(T)) and np.isfinite(logT)


# --------------------------------------------------------------------------
# P8  depth of the surface: exact sphere SDF along a central ray from a camera
#     at distance 3: weights follow the closed form and the weighted depth lands
#     on the analytic hit t* = 2.5; on the 64^3 grid also near t*.
# --------------------------------------------------------------------------
def test_p8_central_ray_analytic_depth():
    N, tau = 64, 64.0
    tn, tf = 2.0, 4.0
    dt = (tf - tn) / N
    t = tn + (np.arange(N) + 0.5) * dt
    s = np.abs(t - 3.0) - 0.5
    alpha, T, w, logT = oracle.composite(s, np.ones(N), tau)
    Phi = _phi(tau * s)
    dec = t[1:] <= 3.0  # pairs with a decreasing SDF
    # the closed form subtracts two values near 1: its own error is ~1e-16 absolute
    np.testing.assert_allclose(w[:-1][dec], (Phi[:-1] - Phi[1:])[dec] / Phi[0], rtol=1e-10,
                               atol=1e-15)
    depth = np.sum(w * (t + dt / 2)) / np.sum(w)
    assert abs(depth - 2.5) < 1e-3


def test_p8_grid_depth_sphere():
    R = 64
    f = wl.random_field(0, R, 16)
    of = oracle.field_from(f)
    o = np.array([[3.0, 0.0, 0.0], [0.0, 3.0, 0.0], [2.0, 2.0, 1.0]])
    tgt = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.1], [0.1, -0.05, 0.0]])
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = oracle.render_forward(of, o, d, n_samples=128, tau=64.0)
    depth = r["depth_wsum"][:, 0] / r["depth_wsum"][:, 1]
    b = -(o * d).sum(1)
    c = (o * o).sum(1) - 0.25
    tstar = b - np.sqrt(b * b - c)
    np.testing.assert_allclose(depth, tstar, atol=2.5e-3)
    assert np.all(r["depth_wsum"][:, 1] > 0.99)


# --------------------------------------------------------------------------
# P9  N = 2: one interval, rgb = alpha_0 C_0 with alpha_0 from the ratio form of
#     Eq. neus (the oracle uses the log form).
# --------------------------------------------------------------------------
def test_p9_two_samples_brute_force():
    of = _small_field(R=8, P=3)
    tau = 10.0
    o = np.array([[2.5, 0.3, -0.2], [0.1, -2.8, 0.4], [0.3, 0.2, 3.0]])
    d = -o + RNG.uniform(-0.3, 0.3, size=(3, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = oracle.render_forward(of, o, d, n_samples=2, tau=tau)
    for b in range(3):
        hit, tn, tf = oracle.ray_box(o[b], d[b])
        assert hit
        dt = (tf - tn) / 2
        x0 = np.clip(o[b] + (tn + 0.5 * dt) * d[b], -1, 1)
        x1 = np.clip(o[b] + (tn + 1.5 * dt) * d[b], -1, 1)
        s0, s1 = oracle.trilinear(of.sdf, x0)[0], oracle.trilinear(of.sdf, x1)[0]
        a0 = max((_phi(tau * s0) - _phi(tau * s1)) / _phi(tau * s0), 0.0)
        C0, _ = oracle.shade(of, x0, -d[b])
        np.testing.assert_allclose(r["rgb"][b], a0 * C0, atol=1e-14)


# --------------------------------------------------------------------------
# ray / box interval: closed-form cases
# --------------------------------------------------------------------------
def test_ray_box_cases():
    hit, tn, tf = oracle.ray_box([3, 0, 0], [-1, 0, 0])
    assert hit and tn == pytest.approx(2.0) and tf == pytest.approx(4.0)
    hit, tn, tf = oracle.ray_box([0, 0, 0], [0, 0, 1])
    assert hit and tn == 0.0 and tf == pytest.approx(1.0)
    hit, *_ = oracle.ray_box([3, 3, 0], [-1, 0, 0])  # parallel, outside
    assert not hit
    hit, *_ = oracle.ray_box([3, 0, 0], [1, 0, 0])   # pointing away
    assert not hit
    d = np.array([-1.0, -1.0, -1.0]) / math.sqrt(3)
    hit, tn, tf = oracle.ray_box([2, 2, 2], d)
    assert hit and tn == pytest.approx(math.sqrt(3)) and tf == pytest.approx(3 * math.sqrt(3))


def test_miss_gives_zero():
    of = _small_field()
    r = oracle.render_forward(of, np.array([[3.0, 3.0, 0.0]]), np.array([[-1.0, 0.0, 0.0]]), 16)
    assert np.all(r["rgb"] == 0) and np.all(r["aux"] == 0)
