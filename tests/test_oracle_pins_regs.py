"""Pins of the oracle's smoothed SDF and remaining regularisers (Sec. 3.3, Eqs.
smooth_sdf, eikonal_reg, smmoth_normals, photo_loss) to facts other than the code:
exactness of the Gaussian on constants and affine fields, its separability and
its limits, the adjoint identity of G and G^T, closed forms of the normal term,
finite differences of every gradient, and reduction to the plain grid step."""
import numpy as np
import pytest

import oracle


def nodes(R):
    a = np.linspace(-1.0, 1.0, R)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return x, y, z


def test_gauss_reproduces_constants_and_interior_affine_fields():
    R = 11
    x, y, z = nodes(R)
    c = np.full((R, R, R), 0.7)
    np.testing.assert_allclose(oracle.smooth(c), c, rtol=0, atol=1e-15)
    f = 0.3 * x - 1.2 * y + 0.5 * z + 0.1
    s = oracle.smooth(f)
    inner = (slice(2, -2),) * 3  # the kernel is symmetric: affine fields are kept
    np.testing.assert_allclose(s[inner], f[inner], rtol=0, atol=1e-14)
    # at the first node the replicated edge reads x_0 for the two outer taps:
    # value = f_0 + slope h (w_1 + 2 w_2) along that axis
    w = oracle.gauss5(1.0)
    h = 2.0 / (R - 1)
    g = 0.3 * x
    sg = oracle.smooth(g)
    np.testing.assert_allclose(sg[5, 5, 0], g[5, 5, 0] + 0.3 * h * (w[3] + 2 * w[4]), atol=1e-14)


def test_gauss_is_separable_normalised_and_has_the_right_limits():
    R = 9
    d = np.zeros((R, R, R))
    d[4, 4, 4] = 1.0
    r = oracle.smooth(d)  # response to a unit impulse = the kernel itself
    assert abs(r.sum() - 1.0) < 1e-14
    wc = r[4, 4, 4] ** (1.0 / 3.0)  # the centre tap
    k1 = r[4, 4, 2:7] / (wc * wc)   # one axis of the kernel
    outer = np.einsum("i,j,k->ijk", k1, k1, k1)
    np.testing.assert_allclose(r[2:7, 2:7, 2:7], outer, rtol=1e-12)
    # a wide Gaussian tends to the 5-tap box filter, a narrow one to the identity
    np.testing.assert_allclose(oracle.gauss5(1e6), np.full(5, 0.2), atol=1e-9)
    np.testing.assert_allclose(oracle.gauss5(1e-3), [0, 0, 1, 0, 0], atol=1e-12)
    # second moment of the kernel: x^2 becomes x^2 + h^2 sum k^2 w_k in the interior
    x, _, _ = nodes(R)
    w = oracle.gauss5(1.0)
    var = sum(k * k * w[k + 2] for k in range(-2, 3))
    h = 2.0 / (R - 1)
    s = oracle.smooth(x ** 2)
    np.testing.assert_allclose(s[4, 4, 2:7], (x ** 2)[4, 4, 2:7] + var * h * h, atol=1e-14)


def test_smooth_transpose_is_the_adjoint():
    rng = np.random.default_rng(1)
    for R in (5, 8):
        a = rng.standard_normal((R, R, R))
        b = rng.standard_normal((R, R, R))
        lhs = np.sum(oracle.smooth(a) * b)
        rhs = np.sum(a * oracle.smooth_T(b))
        assert abs(lhs - rhs) <= 1e-12 * np.abs(a).sum()


def test_normal_term_zero_on_planes_and_closed_form_on_a_crease():
    R = 9
    x, y, z = nodes(R)
    L, _, _ = oracle.sdf_regs(0.6 * x + 0.8 * z - 0.1, smooth=False, lambda_sdf=0,
                              lambda_eik=0, lambda_normal=1.0)
    assert L[2] < 1e-28
    # s = |z| on an odd grid: normals -e_z below the middle plane, 0 on it (central
    # difference 0), +e_z above; only the z-pairs touching the middle plane differ
    # by 1, so L = lambda * 2 (R-2)^2 / (3 (R-2)^2 (R-3))
    L, _, _ = oracle.sdf_regs(np.abs(z), smooth=False, lambda_sdf=0, lambda_eik=0,
                              lambda_normal=1.0)
    np.testing.assert_allclose(L[2], 2.0 / (3.0 * (R - 3)), rtol=1e-14)


def test_sdf_term_zero_without_smoothing_and_on_constants():
    rng = np.random.default_rng(2)
    f = rng.standard_normal((8, 8, 8))
    L, g, s = oracle.sdf_regs(f, smooth=False, lambda_sdf=1.0, lambda_eik=0, lambda_normal=0)
    assert L[0] == 0.0 and not g.any()
    np.testing.assert_array_equal(s, f)
    L, g, _ = oracle.sdf_regs(np.full((8, 8, 8), -0.3), smooth=True, lambda_sdf=1.0,
                              lambda_eik=0, lambda_normal=0)
    assert L[0] < 1e-30 and np.abs(g).max() < 1e-15


def test_eikonal_matches_the_plain_regulariser_without_smoothing():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((7, 7, 7)) * 0.3
    L, g, _ = oracle.sdf_regs(f, smooth=False, lambda_sdf=0, lambda_eik=0.1, lambda_normal=0)
    L0, gs, _, _ = oracle.regularizers(f, np.zeros((7, 7, 7, 3)), np.zeros((2, 2, 2, 9, 4)), 0.1,
                                       0.0, 0.0)
    np.testing.assert_allclose(L[1], L0[0], rtol=1e-14)
    np.testing.assert_allclose(g, gs, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("smooth", [False, True])
def test_regulariser_gradients_by_finite_differences(smooth):
    """dJ/dshat for J = L_sdf + L_Eik + L_normal + sum g_s s(shat), central differences."""
    R = 7
    rng = np.random.default_rng(4)
    x, y, z = nodes(R)
    f = np.sqrt(x ** 2 + y ** 2 + z ** 2) - 0.5 + 0.05 * rng.standard_normal((R, R, R))
    g_s = 0.01 * rng.standard_normal((R, R, R))
    kw = dict(smooth=smooth, lambda_sdf=0.3, lambda_eik=0.1, lambda_normal=0.05)

    def J(a):
        L, _, s = oracle.sdf_regs(a, **kw)
        return L.sum() + np.sum(g_s * s)

    _, g, _ = oracle.sdf_regs(f, g_s=g_s, **kw)
    eps = 1e-6
    for q in rng.choice(R ** 3, 40, replace=False):
        e = np.zeros(R ** 3)
        e[q] = eps
        e = e.reshape(f.shape)
        fd = (J(f + e) - J(f - e)) / (2 * eps)
        assert abs(fd - g.reshape(-1)[q]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, q


def test_weighting_scales_each_node_by_its_distance_factor():
    R = 7
    rng = np.random.default_rng(5)
    f = rng.standard_normal((R, R, R)) * 0.4
    g_s = rng.standard_normal((R, R, R)) * 1e-3
    kw = dict(smooth=False, lambda_sdf=0.0, lambda_eik=0.1, lambda_normal=0.05)
    _, g0, _ = oracle.sdf_regs(f, g_s=np.zeros_like(f), **kw)
    _, gw, _ = oracle.sdf_regs(f, g_s=g_s, weighted=True, **kw)
    np.testing.assert_allclose(gw, g0 / (1.0 + 5.0 * np.abs(f)) + g_s, rtol=1e-12, atol=1e-18)
    # with smoothing the weights sit on the gradient with respect to s, before G^T
    kw["smooth"] = True
    kw["lambda_sdf"] = 0.2
    _, g0, s = oracle.sdf_regs(f, g_s=np.zeros_like(f), weighted=False, **kw)
    _, gw, _ = oracle.sdf_regs(f, g_s=np.zeros_like(f), weighted=True, **kw)
    assert not np.allclose(g0, gw)
    assert np.all(np.isfinite(gw))


def test_step_ext_reduces_to_the_plain_step_and_returns_the_smoothed_field():
    rng = np.random.default_rng(6)
    R, P = 6, 3
    p = dict(sdf=rng.standard_normal((R, R, R)) * 0.3, feat=rng.standard_normal((R, R, R, 3)),
             probes=rng.standard_normal((P, P, P, 9, 4)), mlp=rng.standard_normal(227))
    g = {k: rng.standard_normal(v.shape) * 1e-3 for k, v in p.items()}
    n = sum(v.size for v in p.values())
    m, v = rng.standard_normal(n) * 1e-3, rng.random(n) * 1e-6
    base = oracle.StepOpts()
    plain = oracle.grid_step(p, g, m, v, 3, base)
    ext = oracle.grid_step_ext(p, g, m, v, 3, oracle.StepExt(base, lambda_sdf=0.0,
                                                             lambda_normal=0.0, smooth=False))
    for k in p:
        np.testing.assert_allclose(ext[0][k], plain[0][k], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(ext[1], plain[1], rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(ext[2], plain[2], rtol=1e-14, atol=1e-22)
    np.testing.assert_allclose(ext[3][[1, 3, 4]], plain[3], rtol=1e-14)
    ext = oracle.grid_step_ext(p, g, m, v, 3, oracle.StepExt(base))
    np.testing.assert_allclose(ext[4], oracle.smooth(ext[0]["sdf"]), rtol=0, atol=1e-15)


def test_l2rel_loss_relations():
    rng = np.random.default_rng(7)
    c = rng.random((50, 3))
    t = rng.random((50, 3))
    L, dL = oracle.l2rel_loss(c, t, lam=40.0, eps=1e-3, n_images=4)
    # symmetric in (c, c_gt); linear in lambda / n_images
    L2, dL2 = oracle.l2rel_loss(t, c, lam=40.0, eps=1e-3, n_images=4)
    np.testing.assert_allclose(L2, L, rtol=1e-14)
    np.testing.assert_allclose(dL2, -dL, rtol=1e-14)
    L3, dL3 = oracle.l2rel_loss(c, t, lam=80.0, eps=1e-3, n_images=2)
    np.testing.assert_allclose(L3, 4 * L, rtol=1e-14)
    np.testing.assert_allclose(dL3, 4 * dL, rtol=1e-14)
    # a huge eps makes the weight a constant 1/eps: the plain L2 loss and its gradient
    E = 1e9
    L4, dL4 = oracle.l2rel_loss(c, t, lam=1.0, eps=E)
    np.testing.assert_allclose(L4 * E, np.sum((c - t) ** 2), rtol=1e-8)
    np.testing.assert_allclose(dL4 * E, 2 * (c - t), rtol=1e-8)
