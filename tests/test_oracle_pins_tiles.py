"""Pins of the oracle's sparse tiles with tri-plane spatial features (Sec. 3.1
F_s = F_x (x) F_y (x) F_z on coarse tiles; Sec. 4: 16^3-voxel tiles of 3 x 16 x 16
x n_s coefficients): exact reproduction of affine planes between the texel
centres and their clamped values at tile faces, empty tiles, equivalence with a
dense field on constant planes, the plane smoothness closed forms, and the
reverse mode against finite differences."""
import numpy as np
import pytest

import oracle
import workloads as wl

TILE = 16


def affine_planes(slots, coef):
    """planes whose texel (u, v) of plane a, channel c holds a0 + a1 (u + 1/2) + a2 (v + 1/2)"""
    pl = np.zeros((slots, 3, TILE, TILE, 3))
    uu = np.arange(TILE)[None, :] + 0.5
    vv = np.arange(TILE)[:, None] + 0.5
    for a in range(3):
        for c in range(3):
            a0, a1, a2 = coef[a][c]
            pl[:, a, :, :, c] = a0 + a1 * uu + a2 * vv
    return pl


def test_triplane_reproduces_affine_planes_and_clamps_at_faces():
    f = wl.tiled_field(0, 2)
    rng = np.random.default_rng(1)
    coef = rng.uniform(0.2, 1.0, size=(3, 3, 3)) * np.array([1.0, 0.05, 0.05])
    f.tiles.planes = affine_planes(f.tiles.planes.shape[0], coef)
    of = oracle.field_from(f)
    h = 2.0 / (f.R - 1)
    axes = [(1, 2), (0, 2), (0, 1)]
    for _ in range(200):
        x = rng.uniform(-1, 1, size=3)
        got, slot = oracle.triplane(of, x)
        u = (x + 1) / h
        t = np.minimum(np.floor(np.minimum(u, f.R - 2)), f.R - 2) // TILE
        loc = u - TILE * t
        if slot < 0:
            assert np.all(got == 0)
            continue
        # texel coordinates clamped to [1/2, 15 1/2]: constant beyond the outer centres
        lc = np.clip(loc, 0.5, 15.5)
        expect = np.ones(3)
        for a in range(3):
            ua, va = axes[a]
            for c in range(3):
                a0, a1, a2 = coef[a][c]
                expect[c] *= a0 + a1 * lc[ua] + a2 * lc[va]
        np.testing.assert_allclose(got, expect, rtol=1e-13)


def test_empty_tiles_are_inactive():
    f = wl.tiled_field(0, 2)
    f.tiles.index[:] = -1
    of = oracle.field_from(f)
    o, d = wl.camera_rays(wl.fibonacci_cameras(4, 16, 8), 16, 8)
    ref = oracle.render_forward(of, o, d, 48)
    assert not ref["rgb"].any() and not ref["n_shaded"].any()


def test_constant_planes_match_a_dense_field():
    f = wl.tiled_field(2, 2, margin_voxels=100.0)  # every tile allocated
    assert (f.tiles.index >= 0).all()
    k = np.array([[0.7, -1.1, 0.4], [1.3, 0.9, -0.6], [0.8, 0.5, 1.2]])  # plane a, channel c
    f.tiles.planes[:] = k[None, :, None, None, :]
    k = k.astype(np.float32).astype(np.float64)  # the values the planes hold
    of = oracle.field_from(f)
    dense = wl.Field(R=f.R, P=f.P, n_sh=f.n_sh, sdf=f.sdf,
                     feat=np.broadcast_to(k.prod(axis=0), (f.R, f.R, f.R, 3)).astype(np.float64),
                     probes=f.probes, mlp=f.mlp)
    od = oracle.field_from(dense)
    o, d = wl.camera_rays(wl.fibonacci_cameras(4, 16, 8), 16, 8)
    a = oracle.render_forward(of, o, d, 48)
    b = oracle.render_forward(od, o, d, 48)
    np.testing.assert_allclose(a["rgb"], b["rgb"], rtol=1e-12, atol=1e-15)
    assert np.count_nonzero(a["rgb"].sum(1)) > 20


def test_plane_smoothness_closed_forms():
    pl = np.zeros((2, 3, TILE, TILE, 3)) + 0.3
    L, g = oracle.plane_smooth(pl, 1.0)
    assert L == 0.0 and not g.any()
    # a ramp along u in every plane: 16 rows x 15 unit differences per plane and
    # channel along u, none along v: L = lambda / 2
    pl = np.broadcast_to(np.arange(TILE, dtype=np.float64)[None, None, None, :, None],
                         (2, 3, TILE, TILE, 3)).copy()
    L, _ = oracle.plane_smooth(pl, 0.8)
    np.testing.assert_allclose(L, 0.4, rtol=1e-14)
    rng = np.random.default_rng(3)
    pl = rng.standard_normal((1, 3, TILE, TILE, 3))
    L, g = oracle.plane_smooth(pl, 0.5)
    for q in rng.choice(pl.size, 20, replace=False):
        e = np.zeros(pl.size)
        e[q] = 1e-6
        e = e.reshape(pl.shape)
        fd = (oracle.plane_smooth(pl + e, 0.5)[0] - oracle.plane_smooth(pl - e, 0.5)[0]) / 2e-6
        assert abs(fd - g.reshape(-1)[q]) < 1e-8


@pytest.mark.parametrize("flags", [0, 8 | 16])
def test_tiled_backward_by_finite_differences(flags):
    """dL/d(planes, sdf, probes, mlp) of L = sum dL . rgb on one tile (R = 17)."""
    model = "paper" if flags else "workload"
    f = wl.tiled_field(4, 1, n_sh=9, margin_voxels=100.0, model=model)
    rng = np.random.default_rng(5)
    f.sdf = (f.sdf + 0.01 * rng.standard_normal(f.sdf.shape)).astype(np.float64)
    o, d = wl.camera_rays(wl.fibonacci_cameras(3, 6, 4), 6, 4)
    N = 16
    dL = rng.standard_normal((o.shape[0], 3))

    def loss(of):
        return np.sum(dL * oracle.render_forward(of, o, d, N, tau=16.0, flags=flags)["rgb"])

    of = oracle.field_from(f)
    g = oracle.render_backward(of, o, d, dL, N, tau=16.0, flags=flags)
    assert np.abs(g["feat"]).max() > 0
    eps = 1e-6
    for key, arr in (("feat", "tile_feat"), ("sdf", "sdf"), ("probes", "probes")):
        base = getattr(of, arr)
        picks = rng.choice(base.size, 12, replace=False)
        for q in picks:
            flat = base.reshape(-1)
            old = flat[q]
            flat[q] = old + eps
            lp = loss(of)
            flat[q] = old - eps
            lm = loss(of)
            flat[q] = old
            fd = (lp - lm) / (2 * eps)
            an = g[key].reshape(-1)[q]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (key, q, fd, an)
