"""Pins of the oracle's real-time path (supplementary "Performance Analysis":
per-voxel shading, then volume rendering of the colour field): the shaded band,
the node-to-camera view direction through a closed-form cosine on a plane, and
the volume render against closed forms built from the forward render's weight
sum and depth (constant and affine colour fields, reproduced exactly by trilinear
interpolation)."""
import numpy as np

import oracle
import workloads as wl


def plane_field(R, P=4, z0=0.1):
    a = np.linspace(-1.0, 1.0, R)
    z = np.meshgrid(a, a, a, indexing="ij")[0]
    f = wl.random_field(0, R, P)
    f.sdf = (z - z0).astype(np.float32)  # s = z - z0: the FD normal is +e_z exactly
    return f


def pixel_rays(cam, W, H, ids):
    px, py = ids % W, ids // W
    dc = np.stack([(px + 0.5 - cam[14]) / cam[12], (py + 0.5 - cam[15]) / cam[13],
                   np.ones(ids.size)], axis=1)
    Rm = np.asarray(cam[:12], np.float64).reshape(3, 4)
    d = dc @ Rm[:, :3].T
    o = np.broadcast_to(Rm[:, 3], d.shape).copy()
    return o, d / np.linalg.norm(d, axis=1, keepdims=True)


def test_voxel_shade_band_and_view_direction():
    R = 17
    f = plane_field(R)
    # MLP: hidden unit 0 = relu(c) (c = n.v, input slot 7), output 0 = that unit, the
    # other outputs 0, so C_0 = sigmoid(max(c, 0)) and C_1 = C_2 = 1/2
    m = np.zeros(227)
    m[0 * 10 + 7] = 1.0     # W1[0][7]
    m[176 + 0 * 16 + 0] = 1.0  # W2[0][0]
    f.mlp = m
    of = oracle.field_from(f)
    cam = wl.fibonacci_cameras(3, 8, 8)[1].as_array()
    centre = np.array([cam[3], cam[7], cam[11]])
    band = 0.3
    col = oracle.voxel_shade(of, cam, band)
    s = f.sdf.astype(np.float64)
    shaded = np.abs(s) <= band
    assert np.all(col[~shaded] == 0.0)
    a = np.linspace(-1.0, 1.0, R)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    pts = np.stack([x, y, z], axis=-1)
    v = centre - pts
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    c = v[..., 2]  # n = +e_z
    expect0 = 1.0 / (1.0 + np.exp(-np.maximum(c, 0.0)))
    np.testing.assert_allclose(col[shaded][:, 0], expect0[shaded], rtol=1e-13)
    np.testing.assert_allclose(col[shaded][:, 1:], 0.5, rtol=1e-15)


def test_volume_render_constant_and_affine_colour_fields():
    R = 33
    f = wl.random_field(3, R, 8)
    of = oracle.field_from(f)
    cam = wl.fibonacci_cameras(4, 48, 24)[2].as_array()
    W, H, N = 48, 24, 64
    ids = np.arange(W * H, dtype=np.int64)
    o, d = pixel_rays(cam, W, H, ids)
    fw = oracle.render_forward(of, o, d, N, skip_voxels=4.0)
    wsum, depth = fw["depth_wsum"][:, 1], fw["depth_wsum"][:, 0]
    assert np.count_nonzero(wsum) > 200
    # constant colour k: the render is k times the weight sum
    k = np.array([0.2, 0.5, 0.9])
    col = np.broadcast_to(k, (R, R, R, 3)).copy()
    rgb, _ = oracle.volume_render(of, col, cam, W, H, N, skip_voxels=4.0)
    np.testing.assert_allclose(rgb, wsum[:, None] * k[None, :], rtol=1e-12, atol=1e-15)
    # affine colour A x + b: trilinear reproduces it, and sum_i w_i x_i =
    # o wsum + d (depth - wsum dt / 2), with dt the sample spacing of the ray
    A = np.array([[0.3, -0.2, 0.1], [0.0, 0.4, -0.3], [0.25, 0.05, 0.2]])
    b = np.array([0.5, 0.4, 0.3])
    a1 = np.linspace(-1.0, 1.0, R)
    z, y, x = np.meshgrid(a1, a1, a1, indexing="ij")
    pts = np.stack([x, y, z], axis=-1)
    col = pts @ A.T + b
    rgb, _ = oracle.volume_render(of, col, cam, W, H, N, skip_voxels=4.0)
    dt = np.zeros(ids.size)
    for q in range(ids.size):
        hit, tn, tf = oracle.ray_box(o[q], d[q])
        dt[q] = (tf - tn) / N if hit else 0.0
    sx = o * wsum[:, None] + d * (depth - wsum * dt / 2)[:, None]
    np.testing.assert_allclose(rgb, sx @ A.T + wsum[:, None] * b[None, :], rtol=1e-10,
                               atol=1e-13)
