"""GPU parity of the real-time path (supplementary "Performance Analysis":
per-voxel shading, then volume rendering of the colour field) against the FP64
oracle: the band list, the voxel colours (FP32 and FP16 colour grids, FP32 and
FP16 / MFMA colour model), the volume render (fed the GPU's own colour grid, and
the whole pipeline), and the rt512 launch (512^3 / 128^3 FP16 grids, one
1920x1163 view) on sampled pixels."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_common import (F16_COLOR_ABS, FP32_COLOR_ABS, FP32_COLOR_REL, SKIP_MARGIN, color_check,
                        dev, device_field, scene, torch)

pytestmark = pytest.mark.gpu


def gpu_colours(fld, R, cam, band, colour_dt, flags=0):
    import paper_2412_10084_amd as ps
    t = torch()
    lst = t.empty(R ** 3, dtype=t.int32, device="cuda")
    cnt = t.zeros(1, dtype=t.int32, device="cuda")
    ps.voxel_list(fld.sdf, band, lst, cnt)
    dt = t.float32 if colour_dt == 0 else t.float16
    col = t.zeros((R, R, R, 4), dtype=dt, device="cuda")
    ps.voxel_shade(fld, dev(cam), lst, cnt, col, flags=flags)
    t.cuda.synchronize()
    return col, int(cnt.item()), lst


def test_voxel_list_is_the_band():
    t = torch()
    f = scene(0, 64, 16)
    fld = device_field(f)
    band = float(np.float32(6.0 * 2.0 / 63))
    cam = wl.fibonacci_cameras(4, 64, 32)[0].as_array()
    _, n, lst = gpu_colours(fld, 64, cam, band, 0)
    inband = np.flatnonzero(np.abs(f.sdf.reshape(-1)) <= np.float32(band))
    assert n == inband.size
    np.testing.assert_array_equal(np.sort(lst[:n].cpu().numpy()), inband)
    del t


@pytest.mark.parametrize("half", [False, True])
@pytest.mark.parametrize("offset", [0, 1])
def test_voxel_list_ragged_unaligned_and_capped(half, offset):
    """R = 37 (a ragged last block), the grid at a 16-byte boundary or one element past
    it (the scalar path), and a capacity below the band's size."""
    import paper_2412_10084_amd as ps
    t = torch()
    R = 37
    rng = np.random.default_rng(7 + offset)
    s = rng.uniform(-1, 1, R ** 3).astype(np.float16 if half else np.float32)
    buf = t.from_numpy(np.concatenate([np.zeros(offset, s.dtype), s])).cuda()
    sdf = buf[offset:].view(R, R, R)
    band = 0.25
    inband = np.flatnonzero(np.abs(s.astype(np.float32)) <= np.float32(band))
    for cap in (R ** 3, inband.size // 3):
        lst = t.full((max(cap, 1),), -1, dtype=t.int32, device="cuda")
        cnt = t.zeros(1, dtype=t.int32, device="cuda")
        ps.voxel_list(sdf, band, lst[:cap], cnt)
        t.cuda.synchronize()
        got = lst.cpu().numpy()
        assert int(cnt.item()) == inband.size
        k = min(cap, inband.size)
        assert np.all(got[k:] == -1)
        if cap >= inband.size:
            np.testing.assert_array_equal(np.sort(got[:k]), inband)
        else:
            part = got[:k]
            assert np.unique(part).size == k and np.isin(part, inband).all()


@pytest.mark.parametrize("colour_dt,half,mlp_dt", [(0, False, 0), (1, False, 0), (1, True, 1)])
def test_voxel_shade_matches_oracle(colour_dt, half, mlp_dt):
    R, P = 64, 16
    f = scene(0, R, P)
    fld = device_field(f, feat_half=half, mlp_dtype=mlp_dt)
    band = float(np.float32(6.0 * 2.0 / (R - 1)))
    cam = wl.fibonacci_cameras(4, 64, 32)[1].as_array().astype(np.float32)
    col, n, _ = gpu_colours(fld, R, cam, band, colour_dt)
    of = oracle.field_from(f, half=half, mlp_round="f16" if mlp_dt else "")
    ref = oracle.voxel_shade(of, cam, band)
    got = col.float().cpu().numpy()[..., :3].reshape(-1, 3)
    ref = ref.reshape(-1, 3)
    shaded = np.abs(f.sdf.reshape(-1)) <= np.float32(band)
    assert n == shaded.sum() > 1000
    assert np.all(got[~shaded] == 0.0)
    rel = FP32_COLOR_REL + (2.0 ** -11 if colour_dt else 0.0)  # one FP16 rounding
    if mlp_dt:
        nbad, emax = color_check(got[shaded], ref[shaded], 0.0, F16_COLOR_ABS)
    else:
        nbad, emax = color_check(got[shaded], ref[shaded], rel, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} colours off, max err {emax:.3g}"


@pytest.mark.parametrize("colour_dt", [0, 1])
def test_volume_render_matches_oracle(colour_dt):
    import paper_2412_10084_amd as ps
    t = torch()
    R, P, W, H, N, skip = 64, 16, 96, 48, 96, 4.0
    f = scene(0, R, P)
    fld = device_field(f)
    fld.bounds = ps.sdf_bounds(fld.sdf)
    band = float(np.float32(wl.RT_BAND_VOXELS * 2.0 / (R - 1)))
    cam = wl.fibonacci_cameras(4, W, H)[2].as_array().astype(np.float32)
    col, _, _ = gpu_colours(fld, R, cam, band, colour_dt)
    out = t.empty((H, W, 3), device="cuda")
    ps.volume_render(fld, ps.RenderOpts(N, 64.0, skip, 0), col, dev(cam), W, H, out)
    t.cuda.synchronize()
    got = out.cpu().numpy().reshape(-1, 3)
    of = oracle.field_from(f)
    # the render's own arithmetic: the oracle fed the colour grid the GPU wrote
    gcol = col.float().cpu().numpy()[..., :3].astype(np.float64)
    ref, margin = oracle.volume_render(of, gcol, cam, W, H, N, skip_voxels=skip)
    keep = margin > SKIP_MARGIN
    assert keep.mean() > 0.99
    assert np.count_nonzero(ref.sum(1)) > 300
    nbad, emax = color_check(got, ref, FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} pixels off, max err {emax:.3g}"
    # the whole pipeline against the oracle's
    ocol = oracle.voxel_shade(of, cam, band)
    ref2, _ = oracle.volume_render(of, ocol, cam, W, H, N, skip_voxels=skip)
    rel = FP32_COLOR_REL + (2.0 ** -11 if colour_dt else 0.0)
    nbad, emax = color_check(got, ref2, rel, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} pixels off the pipeline, max err {emax:.3g}"


def test_rt512_full_size_sampled():
    """The benchmark's real-time launch: FP16 grids 512^3 / 128^3, band of 6 voxels,
    one 1920x1163 view, 128 samples with the skip rule; 1500 sampled pixels."""
    import paper_2412_10084_amd as ps
    t = torch()
    w = wl.WORKLOADS["rt512"]
    f = scene(0, w.R, w.P)
    fld = device_field(f, feat_half=True, sdf_half=True)
    fld.bounds = ps.sdf_bounds(fld.sdf)
    band = float(np.float32(wl.RT_BAND_VOXELS * 2.0 / (w.R - 1)))
    cam = wl.fibonacci_cameras(1, w.W, w.H)[0].as_array().astype(np.float32)
    print("rt512 launch: voxel shading + 1920x1163 volume render", flush=True)
    col, n, _ = gpu_colours(fld, w.R, cam, band, 1)
    out = t.empty((w.H, w.W, 3), device="cuda")
    ps.volume_render(fld, ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels, 0), col, dev(cam),
                     w.W, w.H, out)
    t.cuda.synchronize()
    of = oracle.field_from(f, half=True, half_sdf=True)
    rng = np.random.default_rng(23)
    ids = np.sort(rng.choice(w.W * w.H, 1500, replace=False))
    gcol = col.float().cpu().numpy()[..., :3].astype(np.float64)
    ref, margin = oracle.volume_render(of, gcol, cam, w.W, w.H, w.n_samples,
                                       skip_voxels=w.skip_voxels, pixel_ids=ids)
    got = out.reshape(-1, 3)[t.from_numpy(ids).cuda()].cpu().numpy()
    keep = margin > SKIP_MARGIN
    nbad, emax = color_check(got, ref, FP32_COLOR_REL, FP32_COLOR_ABS, keep)
    assert nbad == 0, f"{nbad} pixels off, max err {emax:.3g}"
    assert np.count_nonzero(ref.sum(1)) > 100
    # colours of 3000 sampled band nodes against the oracle's shading
    sh = np.flatnonzero(np.abs(f.sdf.astype(np.float16).astype(np.float32).reshape(-1))
                        <= np.float32(band))
    assert n == sh.size
    pick = np.sort(rng.choice(sh, 3000, replace=False))
    gc = gcol.reshape(-1, 3)[pick]
    R = w.R
    centre = np.array([cam[3], cam[7], cam[11]], np.float64)
    h = 2.0 / (R - 1)
    ref_c = np.zeros((pick.size, 3))
    for q, m in enumerate(pick):
        x = np.array([-1 + (m % R) * h, -1 + (m // R % R) * h, -1 + (m // (R * R)) * h])
        v = centre - x
        ref_c[q], _ = oracle.shade(of, x, v / np.linalg.norm(v))
    nbad, emax = color_check(gc, ref_c, FP32_COLOR_REL + 2.0 ** -11, FP32_COLOR_ABS)
    assert nbad == 0, f"{nbad} voxel colours off, max err {emax:.3g}"
