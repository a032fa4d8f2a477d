"""Every entry point of the oracle once, on tiny inputs: run by
test_oracle_sanitized.py in a process that loads the AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle, so that an out-of-bounds access,
use after free or undefined arithmetic anywhere in it aborts the run.  Sizes are
chosen to reach the edge cases of the indexing: ragged grids, N above the old
fixed-size limit, rays that miss, empty tiles, grid borders."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
import workloads as wl  # noqa: E402


def main() -> None:
    oracle.set_threads(2)
    rng = np.random.default_rng(0)
    o, d = wl.camera_rays(wl.fibonacci_cameras(2, 6, 4), 6, 4)
    for n_sh, model, flags in ((1, "workload", 0), (9, "workload", 4), (16, "paper", 8 | 16)):
        f = wl.random_field(1, 13, 5, n_sh=n_sh, model=model)
        of = oracle.field_from(f)
        for N, skip in ((2, 0.0), (40, 3.0), (1100, 0.0)):
            ref = oracle.render_forward(of, o, d, N, skip_voxels=skip, flags=flags)
            dL = rng.standard_normal(ref["rgb"].shape)
            oracle.render_backward(of, o, d, dL, N, skip_voxels=skip, flags=flags)
        oracle.shade(of, np.array([0.99, -1.0, 0.3]), np.array([0.0, 0.6, 0.8]), flags)
    oracle.render_forward(of, np.array([[5.0, 5.0, 5.0]]), np.array([[1.0, 0.0, 0.0]]), 8, flags=flags)
    # sparse tiles: one allocated tile of eight, both colour models
    for model, flags in (("workload", 0), ("paper", 8 | 16)):
        f = wl.tiled_field(2, 2, model=model, n_sh=9)
        f.tiles.index[:] = -1
        f.tiles.index[0, 0, 0] = 0
        f.tiles.planes = f.tiles.planes[:1].copy()
        of = oracle.field_from(f)
        ref = oracle.render_forward(of, o, d, 24, flags=flags)
        oracle.render_backward(of, o, d, np.ones_like(ref["rgb"]), 24, flags=flags)
        oracle.triplane(of, np.array([-1.0, -1.0, -1.0]))
        oracle.triplane(of, np.array([1.0, 1.0, 1.0]))
    oracle.plane_smooth(rng.standard_normal((2, 3, 16, 16, 3)), 0.1)
    # losses, regularisers and the optimiser steps
    rgb, tgt = rng.uniform(0, 1, (7, 3)), rng.uniform(0, 1, (7, 3))
    oracle.l1_loss(rgb, tgt)
    oracle.l2rel_loss(rgb, tgt)
    f = wl.random_field(3, 7, 4)
    oracle.regularizers(f.sdf, f.feat, f.probes, 0.1, 0.05, 0.2)
    oracle.adam(rng.standard_normal(5), rng.standard_normal(5), np.zeros(5), np.zeros(5), 1, 0.01)
    shat = rng.standard_normal((6, 6, 6))
    oracle.smooth(shat)
    oracle.smooth_T(shat)
    for smooth in (False, True):
        for weighted in (False, True):
            oracle.sdf_regs(shat, rng.standard_normal(shat.shape), smooth=smooth, weighted=weighted)
    params = dict(sdf=f.sdf, feat=f.feat, probes=f.probes, mlp=f.mlp)
    grads = {k: rng.standard_normal(np.shape(v)) * 1e-3 for k, v in params.items()}
    n = sum(np.size(v) for v in params.values())
    oracle.grid_step(params, grads, np.zeros(n), np.zeros(n), 1, oracle.StepOpts())
    oracle.grid_step_ext(params, grads, np.zeros(n), np.zeros(n), 2,
                         oracle.StepExt(oracle.StepOpts(), weighted=True))
    # real-time path and sphere tracing
    f = wl.random_field(4, 11, 4)
    of = oracle.field_from(f)
    cam = wl.fibonacci_cameras(2, 9, 5)[1].as_array()
    col = oracle.voxel_shade(of, cam, 3 * 2.0 / 10)
    oracle.volume_render(of, col, cam, 9, 5, 33, skip_voxels=2.0)
    cams = np.stack([c.as_array() for c in wl.fibonacci_cameras(2, 9, 5)])
    oracle.sphere_trace(of, cams, 9, 5, max_steps=40)
    print("oracle entry points ran clean")


if __name__ == "__main__":
    main()
