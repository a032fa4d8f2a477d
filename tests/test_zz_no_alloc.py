"""The allocation-free backward (psdf_render_backward_noalloc) against the
backward with a caller workspace of the same size, through the C ABI: two calls
in a row on one GPU, the second with a smaller batch (the static scratch keeps
the first call's contents), and a third whose shaded samples overflow the
scratch (those waves take the fused schedule).  Both are also held to the FP64
oracle's gradients."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_common import dev, device_field, gpu_forward, grad_check, rays, scene, torch

pytestmark = pytest.mark.gpu


def _grads(fld):
    t = torch()
    return dict(sdf=t.zeros(fld.sdf.shape, device="cuda"), feat=t.zeros(fld.feat.shape, device="cuda"),
                probes=t.zeros(fld.probes.shape, device="cuda"), mlp=t.zeros(227, device="cuda"))


def _case(f, o, d, N, skip, seed, with_oracle=True):
    import paper_2412_10084_amd as ps
    t = torch()
    print(f"no-alloc case: B={o.shape[0]} R={f.R} P={f.P} N={N} skip={skip}", flush=True)
    fld = device_field(f)
    if skip > 0:
        fld.bounds = ps.sdf_bounds(fld.sdf)
    got = gpu_forward(fld, o, d, N, skip=skip)
    do, dd, _, aux = got["dev"]
    rng = np.random.default_rng(seed)
    B = o.shape[0]
    dL = (rng.choice([-1.0, 0.0, 1.0], size=(B, 3)) / (3.0 * B)).astype(np.float32)
    opts = ps.RenderOpts(N, 64.0, skip, 0)
    g_na = _grads(fld)
    ps.render_backward_noalloc(fld, opts, do, dd, aux, dev(dL), g_na)
    ws = t.empty(ps.NOALLOC_SCRATCH_BYTES, dtype=t.uint8, device="cuda")
    g_ws = _grads(fld)
    ps.render_backward(fld, opts, do, dd, aux, dev(dL), g_ws, workspace=ws)
    t.cuda.synchronize()
    a = {k: v.cpu().numpy().astype(np.float64) for k, v in g_na.items()}
    b = {k: v.cpu().numpy().astype(np.float64) for k, v in g_ws.items()}
    grad_check(a, b, "fp32")  # no-alloc vs workspace
    for k in a:
        assert np.count_nonzero(a[k]) > 0, f"{k}: no gradient"
    if with_oracle:
        ref = oracle.render_backward(oracle.field_from(f), o, d, dL.astype(np.float64), N,
                                     skip_voxels=skip)
        grad_check(a, ref, "fp32")  # no-alloc vs oracle


def test_noalloc_backward_two_calls_then_overflow():
    f = scene(0, 64, 16)
    o, d = rays(8, 32, 16)
    # first call: 4096 rays, every sample active
    _case(f, o, d, 64, 0.0, seed=1)
    # second call, smaller and ragged (not a multiple of 64 rays), with the skip rule
    sub = np.arange(0, o.shape[0], 3)[:1000]
    _case(f, np.ascontiguousarray(o[sub]), np.ascontiguousarray(d[sub]), 64, 4.0, seed=2)
    # third: ~2^16 rays x ~30 shaded samples, more than the scratch holds
    o2, d2 = rays(8, 128, 64)
    _case(f, o2, d2, 64, 0.0, seed=3, with_oracle=False)
