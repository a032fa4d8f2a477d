"""The C-ABI library loads, exports every symbol include/probesdf.h declares,
and rejects bad arguments on the host before any HIP call (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import paper_2412_10084_amd as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # a well-aligned non-NULL address; never dereferenced on these paths


def _declared():
    src = open(os.path.join(ROOT, "include", "probesdf.h")).read()
    return sorted(set(re.findall(r"\b(psdf_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = ps.lib()
    names = _declared()
    assert set(names) == set(ps.EXPORTS)
    for n in names:
        assert hasattr(L, n), n
    assert L.psdf_abi_version() == ps.ABI_VERSION


def _field(**kw):
    f = ps._Field(C.sizeof(ps._Field), 64, 16, 3, 9, 4, 16, 0, 0, 0, FAKE, FAKE, FAKE, FAKE)
    f.mlp_layers = 1
    for k, v in kw.items():
        setattr(f, k, v)
    return f


def _opts(**kw):
    o = ps._RenderOpts(C.sizeof(ps._RenderOpts), 64, 64.0, 0.0, 0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _fwd(f, o, B=0):
    L = ps.lib()
    return L.psdf_render_forward(C.byref(f) if f is not None else None,
                                 C.byref(o) if o is not None else None, B, FAKE, FAKE, FAKE, None,
                                 None, None, 0, None)


def test_empty_batch_ok():
    assert _fwd(_field(), _opts(), 0) == ps.OK


@pytest.mark.parametrize("kw,code", [
    (dict(struct_size=12), ps.EINVAL),
    (dict(R=1), ps.EINVAL),
    (dict(P=4096), ps.EINVAL),
    (dict(n_feat=4), ps.EUNSUPPORTED),
    (dict(sh_coeffs=5), ps.EUNSUPPORTED),
    (dict(mlp_hidden=32), ps.EUNSUPPORTED),
    (dict(mlp_layers=2), ps.EUNSUPPORTED),
    (dict(mlp_layers=0), ps.EUNSUPPORTED),
    (dict(feat_dtype=2), ps.EUNSUPPORTED),
    (dict(mlp_dtype=7), ps.EUNSUPPORTED),
    (dict(sdf=None), ps.EINVAL),
    (dict(probes=FAKE + 4), ps.EALIGN),
    (dict(sdf=FAKE + 2), ps.EALIGN),
    (dict(R=1000), ps.EINVAL),  # 1000^3 * 3 >= 2^31
    (dict(sdf_bounds=FAKE + 4), ps.EALIGN),
])
def test_field_validation(kw, code):
    assert _fwd(_field(**kw), _opts()) == code
    assert ps.last_error() != ""


@pytest.mark.parametrize("kw", [dict(n_samples=1), dict(n_samples=5000), dict(tau=0.0),
                                dict(tau=float("nan")), dict(flags=32), dict(struct_size=3)])
def test_opts_validation(kw):
    assert _fwd(_field(), _opts(**kw)) == ps.EINVAL


# the paper colour model's kernels and their limits
PAPER = dict(mlp_hidden=32, mlp_layers=2)


@pytest.mark.parametrize("fkw,okw", [
    (dict(sdf_dtype=1, feat_dtype=1, mlp_dtype=1), dict()),  # FP16 sdf
    (dict(mlp_dtype=1), dict()),                               # FP32 features, FP16 MLP
    (dict(feat_dtype=1), dict()),                              # FP16 features, FP32 MLP
    (dict(sh_coeffs=4), dict()),
    (dict(), dict(n_samples=514)),
])
def test_paper_model_limits(fkw, okw):
    assert _fwd(_field(**PAPER, **fkw), _opts(**okw), 10) == ps.EUNSUPPORTED
    assert "paper colour model" in ps.last_error()
    # the same limits hold when only a flag selects the paper model
    if "mlp_layers" not in fkw:
        f = _field(**fkw)
        assert _fwd(f, _opts(flags=ps.FLAG_SH_REFLECT, **okw), 10) == ps.EUNSUPPORTED


def test_paper_model_empty_batch_and_no_trace():
    assert _fwd(_field(**PAPER), _opts(flags=ps.FLAG_SH_REFLECT | ps.FLAG_FRESNEL_PAPER)) == ps.OK
    L = ps.lib()
    to = ps._TraceOpts(C.sizeof(ps._TraceOpts), 1e-3, 256, 0)
    assert L.psdf_render_sphere_trace(C.byref(_field(**PAPER)), C.byref(to), 1, FAKE, 8, 8, FAKE,
                                      None) == ps.EUNSUPPORTED


def test_mlp_sizes():
    assert ps.mlp_size() == ps.N_MLP == 227
    assert ps.mlp_size(ps.FLAG_FRESNEL_PAPER, 32, 2) == 32 * 13 + 32 + 32 * 32 + 32 + 3 * 32 + 3


def test_null_descriptors_and_negative_batch():
    assert _fwd(None, _opts()) == ps.EINVAL
    assert _fwd(_field(), None) == ps.EINVAL
    assert _fwd(_field(), _opts(), -1) == ps.EINVAL
    L = ps.lib()
    assert L.psdf_render_forward(C.byref(_field()), C.byref(_opts()), 10, None, FAKE, FAKE, None,
                                 None, None, 0, None) == ps.EINVAL
    assert L.psdf_render_forward(C.byref(_field()), C.byref(_opts()), 10, FAKE + 1, FAKE, FAKE,
                                 None, None, None, 0, None) == ps.EALIGN
    # a tape must be aligned and hold at least the per-wave arrays
    need = ps.backward_workspace_bytes(10, 16, 0)
    assert L.psdf_render_forward(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, FAKE, None,
                                 None, FAKE + 64, need, None) == ps.EALIGN
    assert L.psdf_render_forward(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, FAKE, None,
                                 None, FAKE, need - 1, None) == ps.EINVAL


def test_backward_requires_grads_and_aux():
    L = ps.lib()
    g = ps._Grads(FAKE, FAKE, FAKE, FAKE)
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, FAKE, FAKE,
                                  None, None, 0, 0, None) == ps.EINVAL
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, None, FAKE,
                                  C.byref(g), None, 0, 0, None) == ps.EINVAL
    g.probes = FAKE + 2
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, FAKE, FAKE,
                                  C.byref(g), None, 0, 0, None) == ps.EALIGN


def test_backward_workspace_validation():
    L = ps.lib()
    g = ps._Grads(FAKE, FAKE, FAKE, FAKE)
    B = 1000
    need = ps.backward_workspace_bytes(B, 16, 0)
    assert need > 0
    assert ps.backward_workspace_bytes(B, 16, 10) == need + 10 * 288
    assert ps.backward_workspace_bytes(B, 32, 0) > need
    # misaligned workspace
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), B, FAKE, FAKE, FAKE, FAKE,
                                  C.byref(g), FAKE + 64, need, 0, None) == ps.EALIGN
    # too small for the per-wave arrays
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), B, FAKE, FAKE, FAKE, FAKE,
                                  C.byref(g), FAKE, need - 1, 0, None) == ps.EINVAL
    assert "workspace" in ps.last_error()
    assert L.psdf_backward_workspace_bytes(-1, 16, 0) == -1
    assert L.psdf_backward_workspace_bytes(10, 16, -5) == -1
    assert L.psdf_backward_workspace_bytes(10, 1, 0) == -1
    # unknown flags; a tape backward without a workspace
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), B, FAKE, FAKE, FAKE, FAKE,
                                  C.byref(g), FAKE, need, 2, None) == ps.EINVAL
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), B, FAKE, FAKE, FAKE, FAKE,
                                  C.byref(g), None, 0, ps.BWD_FROM_TAPE, None) == ps.EINVAL
    # B = 0 with a workspace is a no-op
    assert L.psdf_render_backward(C.byref(_field()), C.byref(_opts()), 0, FAKE, FAKE, FAKE, FAKE,
                                  C.byref(g), FAKE, 0, 0, None) == ps.OK


def _step_args(**kw):
    a = ps._StepArgs()
    a.struct_size = C.sizeof(ps._StepArgs)
    a.R, a.P, a.n_feat, a.n_pc, a.n_mlp, a.step = 8, 4, 3, 36, 227, 1
    a.lr_sdf = a.lr_feat = a.lr_probe = a.lr_mlp = 0.01
    a.beta1, a.beta2, a.eps = 0.9, 0.995, 1e-8
    base = 0x100000
    ptrs = [n for n, ty in ps._StepArgs._fields_ if ty is C.c_void_p]
    for i, n in enumerate(ptrs):
        setattr(a, n, base + i * 0x100000)  # disjoint buffers
    a.sdf_half_out = a.feat_half_out = a.probes_half_out = a.losses = None
    a.s_in = a.s_out = a.work = a.losses_ext = None  # Sec. 3.3 regularisers unused
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def test_grid_step_validation():
    L = ps.lib()
    bad = _step_args(step=0)
    assert L.psdf_grid_step(C.byref(bad), None) == ps.EINVAL
    a = _step_args()
    a.sdf_out = a.sdf_in + 16  # overlapping in/out
    assert L.psdf_grid_step(C.byref(a), None) == ps.EINVAL
    assert "out of place" in ps.last_error()
    assert L.psdf_grid_step(C.byref(_step_args(beta1=1.0)), None) == ps.EINVAL
    assert L.psdf_grid_step(C.byref(_step_args(g_feat=None)), None) == ps.EINVAL
    assert L.psdf_grid_step(None, None) == ps.EINVAL
    a = _step_args()
    a.m_feat = a.m_feat + 4  # grid buffers must be 16-byte aligned
    assert L.psdf_grid_step(C.byref(a), None) == ps.EALIGN


def test_sphere_trace_and_loss_validation():
    L = ps.lib()
    to = ps._TraceOpts(C.sizeof(ps._TraceOpts), 1e-3, 256, 0)
    assert L.psdf_render_sphere_trace(C.byref(_field()), C.byref(to), 0, FAKE, 64, 64, FAKE,
                                      None) == ps.OK
    to.eps = 0.0
    assert L.psdf_render_sphere_trace(C.byref(_field()), C.byref(to), 1, FAKE, 64, 64, FAKE,
                                      None) == ps.EINVAL
    assert L.psdf_l1_loss(0, None, None, None, None, None) == ps.OK
    assert L.psdf_l1_loss(5, FAKE, None, FAKE, None, None) == ps.EINVAL


def test_sdf_bounds_validation():
    L = ps.lib()
    assert L.psdf_sdf_bounds(1, 0, FAKE, FAKE, None) == ps.EINVAL
    assert L.psdf_sdf_bounds(2000, 0, FAKE, FAKE, None) == ps.EINVAL
    assert L.psdf_sdf_bounds(64, 2, FAKE, FAKE, None) == ps.EUNSUPPORTED
    assert L.psdf_sdf_bounds(64, 0, None, FAKE, None) == ps.EINVAL
    assert L.psdf_sdf_bounds(64, 0, FAKE, None, None) == ps.EINVAL
    assert L.psdf_sdf_bounds(64, 0, FAKE + 2, FAKE, None) == ps.EALIGN
    assert L.psdf_sdf_bounds(64, 0, FAKE, FAKE + 4, None) == ps.EALIGN
    assert ps.n_bricks(2) == 1 and ps.n_bricks(9) == 1 and ps.n_bricks(10) == 2
    assert ps.n_bricks(256) == 32 and ps.n_bricks(257) == 32 and ps.n_bricks(258) == 33


def test_grid_step_regulariser_validation():
    """Sec. 3.3's regularisers: a work buffer of the stated size, the smoothed
    fields with PSDF_STEP_SMOOTH, L_sdf only with smoothing, a positive width."""
    L = ps.lib()
    need = ps.step_work_bytes(8)
    assert need == 8 * 8 ** 3 * 4
    assert ps.lib().psdf_step_work_bytes(1) == -1
    W = 0x7000000
    assert L.psdf_grid_step(C.byref(_step_args(lambda_normal=0.1)), None) == ps.EINVAL
    assert "work buffer" in ps.last_error()
    assert L.psdf_grid_step(C.byref(_step_args(lambda_normal=0.1, work=W, work_bytes=need - 1)),
                            None) == ps.EINVAL
    assert L.psdf_grid_step(C.byref(_step_args(lambda_normal=0.1, work=W + 4, work_bytes=need)),
                            None) == ps.EALIGN
    assert L.psdf_grid_step(C.byref(_step_args(lambda_sdf=0.1, work=W, work_bytes=need)),
                            None) == ps.EINVAL
    assert "PSDF_STEP_SMOOTH" in ps.last_error()
    sm = dict(sdf_reg_flags=ps.STEP_SMOOTH, work=W, work_bytes=need, smooth_sigma=1.0)
    assert L.psdf_grid_step(C.byref(_step_args(**sm)), None) == ps.EINVAL  # no s_in / s_out
    sm.update(s_in=0x8000000, s_out=0x9000000)
    assert L.psdf_grid_step(C.byref(_step_args(**dict(sm, smooth_sigma=0.0))), None) == ps.EINVAL
    assert L.psdf_grid_step(C.byref(_step_args(**dict(sm, sdf_reg_flags=8))), None) == ps.EINVAL
    a = _step_args(**sm)
    a.s_out = a.sdf_out
    assert L.psdf_grid_step(C.byref(a), None) == ps.EINVAL
    # smoothing and the relative L2 loss validate before launching
    assert L.psdf_smooth_sdf(8, 0.0, FAKE, FAKE + 4096, None, None) == ps.EINVAL
    assert L.psdf_smooth_sdf(8, 1.0, FAKE, FAKE + 16, None, None) == ps.EINVAL  # overlap
    assert L.psdf_smooth_sdf(1, 1.0, FAKE, FAKE + 4096, None, None) == ps.EINVAL
    assert L.psdf_l2rel_loss(10, FAKE, FAKE, FAKE, None, 40.0, 0.0, 1.0, None) == ps.EINVAL
    assert L.psdf_l2rel_loss(10, FAKE, FAKE, FAKE, None, 40.0, 1e-3, 0.0, None) == ps.EINVAL
    assert L.psdf_l2rel_loss(0, None, None, None, None, 40.0, 1e-3, 1.0, None) == ps.OK


def test_grid_step_bounds_alignment():
    L = ps.lib()
    a = _step_args()
    a.sdf_bounds_out = a.sdf_bounds_out + 4
    assert L.psdf_grid_step(C.byref(a), None) == ps.EALIGN


def test_backward_noalloc_validation():
    """The allocation-free backward validates like render_backward and rejects
    batches whose fixed workspace part exceeds its static scratch, before any
    HIP call."""
    L = ps.lib()
    g = ps._Grads(FAKE, FAKE, FAKE, FAKE)
    fn = L.psdf_render_backward_noalloc
    assert fn(C.byref(_field()), C.byref(_opts()), 0, FAKE, FAKE, FAKE, FAKE, C.byref(g),
              None) == ps.OK
    assert fn(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, FAKE, FAKE, None,
              None) == ps.EINVAL
    assert fn(C.byref(_field()), C.byref(_opts()), 10, FAKE, FAKE, None, FAKE, C.byref(g),
              None) == ps.EINVAL
    assert fn(None, C.byref(_opts()), 10, FAKE, FAKE, FAKE, FAKE, C.byref(g), None) == ps.EINVAL
    # P = 256: the probe-cell bins alone (3 x 4 B x 8 x 128^3) exceed 128 MiB
    assert fn(C.byref(_field(P=256)), C.byref(_opts()), 10, FAKE, FAKE, FAKE, FAKE, C.byref(g),
              None) == ps.EINVAL
    assert "static scratch" in ps.last_error()
    # 2^31 rays: the per-wave arrays alone (3 x 4 B x 2^25) exceed it
    assert fn(C.byref(_field()), C.byref(_opts()), 1 << 31, FAKE, FAKE, FAKE, FAKE, C.byref(g),
              None) == ps.EINVAL
    assert "static scratch" in ps.last_error()
    assert ps.backward_workspace_bytes(1 << 20, 128, 0) < ps.NOALLOC_SCRATCH_BYTES


def test_binding_rejects_wrong_dtype_and_host_tensors():
    """The binding refuses float64 and host tensors before anything reaches the library
    (no GPU needed: the checks run on the host)."""
    import torch
    import paper_2412_10084_amd as ps
    fld = ps.Field(sdf=torch.zeros(4, 4, 4), feat=torch.zeros(4, 4, 4, 3),
                   probes=torch.zeros(2, 2, 2, 9, 4), mlp=torch.zeros(227))
    o = torch.zeros(8, 3)
    rgb = torch.zeros(8, 3)
    with pytest.raises(ps.PsdfError, match="float32"):
        ps.render_forward(fld, ps.RenderOpts(), o.double(), o, rgb)
    with pytest.raises(ps.PsdfError, match="not on the GPU"):
        ps.render_forward(fld, ps.RenderOpts(), o, o, rgb)
    with pytest.raises(ps.PsdfError, match="float32"):
        ps.l1_loss(rgb, rgb.half(), rgb)


def test_realtime_validation():
    """Band list, voxel shading and volume rendering validate before launching."""
    L = ps.lib()
    assert L.psdf_voxel_list(1, 0, FAKE, 0.1, FAKE, 8, FAKE, None) == ps.EINVAL
    assert L.psdf_voxel_list(8, 2, FAKE, 0.1, FAKE, 8, FAKE, None) == ps.EUNSUPPORTED
    assert L.psdf_voxel_list(8, 0, FAKE, 0.1, FAKE, 513, FAKE, None) == ps.EINVAL  # > R^3
    assert L.psdf_voxel_list(8, 0, FAKE, float("nan"), FAKE, 8, FAKE, None) == ps.EINVAL
    assert L.psdf_voxel_list(8, 0, FAKE + 2, 0.1, FAKE, 8, FAKE, None) == ps.EALIGN
    vs = L.psdf_voxel_shade
    assert vs(C.byref(_field()), 8, FAKE, FAKE, FAKE, 16, FAKE, 0, None) == ps.EINVAL  # flags
    assert vs(C.byref(_field()), 0, FAKE, FAKE, FAKE, 16, FAKE, 2, None) == ps.EUNSUPPORTED
    assert vs(C.byref(_field()), 0, FAKE, FAKE, FAKE, 16, FAKE + 8, 0, None) == ps.EALIGN
    assert vs(C.byref(_field(mlp_hidden=32, mlp_layers=2)), 0, FAKE, FAKE, FAKE, 16, FAKE, 0,
              None) == ps.EUNSUPPORTED
    assert vs(C.byref(_field()), 0, FAKE, FAKE, FAKE, 0, FAKE, 0, None) == ps.OK  # nothing listed
    vr = L.psdf_volume_render
    assert vr(C.byref(_field()), C.byref(_opts(flags=1)), FAKE, 0, FAKE, 8, 8, FAKE,
              None) == ps.EINVAL
    assert vr(C.byref(_field()), C.byref(_opts()), FAKE, 0, FAKE, -1, 8, FAKE, None) == ps.EINVAL
    assert vr(C.byref(_field()), C.byref(_opts()), FAKE, 0, FAKE, 0, 8, FAKE, None) == ps.OK


def test_tile_and_plane_step_validation():
    L = ps.lib()
    assert _fwd(_field(tile_T=1), _opts(), 10) == ps.EINVAL  # R must be 16 T + 1
    assert _fwd(_field(R=65, tile_T=4), _opts(), 10) == ps.EINVAL  # no tile index
    assert _fwd(_field(R=65, tile_T=4, tile_index=FAKE + 2), _opts(), 10) == ps.EALIGN
    assert _fwd(_field(R=65, tile_T=4, tile_index=FAKE, n_tiles=65), _opts(), 10) == ps.EINVAL
    # tiled fields take the paper colour model's kernels and their limits
    assert _fwd(_field(R=65, tile_T=4, tile_index=FAKE, n_tiles=8, sh_coeffs=4), _opts(),
                10) == ps.EUNSUPPORTED
    ps_ = L.psdf_plane_step
    args = dict(n=2, nf=3, i=FAKE, o=FAKE * 64, g=FAKE * 128, m=FAKE * 192, v=FAKE * 256)

    def call(**kw):
        a = dict(args, **kw)
        return ps_(a["n"], a["nf"], a["i"], a["o"], a["g"], a["m"], a["v"], kw.get("step", 1),
                   0.01, 0.9, 0.995, 1e-8, 0.05, None, None, None)

    assert call(nf=4) == ps.EUNSUPPORTED
    assert call(step=0) == ps.EINVAL
    assert call(o=FAKE + 16) == ps.EINVAL  # in / out overlap
    assert call(m=FAKE * 192 + 4) == ps.EALIGN
    assert call(n=0) == ps.OK
