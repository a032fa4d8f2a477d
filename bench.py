"""Benchmark of the ProbeSDF render step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one training iteration of the render path on the train256 workload
(256^3 SDF + 3 features, 64^3 probes x 9 SH x 4, MLP 10-16-3; 2^18 rays from 8
cameras at 256x128, 128 samples, skip |s| > 4 voxels; L1 loss against a torus
target): render_forward (recording its tape) -> l1_loss -> render_backward (from
the tape) -> grid_step (eikonal + smoothness + Adam over all 76.5 M parameters,
writing the SDF brick bounds the next forward skips empty space with).  Inputs
are resident in HBM before timing starts.  value = rays per second of that whole
step.

The JSON line also carries the per-kernel times, the roofline of the dominant
kernel (HIP events on the stream the kernels run on), the same step with FP16
storage and the MLP on FP16 MFMA, the sphere-traced 1080p inference rate, and
the FP64 oracle timed on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class KernelTimer:
    """Events around each launch on torch's current stream (the launch stream); `only`
    limits them to the named entry points."""

    def __init__(self, torch, only=None):
        self.torch = torch
        self.pending = []
        self.enabled = False
        self.only = only

    def run(self, name, fn):
        if not self.enabled or (self.only is not None and name not in self.only):
            fn()
            return
        t = self.torch
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.pending.append((name, a, b))

    def summary(self):
        out = {}
        for name, a, b in self.pending:
            out.setdefault(name, []).append(a.elapsed_time(b))
        return {k: sum(v) / len(v) for k, v in out.items()}


def ws_samples(w, B):
    """Room for shaded samples in the backward workspace: with the skip rule about one
    sample per ray is shaded (train256: 1.09), so 8 per ray; without it up to N - 1."""
    return 8 * B if w.skip_voxels > 0 else (w.n_samples - 1) * B


def make_state(torch, ps, wl, w, feat_half=False, mlp_dtype=0, seed=0, order="image"):
    import numpy as np
    f = wl.random_field(seed, w.R, w.P, n_sh=w.n_sh)
    ft = wl.random_field(seed + 1, w.R, w.P, n_sh=w.n_sh, shape="torus")
    if order == "shuffled":
        o, d = wl.shuffled(*wl.workload_rays(w), seed=2)
    else:
        o, d = wl.workload_rays(w, order)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    master = dict(sdf=cu(f.sdf), feat=cu(f.feat), probes=cu(f.probes), mlp=cu(f.mlp))
    spare = {k: torch.empty_like(v) for k, v in master.items() if k != "mlp"}
    half = {}
    if feat_half:
        half = dict(feat=master["feat"].half(), probes=master["probes"].half())
    st = dict(master=master, spare=spare, half=half, mlp_dtype=mlp_dtype,
              o=cu(o), d=cu(d), B=o.shape[0],
              grads={k: torch.zeros_like(v) for k, v in master.items()},
              m={k: torch.zeros_like(v) for k, v in master.items()},
              v={k: torch.zeros_like(v) for k, v in master.items()})
    B = o.shape[0]
    st["rgb"] = torch.empty((B, 3), device="cuda")
    st["aux"] = torch.empty((B, 4), device="cuda")
    st["dL"] = torch.empty((B, 3), device="cuda")
    st["loss"] = torch.empty(1, device="cuda")
    # brick bounds of the initial SDF; every grid step writes those of the next one
    st["bounds"] = ps.sdf_bounds(master["sdf"])
    st["ws"] = ps.backward_workspace(B, w.P, ws_samples(w, B))
    # target image: the torus field rendered by the same forward kernel
    tfield = ps.Field(cu(ft.sdf), cu(ft.feat), cu(ft.probes), cu(ft.mlp))
    st["target"] = torch.empty((B, 3), device="cuda")
    ps.render_forward(tfield, ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels), st["o"], st["d"],
                      st["target"])
    torch.cuda.synchronize()
    del tfield
    return st, f, (o, d)


def train_step(ps, w, st, step, timer):
    p = st["master"]
    if st["half"]:
        fld = ps.Field(p["sdf"], st["half"]["feat"], st["half"]["probes"], p["mlp"], st["mlp_dtype"],
                       st["bounds"])
    else:
        fld = ps.Field(p["sdf"], p["feat"], p["probes"], p["mlp"], st["mlp_dtype"], st["bounds"])
    opts = ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels)
    timer.run("render_forward", lambda: ps.render_forward(fld, opts, st["o"], st["d"], st["rgb"],
                                                           st["aux"], tape=st["ws"]))
    timer.run("l1_loss", lambda: ps.l1_loss(st["rgb"], st["target"], st["dL"], st["loss"]))
    timer.run("render_backward", lambda: ps.render_backward(fld, opts, st["o"], st["d"], st["aux"],
                                                             st["dL"], st["grads"],
                                                             workspace=st["ws"], from_tape=True))
    out = dict(st["spare"], mlp=p["mlp"])
    timer.run("grid_step", lambda: ps.grid_step(p, out, st["grads"], st["m"], st["v"], step,
                                                ps.StepOpts(), half_out=st["half"] or None,
                                                bounds_out=st["bounds"]))
    # ping-pong the grids (the step is out of place)
    st["spare"] = {k: p[k] for k in ("sdf", "feat", "probes")}
    st["master"] = dict(sdf=out["sdf"], feat=out["feat"], probes=out["probes"], mlp=p["mlp"])


def clone_state(torch, st, memo=None):
    """Copy of a training state: tensors cloned (a tensor held twice stays one tensor),
    containers rebuilt, everything else shared."""
    memo = {} if memo is None else memo
    if isinstance(st, torch.Tensor):
        if id(st) not in memo:
            memo[id(st)] = st.clone()
        return memo[id(st)]
    if isinstance(st, dict):
        return {k: clone_state(torch, v, memo) for k, v in st.items()}
    if isinstance(st, (list, tuple)):
        return type(st)(clone_state(torch, v, memo) for v in st)
    return st


def time_training(torch, ps, w, st, steps, warmup, label, live=("grid_step",)):
    """ms per step over `steps` timed steps, and the mean time of each entry point.
    In the timed steps only the `live` entry points (the roofline's) are bracketed by
    events: an event pair around every entry point adds ~25 us to a 0.9 ms step. The
    other entry points are timed in a second, untimed pass of as many steps."""
    timer = KernelTimer(torch, only=set(live))
    for i in range(warmup):
        train_step(ps, w, st, i + 1, timer)
    torch.cuda.synchronize()
    log(f"{label}: warmup done ({warmup} steps)")
    snap = clone_state(torch, st)
    timer.enabled = True
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for i in range(steps):
        train_step(ps, w, st, warmup + i + 1, timer)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    # the same steps again from the state the timed ones started from
    every = KernelTimer(torch)
    every.enabled = True
    for i in range(steps):
        train_step(ps, w, snap, warmup + i + 1, every)
    torch.cuda.synchronize()
    del snap
    kern = every.summary()
    kern.update(timer.summary())
    log(f"{label}: {ms:.3f} ms/step, kernels " + ", ".join(f"{k} {v:.3f}" for k, v in kern.items()))
    return ms, kern


def time_inference(torch, ps, wl, steps, warmup):
    """Sphere-traced inference, FP16 grids 512^3 / 128^3, 16 views at 1920x1080."""
    import numpy as np
    w = wl.WORKLOADS["trace512"]
    fld = gpu_field(torch, ps, wl, w, 0, feat_half=True, sdf_half=True)
    cams = torch.from_numpy(np.stack([c.as_array() for c in wl.fibonacci_cameras(w.views, w.W, w.H)])).cuda()
    out = torch.empty((w.views, w.H, w.W, 3), device="cuda")
    for _ in range(warmup):
        ps.sphere_trace(fld, cams, w.W, w.H, out)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        ps.sphere_trace(fld, cams, w.W, w.H, out)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    rays = w.views * w.W * w.H
    log(f"inference: {ms:.3f} ms per launch of {w.views} views")
    return dict(workload="trace512", ms_per_frame=ms / w.views, rays_per_s=rays / (ms * 1e-3),
                views=w.views, W=w.W, H=w.H, grids="fp16 512^3 / 128^3", mlp="f32")


def gpu_field(torch, ps, wl, w, seed, shape="sphere", feat_half=False, sdf_half=False,
              mlp_dtype=0):
    """Seeded synthetic field generated on the GPU (large grids; no oracle needed)."""
    import numpy as np
    g = torch.Generator(device="cuda").manual_seed(seed)
    R, P = w.R, w.P
    a = torch.linspace(-1.0, 1.0, R, device="cuda", dtype=torch.float64)
    sdf = torch.empty((R, R, R), device="cuda", dtype=torch.float32)
    for k in range(R):  # slice by slice keeps the FP64 temporaries small
        y, x = torch.meshgrid(a, a, indexing="ij")
        if shape == "sphere":
            v = torch.sqrt(x * x + y * y + a[k] * a[k]) - 0.5
        else:
            v = torch.sqrt((torch.sqrt(x * x + y * y) - 0.5) ** 2 + a[k] * a[k]) - 0.2
        sdf[k] = v.float()
    feat = torch.randn((R, R, R, 3), generator=g, device="cuda") * 0.1
    probes = torch.randn((P, P, P, w.n_sh, 4), generator=g, device="cuda") * 0.1
    mlp = torch.from_numpy(wl.xavier_uniform_mlp(np.random.default_rng(seed))).cuda()
    if feat_half:
        feat, probes = feat.half(), probes.half()
    if sdf_half:
        sdf = sdf.half()
    return ps.Field(sdf, feat, probes, mlp, mlp_dtype)


def time_fwd_bwd_512(torch, ps, wl, steps, warmup):
    """mixed512: forward + L1 + backward at 512^3 / 128^3, 2^20 rays, N = 64, no skip,
    FP32 and FP16 storage with the MLP on FP16 MFMA (and BF16)."""
    import numpy as np
    w = wl.WORKLOADS["mixed512"]
    o, d = wl.workload_rays(w)
    do, dd = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    B = o.shape[0]
    opts = ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels)
    tgt = torch.empty((B, 3), device="cuda")
    tf = gpu_field(torch, ps, wl, w, 1, shape="torus")
    ps.render_forward(tf, opts, do, dd, tgt)
    del tf
    out = {}
    base = gpu_field(torch, ps, wl, w, 0)
    ws = ps.backward_workspace(B, w.P, ws_samples(w, B))
    for label, half, mdt in (("fp32", False, 0), ("fp16", True, 1), ("bf16", True, 2)):
        fld = ps.Field(base.sdf, base.feat.half() if half else base.feat,
                       base.probes.half() if half else base.probes, base.mlp, mdt)
        rgb = torch.empty((B, 3), device="cuda")
        aux = torch.empty((B, 4), device="cuda")
        dL = torch.empty((B, 3), device="cuda")
        grads = {k: torch.zeros(v.shape, device="cuda", dtype=torch.float32) for k, v in
                 dict(sdf=fld.sdf, feat=fld.feat, probes=fld.probes, mlp=fld.mlp).items()}
        def step():
            ps.render_forward(fld, opts, do, dd, rgb, aux, tape=ws)
            ps.l1_loss(rgb, tgt, dL)
            ps.render_backward(fld, opts, do, dd, aux, dL, grads, workspace=ws, from_tape=True)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        tf_ms = tb_ms = 0.0
        for _ in range(steps):
            e[0].record()
            ps.render_forward(fld, opts, do, dd, rgb, aux, tape=ws)
            e[1].record()
            ps.l1_loss(rgb, tgt, dL)
            e[2].record()
            ps.render_backward(fld, opts, do, dd, aux, dL, grads, workspace=ws, from_tape=True)
            e[3].record()
            torch.cuda.synchronize()
            tf_ms += e[0].elapsed_time(e[1])
            tb_ms += e[2].elapsed_time(e[3])
        tf_ms /= steps
        tb_ms /= steps
        A = recorded_samples(torch, ws) / B
        half_b = label != "fp32"
        out[label] = {"fwd_ms": tf_ms, "bwd_ms": tb_ms,
                      "fwd_bwd_rays_per_s": B / ((tf_ms + tb_ms) * 1e-3),
                      "shaded_samples_per_ray": A,
                      "roofline_render": {
                          e: roofline_obj(e, B * alg_bytes_per_ray(e, w.n_samples, A, half_b), t,
                                          measured_traffic(e, "mixed512", label))
                          for e, t in (("render_forward", tf_ms), ("render_backward", tb_ms))}}
        log(f"mixed512 {label}: fwd {tf_ms:.3f} ms, bwd {tb_ms:.3f} ms")
        del fld, grads
        torch.cuda.empty_cache()
    out["ratio_fp16_vs_fp32"] = out["fp16"]["fwd_bwd_rays_per_s"] / out["fp32"]["fwd_bwd_rays_per_s"]
    out["ratio_bf16_vs_fp32"] = out["bf16"]["fwd_bwd_rays_per_s"] / out["fp32"]["fwd_bwd_rays_per_s"]
    out["config"] = {"R": w.R, "P": w.P, "rays": B, "samples": w.n_samples, "skip_voxels": 0}
    return out


def time_iter512(torch, ps, wl, iters, warmup):
    """iter512: full training iteration (forward, L1, backward, grid step over all
    512^3 x 4 + 128^3 x 36 + 227 parameters) at 2^20 rays, N = 128, skip 4 voxels."""
    w = wl.WORKLOADS["iter512"]
    o, d = wl.workload_rays(w)
    st = dict(o=torch.from_numpy(o).cuda(), d=torch.from_numpy(d).cuda(), B=o.shape[0], half={},
              mlp_dtype=0)
    f0 = gpu_field(torch, ps, wl, w, 0)
    st["master"] = dict(sdf=f0.sdf, feat=f0.feat, probes=f0.probes, mlp=f0.mlp)
    st["spare"] = {k: torch.empty_like(v) for k, v in st["master"].items() if k != "mlp"}
    st["grads"] = {k: torch.zeros_like(v) for k, v in st["master"].items()}
    st["m"] = {k: torch.zeros_like(v) for k, v in st["master"].items()}
    st["v"] = {k: torch.zeros_like(v) for k, v in st["master"].items()}
    B = st["B"]
    for k in ("rgb", "dL", "target"):
        st[k] = torch.empty((B, 3), device="cuda")
    st["aux"] = torch.empty((B, 4), device="cuda")
    st["loss"] = torch.empty(1, device="cuda")
    st["bounds"] = ps.sdf_bounds(f0.sdf)
    st["ws"] = ps.backward_workspace(B, w.P, ws_samples(w, B))
    tf = gpu_field(torch, ps, wl, w, 1, shape="torus")
    ps.render_forward(tf, ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels), st["o"], st["d"],
                      st["target"])
    del tf
    ms, kern = time_training(torch, ps, w, st, iters, warmup, "iter512")
    return {"ms_per_iteration": ms, "iterations": iters, "kernels_ms": kern,
            "rays_per_s": B / (ms * 1e-3),
            "params": w.R ** 3 * 4 + w.P ** 3 * w.n_sh * 4 + 227,
            "grid_step_GBps": 32.0 * (w.R ** 3 * 4 + w.P ** 3 * w.n_sh * 4) / (kern["grid_step"] * 1e-3) / 1e9}


def ev_time(torch, fn, reps):
    """Mean ms of `fn` over `reps` launches: HIP events on torch's current stream, the
    stream the library launches on."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def recorded_samples(torch, ws) -> int:
    """Shaded samples the last taped forward recorded (the workspace's slot counter)."""
    return int(ws[:8].view(torch.int64).item())


def alg_bytes_per_ray(entry: str, N: int, A: float, half: bool) -> float:
    """Algorithmic bytes per ray of the render entry points (every sample's SDF
    scanned, 8 corners x 4 B; per shaded sample the FD stencil, features and probes:
    1344 B FP32, 720 B with FP16 features and probes, plus the 32 B of its own cell in
    the backward, which also writes the same footprint of FP32 gradients, 1376 B;
    ray / colour I/O)."""
    per = 720.0 if half else 1344.0
    if entry == "render_forward":
        return 32.0 * N + A * per + 64.0
    return 32.0 * N + A * (per + 32.0 + 1376.0) + 52.0


def alg_bytes_model(entry: str, N: int, A: float, half: bool, n_sh: int, tiled: bool) -> float:
    """Algorithmic bytes per ray of the paper colour model's kernels (and of tiled
    fields, which run on them): the SDF scan, and per shaded sample the FD stencil (96 B),
    the spatial features (8 corners x 3, or 12 tri-plane texels x 3, in the storage
    precision) and 8 probe corners x n_sh x 4 coefficients; the backward also writes
    the same footprint of FP32 gradients plus the 32 B of the sample's own cell."""
    fb = 2.0 if half else 4.0
    feat = (12 if tiled else 8) * 3
    shade = 96.0 + feat * fb + 8 * n_sh * 4 * fb
    if entry == "render_forward":
        return 32.0 * N + A * shade + 64.0
    return 32.0 * N + A * (shade + 32.0 + 96.0 + feat * 4.0 + 8 * n_sh * 16.0) + 52.0


def shaded_per_ray(torch, ps, w, sdf, P, o, d) -> float:
    """Shaded samples per ray (active, alpha > 0) of an SDF: they depend on the SDF and
    the rays only, so the workload model's taped forward over zero features counts them."""
    R = sdf.shape[0]
    fld = ps.Field(sdf, torch.zeros((R, R, R, 3), device="cuda", dtype=torch.float32),
                   torch.zeros((P, P, P, w.n_sh, 4), device="cuda"),
                   torch.zeros(227, device="cuda"), 0, ps.sdf_bounds(sdf))
    B = o.shape[0]
    ws = ps.backward_workspace(B, P, ws_samples(w, B))
    rgb, aux = torch.empty((B, 3), device="cuda"), torch.empty((B, 4), device="cuda")
    ps.render_forward(fld, ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels), o, d, rgb, aux,
                      tape=ws)
    torch.cuda.synchronize()
    A = recorded_samples(torch, ws) / B
    del fld, ws
    torch.cuda.empty_cache()
    return A


def roofline_obj(kernel: str, per_launch: float, ms: float, traffic):
    ach = per_launch / (ms * 1e-3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": per_launch, "launch_ms": ms}


def train256_extras(torch, ps, w, st, kern, reps):
    """Shaded samples per ray (the tape's counter), the render steps' rooflines and the
    re-marching backward (entry-parallel schedule, no tape) beside the taped one."""
    p = st["master"]
    fld = ps.Field(p["sdf"], p["feat"], p["probes"], p["mlp"], 0, st["bounds"])
    opts = ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels)
    ps.render_forward(fld, opts, st["o"], st["d"], st["rgb"], st["aux"], tape=st["ws"])
    torch.cuda.synchronize()
    B = st["B"]
    A = recorded_samples(torch, st["ws"]) / B
    remarch = ev_time(torch, lambda: ps.render_backward(fld, opts, st["o"], st["d"], st["aux"],
                                                        st["dL"], st["grads"],
                                                        workspace=st["ws"]), reps)
    for g in st["grads"].values():
        g.zero_()
    roof = {e: roofline_obj(e, B * alg_bytes_per_ray(e, w.n_samples, A, False), kern[e],
                            measured_traffic(e))
            for e in ("render_forward", "render_backward")}
    return A, remarch, roof


def paper_field(torch, ps, wl, w, seed, half=False, mlp_dtype=0):
    """The paper's colour model at a workload's grid sizes: 16 SH coefficients, MLP
    13 -> 32 -> 32 -> 3 (inputs F_s, F_a at the reflected vector, (1 - n.v)^0..5)."""
    import numpy as np
    g = torch.Generator(device="cuda").manual_seed(seed)
    base = gpu_field(torch, ps, wl, w, seed)
    probes = torch.randn((w.P, w.P, w.P, 16, 4), generator=g, device="cuda") * 0.1
    mlp = torch.from_numpy(wl.xavier_uniform_mlp(np.random.default_rng(seed), wl.PAPER_N_IN,
                                                 wl.PAPER_HIDDEN, wl.N_OUT,
                                                 wl.PAPER_LAYERS)).cuda()
    feat = base.feat.half() if half else base.feat
    probes = probes.half() if half else probes
    return ps.Field(base.sdf, feat, probes, mlp, mlp_dtype, ps.sdf_bounds(base.sdf),
                    wl.PAPER_HIDDEN, wl.PAPER_LAYERS)


def time_paper_model(torch, ps, wl, reps):
    """train256 shapes with the paper's colour model (SH at the reflected vector,
    16 coefficients, (1 - n.v)^0..5, MLP 2 x 32): forward + L1 + backward (re-marching,
    one ray per wave), FP32 and FP16 storage with the FP16 MLP."""
    w = wl.WORKLOADS["train256"]
    o, d = wl.workload_rays(w)
    do, dd = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    B = o.shape[0]
    opts = ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels, ps.FLAG_SH_REFLECT | ps.FLAG_FRESNEL_PAPER)
    rgb, aux = torch.empty((B, 3), device="cuda"), torch.empty((B, 4), device="cuda")
    tgt, dL = torch.full((B, 3), 0.5, device="cuda"), torch.empty((B, 3), device="cuda")
    out = {}
    base = gpu_field(torch, ps, wl, w, 0)
    A = shaded_per_ray(torch, ps, w, base.sdf, w.P, do, dd)
    del base
    for label, half, mdt in (("fp32", False, 0), ("fp16", True, 1)):
        fld = paper_field(torch, ps, wl, w, 0, half, mdt)
        grads = {k: torch.zeros(getattr(fld, k).shape, device="cuda") for k in
                 ("sdf", "feat", "probes", "mlp")}
        tf = ev_time(torch, lambda: ps.render_forward(fld, opts, do, dd, rgb, aux), reps)
        ps.l1_loss(rgb, tgt, dL)
        tb = ev_time(torch, lambda: ps.render_backward(fld, opts, do, dd, aux, dL, grads), reps)
        roof = {}
        for e, ms in (("render_forward", tf), ("render_backward", tb)):
            per = B * alg_bytes_model(e, w.n_samples, A, half, 16, False)
            roof[e] = roofline_obj(e, per, ms, measured_traffic(e + "_model", "paper", label))
        out[label] = {"fwd_ms": tf, "bwd_ms": tb, "fwd_bwd_rays_per_s": B / ((tf + tb) * 1e-3),
                      "roofline": roof}
        log(f"paper model {label}: fwd {tf:.3f} ms, bwd {tb:.3f} ms")
        del fld, grads
    out["ratio_fp16_vs_fp32"] = out["fp16"]["fwd_bwd_rays_per_s"] / out["fp32"]["fwd_bwd_rays_per_s"]
    out["shaded_samples_per_ray"] = A
    out["config"] = {"R": w.R, "P": w.P, "sh_coeffs": 16, "mlp": "13-32-32-3", "rays": B,
                     "samples": w.n_samples, "skip_voxels": w.skip_voxels,
                     "flags": "SH_REFLECT | FRESNEL_PAPER"}
    return out


def time_tiled(torch, ps, wl, reps):
    """Sparse 16^3-cell tiles with tri-plane features at 257^3 (T = 16, probes at the
    tile corners, P = 17): forward + L1 + backward over train256's rays, and the plane
    optimiser step."""
    w = wl.WORKLOADS["train256"]
    f = wl.tiled_field(0, 16)
    o, d = wl.workload_rays(w)
    cu = lambda a: torch.from_numpy(a).cuda()
    do, dd = cu(o), cu(d)
    B = o.shape[0]
    fld = ps.Field(cu(f.sdf), cu(f.tiles.planes), cu(f.probes), cu(f.mlp), tiles=cu(f.tiles.index))
    fld.bounds = ps.sdf_bounds(fld.sdf)
    opts = ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels)
    rgb, aux = torch.empty((B, 3), device="cuda"), torch.empty((B, 4), device="cuda")
    tgt, dL = torch.full((B, 3), 0.5, device="cuda"), torch.empty((B, 3), device="cuda")
    grads = {k: torch.zeros(getattr(fld, k).shape, device="cuda") for k in
             ("sdf", "feat", "probes", "mlp")}
    tf = ev_time(torch, lambda: ps.render_forward(fld, opts, do, dd, rgb, aux), reps)
    ps.l1_loss(rgb, tgt, dL)
    tb = ev_time(torch, lambda: ps.render_backward(fld, opts, do, dd, aux, dL, grads), reps)
    pl = fld.feat
    po, m, v = torch.empty_like(pl), torch.zeros_like(pl), torch.zeros_like(pl)
    ts = ev_time(torch, lambda: ps.plane_step(pl, po, grads["feat"], m, v, 1), reps)
    n_tiles = int(f.tiles.planes.shape[0])
    log(f"tiled: fwd {tf:.3f} ms, bwd {tb:.3f} ms, plane step {ts:.3f} ms ({n_tiles} tiles)")
    del grads, po, m, v
    A = shaded_per_ray(torch, ps, w, fld.sdf, f.P, do, dd)
    roof = {}
    for e, ms in (("render_forward", tf), ("render_backward", tb)):
        per = B * alg_bytes_model(e, w.n_samples, A, False, f.n_sh, True)
        roof[e] = roofline_obj(e, per, ms, measured_traffic(e + "_model", "tiled"))
    return {"fwd_ms": tf, "bwd_ms": tb, "plane_step_ms": ts,
            "fwd_bwd_rays_per_s": B / ((tf + tb) * 1e-3), "shaded_samples_per_ray": A,
            "roofline": roof,
            "config": {"T": 16, "R": f.R, "P": f.P, "tiles": n_tiles,
                       "tile_fraction": n_tiles / 16 ** 3, "rays": B, "samples": w.n_samples,
                       "skip_voxels": w.skip_voxels,
                       "feature_bytes": int(f.tiles.planes.nbytes),
                       "dense_feature_bytes": f.R ** 3 * 3 * 4}}


def time_regs(torch, ps, wl, reps):
    """train256's grid step with the paper's remaining SDF regularisers (smoothed SDF
    G(shat), L_sdf, L_normal, the (1 + 5|s|)^-1 weighting) beside the plain one."""
    w = wl.WORKLOADS["train256"]
    f = gpu_field(torch, ps, wl, w, 0)
    p = dict(sdf=f.sdf, feat=f.feat, probes=f.probes, mlp=f.mlp)
    out = {k: torch.empty_like(v) for k, v in p.items()}
    g = {k: torch.zeros_like(v) for k, v in p.items()}
    m = {k: torch.zeros_like(v) for k, v in p.items()}
    v = {k: torch.zeros_like(t) for k, t in p.items()}
    s_in, s_out = torch.empty_like(f.sdf), torch.empty_like(f.sdf)
    ps.smooth_sdf(p["sdf"], s_in)
    work = torch.empty(ps.step_work_bytes(w.R), dtype=torch.uint8, device="cuda")
    plain = ps.StepOpts()
    ext = ps.StepOpts(smooth=True, reg_weight=True, lambda_sdf=0.2, lambda_normal=0.05)
    t_plain = ev_time(torch, lambda: ps.grid_step(p, out, g, m, v, 1, plain), reps)
    t_ext = ev_time(torch, lambda: ps.grid_step(p, out, g, m, v, 1, ext, s_in=s_in, s_out=s_out,
                                                work=work), reps)
    t_smooth = ev_time(torch, lambda: ps.smooth_sdf(p["sdf"], s_out), reps)
    log(f"regularisers: plain step {t_plain:.3f} ms, with Sec. 3.3's SDF terms {t_ext:.3f} ms")
    return {"plain_step_ms": t_plain, "extended_step_ms": t_ext, "smooth_sdf_ms": t_smooth,
            "config": {"R": w.R, "P": w.P, "lambda_sdf": 0.2, "lambda_normal": 0.05,
                       "sigma_voxels": 1.0, "weighted": True}}


def time_realtime(torch, ps, wl, reps):
    """rt512: FP16 grids 512^3 / 128^3, one 1920x1163 view; per-voxel shading of the
    band nodes into an FP16 colour grid, then volume rendering (128 samples, skip 4)."""
    import numpy as np
    w = wl.WORKLOADS["rt512"]
    fld = gpu_field(torch, ps, wl, w, 0, feat_half=True, sdf_half=True)
    fld.bounds = ps.sdf_bounds(fld.sdf)
    band = float(np.float32(wl.RT_BAND_VOXELS * 2.0 / (w.R - 1)))
    cam = torch.from_numpy(wl.fibonacci_cameras(1, w.W, w.H)[0].as_array().astype(np.float32)).cuda()
    lst = torch.empty(w.R ** 3 // 8, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    t_list = ev_time(torch, lambda: ps.voxel_list(fld.sdf, band, lst, cnt), reps)
    n = int(cnt.item())
    assert n <= lst.numel()
    col = torch.zeros((w.R, w.R, w.R, 4), dtype=torch.float16, device="cuda")
    out = torch.empty((w.H, w.W, 3), device="cuda")
    t_shade = ev_time(torch, lambda: ps.voxel_shade(fld, cam, lst, cnt, col), reps)
    opts = ps.RenderOpts(w.n_samples, w.tau, w.skip_voxels)
    t_render = ev_time(torch, lambda: ps.volume_render(fld, opts, col, cam, w.W, w.H, out), reps)
    log(f"real-time: list {t_list:.3f} ms ({n} voxels), shading {t_shade:.3f} ms, "
        f"render {t_render:.3f} ms")
    del lst, col, out
    torch.cuda.empty_cache()
    # algorithmic bytes: the band list reads the FP16 SDF and writes the indices; a band
    # node's shading reads its index, its own and six neighbouring SDF nodes, its features
    # and 8 probe corners (FP16) and writes one FP16 colour; a pixel reads 8 FP16 SDF
    # corners per sample and 8 FP16 colour corners per shaded sample
    o, d = wl.camera_rays(wl.fibonacci_cameras(1, w.W, w.H), w.W, w.H)
    A = shaded_per_ray(torch, ps, w, fld.sdf, w.P, torch.from_numpy(o).cuda(),
                       torch.from_numpy(d).cuda())
    node = 4 + 7 * 2 + 3 * 2 + 8 * w.n_sh * 4 * 2 + 8
    roof = {"voxel_list": roofline_obj("voxel_list", w.R ** 3 * 2.0 + n * 4.0, t_list,
                                       measured_traffic("voxel_list", "realtime")),
            "voxel_shade": roofline_obj("voxel_shade", n * float(node), t_shade,
                                        measured_traffic("voxel_shade", "realtime")),
            "volume_render": roofline_obj("volume_render",
                                          w.W * w.H * (16.0 * w.n_samples + A * 64.0 + 12.0),
                                          t_render, measured_traffic("volume_render", "realtime"))}
    return {"workload": "rt512", "voxel_list_ms": t_list, "voxel_shade_ms": t_shade,
            "volume_render_ms": t_render, "ms_per_frame": t_shade + t_render,
            "shaded_voxels": n, "render_rays_per_s": w.W * w.H / (t_render * 1e-3),
            "shaded_samples_per_pixel": A, "roofline": roof,
            "config": {"R": w.R, "P": w.P, "W": w.W, "H": w.H, "band_voxels": wl.RT_BAND_VOXELS,
                       "samples": w.n_samples, "skip_voxels": w.skip_voxels,
                       "grids": "fp16", "colour_grid": "fp16"}}


def kernel_source_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2412_10084_amd", "csrc", "*"))):
        if p.endswith((".hip", ".h", ".cpp")):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_KERNELS = {
    # the kernels each entry point launches on the benchmark's path (taped training step),
    # by name without template arguments
    "render_backward": ("bwd_ws_clear_kernel", "scan_sums_kernel", "scan_partials_kernel",
                        "scan_offsets_kernel", "tape_walk_kernel", "tape_shade_kernel",
                        "mlp_round_kernel", "mlp_reduce_kernel", "bwd_box_kernel",
                        "probe_reduce_kernel", "render_bwd_kernel"),
    "render_forward": ("may_box_kernel", "render_fwd_kernel"),
    "grid_step": ("zero3_kernel", "bounds_init_kernel", "step_sdf_tiled_kernel",
                  "bounds_decode_kernel", "step_tv3v_kernel", "step_tv4_kernel", "step_mlp_kernel"),
    # the paper colour model's and the tiled fields' kernels
    "render_forward_model": ("model_fwd_kernel",),
    "render_backward_model": ("model_bwd_kernel",),
    "voxel_list": ("zero_count_kernel", "voxel_list_kernel"),
    "voxel_shade": ("voxel_shade_kernel",),
    "volume_render": ("volume_render_kernel",),
}


def kernel_base_name(full: str) -> str:
    """'void psdf::tape_shade_kernel<0>(psdf::RenderArgs, ...)' -> 'tape_shade_kernel'; a
    name the profiler left mangled ('_ZN4psdf17render_fwd_kernelIf...') gives its last
    nested identifier the same way"""
    if full.startswith("_ZN"):
        rest, last = full[3:], ""
        while rest[:1].isdigit():
            n = len(rest) - len(rest.lstrip("0123456789"))
            k = int(rest[:n])
            last, rest = rest[n:n + k], rest[n + k:]
        return last
    name = full.split("(", 1)[0].split("<", 1)[0]
    words = name.rsplit("::", 1)[-1].split()
    return words[-1] if words else ""


def measured_traffic(kernel: str, workload: str = "train256", variant: str = ""):
    """HBM bytes per launch of an entry point from the committed rocprofv3 counter
    summary of a workload (profiles/hbm_traffic_<workload>[_<variant>].txt), or None
    when the kernels changed since the counters were taken (source hash mismatch)."""
    name = f"hbm_traffic_{workload}" + (f"_{variant}" if variant else "") + ".txt"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path) or kernel not in TRAFFIC_KERNELS:
        return None
    total, found, ok = 0.0, 0, False
    for line in open(path):
        if line.startswith("# kernel source hash:"):
            ok = line.split(":", 1)[1].strip() == kernel_source_hash()
        elif line[:1] != "#" and line.strip():
            parts = line.split(None, 4)
            if len(parts) == 5 and kernel_base_name(parts[4]) in TRAFFIC_KERNELS[kernel]:
                total += float(parts[3])
                found += 1
    return total if ok and found else None


def cpu_baseline(wl, w, field, rays, n_rays=16384):
    """FP64 oracle on the host cores: forward + L1 + backward on a ray sample,
    plus one full oracle grid step, scaled to a step over the whole batch."""
    import numpy as np
    import oracle
    o, d = rays
    idx = np.linspace(0, o.shape[0] - 1, n_rays).astype(np.int64)
    of = oracle.field_from(field)
    t0 = time.time()
    ref = oracle.render_forward(of, o[idx], d[idx], w.n_samples, tau=w.tau,
                                skip_voxels=w.skip_voxels)
    _, dL = oracle.l1_loss(ref["rgb"], np.full_like(ref["rgb"], 0.5))
    oracle.render_backward(of, o[idx], d[idx], dL, w.n_samples, tau=w.tau,
                           skip_voxels=w.skip_voxels)
    t_rays = time.time() - t0
    params = dict(sdf=of.sdf, feat=of.feat, probes=of.probes, mlp=of.mlp)
    grads = {k: np.zeros_like(v) for k, v in params.items()}
    n = sum(v.size for v in params.values())
    t0 = time.time()
    oracle.grid_step(params, grads, np.zeros(n), np.zeros(n), 1, oracle.StepOpts())
    t_step = time.time() - t0
    B = o.shape[0]
    t_full = t_rays * B / n_rays + t_step
    shaded = float(ref["n_shaded"].mean())
    cores = oracle.max_threads()
    # the same work on one thread: a quarter of the ray sample and the grid step
    oracle.set_threads(1)
    n1 = n_rays // 4
    t0 = time.time()
    r1 = oracle.render_forward(of, o[idx[:n1]], d[idx[:n1]], w.n_samples, tau=w.tau,
                               skip_voxels=w.skip_voxels)
    _, dL1 = oracle.l1_loss(r1["rgb"], np.full_like(r1["rgb"], 0.5))
    oracle.render_backward(of, o[idx[:n1]], d[idx[:n1]], dL1, w.n_samples, tau=w.tau,
                           skip_voxels=w.skip_voxels)
    t_rays1 = time.time() - t0
    t0 = time.time()
    oracle.grid_step(params, grads, np.zeros(n), np.zeros(n), 1, oracle.StepOpts())
    t_step1 = time.time() - t0
    oracle.set_threads(cores)
    t_full1 = t_rays1 * B / n1 + t_step1
    return dict(value=B / t_full, unit="rays/s", cores=cores, kind="oracle",
                value_1thread=B / t_full1,
                sample=(f"fwd+L1+bwd on {n_rays} evenly spaced rays of the {B}-ray batch "
                        f"({t_rays:.2f} s on {cores} threads) scaled to the batch, plus one full "
                        f"grid step over {n} parameters ({t_step:.2f} s, its Adam loop threaded); "
                        f"value_1thread: {n1} rays ({t_rays1:.2f} s) and the grid step "
                        f"({t_step1:.2f} s) on one thread")), shaded


def copy_bandwidth(torch) -> dict:
    """Rate of a plain 1 GiB device-to-device copy (torch's copy kernel), read + write
    bytes over its event-timed duration: what a streaming kernel reaches on this part,
    beside the published peak the rooflines use."""
    x = torch.empty(1 << 28, device="cuda")
    y = torch.empty_like(x)
    ms = ev_time(torch, lambda: y.copy_(x), 5)
    byts = 2 * x.numel() * 4
    del x, y
    return {"bytes": byts, "ms": ms, "GBps": byts / (ms * 1e-3) / 1e9}


def calib_copy(torch) -> int:
    """Three 1 GiB device copies: what FETCH_SIZE / WRITE_SIZE read for known bytes."""
    x = torch.empty(1 << 28, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return 2 * x.numel() * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="skip mixed precision and inference")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--order", choices=("image", "tile8", "shuffled"), default="image",
                    help="ray order of the timed train256 step (image order by default)")
    ap.add_argument("--only", choices=("mixed512", "iter512", "trace512", "paper", "tiled",
                                       "regs", "realtime"),
                    help="run one secondary workload alone (for profiling) and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the render step is measured on one MI355X (one process, "
                                   "one GPU); --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2412_10084_amd as ps
    import workloads as wl

    ps.lib()
    torch.cuda.set_device(0)
    if args.only:
        reps = max(2, args.steps // 4)
        legs = {"mixed512": lambda: time_fwd_bwd_512(torch, ps, wl, reps, 1),
                "iter512": lambda: time_iter512(torch, ps, wl, args.steps, args.warmup),
                "trace512": lambda: time_inference(torch, ps, wl, reps, 1),
                "paper": lambda: time_paper_model(torch, ps, wl, reps),
                "tiled": lambda: time_tiled(torch, ps, wl, reps),
                "regs": lambda: time_regs(torch, ps, wl, reps),
                "realtime": lambda: time_realtime(torch, ps, wl, reps)}
        res = {"only": args.only, args.only: legs[args.only]()}
        if args.calib_copy:
            res["calib_copy_bytes"] = calib_copy(torch)
        print(json.dumps(res), flush=True)
        return
    w = wl.WORKLOADS["train256"]
    log(f"setting up {w.name}: R={w.R} P={w.P} B={w.rays} N={w.n_samples}")
    st, field, rays = make_state(torch, ps, wl, w, order=args.order)
    ms, kern = time_training(torch, ps, w, st, args.steps, args.warmup, "fp32")
    B = st["B"]
    value = B / (ms * 1e-3)
    A, remarch_ms, roof_render = train256_extras(torch, ps, w, st, kern, max(2, args.steps // 4))
    log(f"shaded samples per ray {A:.3f}; re-marching backward {remarch_ms:.3f} ms")
    del st
    torch.cuda.empty_cache()

    result = {
        "metric": "train rays/s (fwd+bwd) FP32 vs FP16-MFMA at 256^3/64^3; ms per 1080p frame",
        "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "train256", "R": w.R, "P": w.P, "sh_coeffs": w.n_sh,
                   "rays": B, "samples": w.n_samples, "skip_voxels": w.skip_voxels, "ray_order": args.order,
                   "step": "render_forward + l1_loss + render_backward + grid_step"},
        "kernels_ms": kern,
        "fwd_bwd_rays_per_s": B / ((kern["render_forward"] + kern["render_backward"]) * 1e-3),
        "shaded_samples_per_ray": A,
        "render_backward_remarch_ms": remarch_ms,
        "roofline_render": roof_render,
    }

    shaded = A
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, shaded_cpu = cpu_baseline(wl, w, field, rays)
        result["cpu_baseline"] = cb
        result["shaded_samples_per_ray_oracle"] = shaded_cpu
        log(f"cpu baseline: {cb['value']:.4g} rays/s on {cb['cores']} threads, "
            f"{cb['value_1thread']:.4g} on one")

    # roofline of the dominant kernel: algorithmic bytes per launch / launch time
    n_params = w.R ** 3 * 4 + w.P ** 3 * w.n_sh * 4 + 227
    dom = max(kern, key=kern.get)
    per_launch = None
    if dom == "grid_step":
        # read p, g, m, v; write p, m, v, g (zero): 8 x 4 B per parameter
        per_launch = 32.0 * n_params
    elif dom in ("render_forward", "render_backward"):
        per_launch = B * alg_bytes_per_ray(dom, w.n_samples, shaded, False)
    if per_launch is not None:
        result["roofline"] = roofline_obj(dom, per_launch, kern[dom], measured_traffic(dom))
    result["copy_bandwidth"] = copy_bandwidth(torch)
    torch.cuda.empty_cache()

    if not args.no_extras:
        log("mixed precision (fp16 storage, fp16 MFMA MLP) ...")
        stm, _, _ = make_state(torch, ps, wl, w, feat_half=True, mlp_dtype=1)
        msm, kernm = time_training(torch, ps, w, stm, args.steps, args.warmup, "mixed")
        del stm
        torch.cuda.empty_cache()
        result["mixed"] = {"rays_per_s": B / (msm * 1e-3), "ms_per_step": msm, "kernels_ms": kernm,
                           "dtype": "f16 storage, f16 MFMA MLP, f32 accumulate",
                           "speedup_vs_fp32": ms / msm}
        for order in ("tile8", "shuffled"):
            log(f"ray order {order} ...")
            sto, _, _ = make_state(torch, ps, wl, w, order=order)
            mso, kerno = time_training(torch, ps, w, sto, args.steps, args.warmup, order)
            result[f"order_{order}"] = {"rays_per_s": B / (mso * 1e-3), "ms_per_step": mso,
                                        "kernels_ms": kerno}
            del sto
            torch.cuda.empty_cache()
        log("inference (sphere trace, 16 x 1080p) ...")
        result["inference"] = time_inference(torch, ps, wl, max(2, args.steps // 4), 1)
        torch.cuda.empty_cache()
        log("mixed512 (fp32 vs fp16/bf16 MFMA, 512^3 / 128^3, 2^20 rays) ...")
        result["mixed512"] = time_fwd_bwd_512(torch, ps, wl, max(2, args.steps // 4), 1)
        torch.cuda.empty_cache()
        log("iter512 (full iteration, 100 iterations) ...")
        result["iter512"] = time_iter512(torch, ps, wl, 100, 2)
        torch.cuda.empty_cache()
        reps = max(2, args.steps // 4)
        log("paper colour model at train256 shapes ...")
        result["paper_model"] = time_paper_model(torch, ps, wl, reps)
        torch.cuda.empty_cache()
        log("sparse tiles with tri-plane features (T = 16) ...")
        result["tiled"] = time_tiled(torch, ps, wl, reps)
        torch.cuda.empty_cache()
        log("grid step with the smoothed SDF and the remaining regularisers ...")
        result["regularisers"] = time_regs(torch, ps, wl, reps)
        torch.cuda.empty_cache()
        log("real-time render (voxel shading + volume rendering, rt512) ...")
        result["realtime"] = time_realtime(torch, ps, wl, reps)
        torch.cuda.empty_cache()

    if args.calib_copy:
        result["calib_copy_bytes"] = calib_copy(torch)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
