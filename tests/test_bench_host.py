"""Host-side pieces of the benchmark driver (no GPU): the state copy its per-entry
timing pass starts from, the event filter of the timed pass, and the one-GPU rule."""
import json
import subprocess
import sys
from pathlib import Path

import torch

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_clone_state_keeps_aliasing_and_copies_tensors():
    a, b = torch.arange(4.0), torch.ones(2)
    st = {"master": {"sdf": a, "mlp": b}, "spare": {"sdf": a}, "order": [b, 3], "half": None}
    c = bench.clone_state(torch, st)
    assert c["master"]["sdf"] is c["spare"]["sdf"] and c["master"]["mlp"] is c["order"][0]
    assert c["master"]["sdf"] is not a and c["order"][1] == 3 and c["half"] is None
    c["master"]["sdf"].add_(1.0)
    assert torch.equal(a, torch.arange(4.0))


def test_kernel_timer_only_brackets_the_named_entry_points():
    calls = []
    t = bench.KernelTimer(torch, only={"grid_step"})
    t.enabled = True
    t.run("render_forward", lambda: calls.append("f"))  # no events: runs on the CPU
    assert calls == ["f"] and t.pending == []


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus must be 1" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_alg_bytes_and_kernel_names():
    # train256: N = 128, A shaded samples per ray
    assert bench.alg_bytes_per_ray("render_forward", 128, 1.0, False) == 32 * 128 + 1344 + 64
    assert bench.alg_bytes_per_ray("render_backward", 128, 2.0, True) == 32 * 128 + 2 * (720 + 32 + 1376) + 52
    assert bench.kernel_base_name("void psdf::tape_shade_kernel<1>(psdf::RenderArgs, psdf::BwdWs)") == "tape_shade_kernel"
    assert bench.kernel_base_name("psdf::bwd_box_kernel(psdf::RenderArgs, psdf::BwdWs)") == "bwd_box_kernel"
    # names the profiler leaves mangled, and library kernels in anonymous namespaces
    assert bench.kernel_base_name("_ZN4psdf17render_fwd_kernelIfDF16_Li9ELi1EEEvNS_10RenderArgsENS_5BwdWsEi") \
        == "render_fwd_kernel"
    assert bench.kernel_base_name("void at::native::(anonymous namespace)::distribution_kernel<float>(int)") == ""
    # paper model: 16 SH, FP32; dense and tiled features; FP16 halves features and probes
    assert bench.alg_bytes_model("render_forward", 128, 1.0, False, 16, False) == \
        32 * 128 + (96 + 96 + 2048) + 64
    assert bench.alg_bytes_model("render_forward", 64, 2.0, True, 9, True) == \
        32 * 64 + 2 * (96 + 72 + 576) + 64
    assert bench.alg_bytes_model("render_backward", 128, 1.0, False, 16, False) == \
        32 * 128 + (96 + 96 + 2048) + 32 + (96 + 96 + 2048) + 52
    r = bench.roofline_obj("render_forward", 8e9, 1.0, None)
    assert abs(r["frac"] - 1.0) < 1e-12 and r["achieved"] == 8000.0
