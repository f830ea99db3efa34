"""Host-side parts of bench.py: the algorithmic byte counts behind every HBM
roofline figure it reports (one eval = one primitive-view pair; each input
read once, each output written once), pinned to per-eval values worked out
by hand from the layouts (lobe parameters 44 B in FP32, 22 B in bf16;
colour and mean 24 B per primitive; 12 B per rgb or upstream-gradient
triple; 48 SH coefficients 192 B), the comment-blind source hash that ties
committed counters to kernel sources, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

import bench

N = 1000  # per-eval figures are exact multiples of N


def per_eval(total, n, v):
    return total / (n * v)


def test_one_camera_bytes():
    # K = 8: params 8 x 44 + 24 = 376 read, 376 of gradients written, 12 + 12 of view data
    assert per_eval(bench.algorithmic_bytes(N, 8, 1), N, 1) == 776
    sep = bench.algorithmic_bytes(N, 8, 1, bwd=False) + bench.algorithmic_bytes(N, 8, 1, rgb_out=False)
    assert per_eval(sep, N, 1) == 1152                       # separate forward and backward
    assert per_eval(bench.sh_bytes(N, 1), N, 1) == 432       # SH: 204 read, 204 written, 24
    sep_sh = bench.sh_bytes(N, 1, bwd=False) + bench.sh_bytes(N, 1, fwd=False)
    assert per_eval(sep_sh, N, 1) == 636


def test_headline_bytes():
    # 3 M x 16 cameras: the per-primitive bytes are shared by the 16 views
    assert per_eval(bench.algorithmic_bytes(N, 8, 16), N, 16) == 71
    assert bench.algorithmic_bytes(3_000_000, 8, 16) == 3_408_000_000
    sep = bench.algorithmic_bytes(N, 8, 16, bwd=False) + bench.algorithmic_bytes(N, 8, 16, rgb_out=False)
    assert per_eval(sep, N, 16) == 94.5
    # sixteen one-view launches, all but the first accumulating (read-modify-write)
    single = bench.algorithmic_bytes(N, 8, 1) + 15 * bench.algorithmic_bytes(N, 8, 1, accumulate=True)
    assert per_eval(single, N, 16) == 1128.5
    assert per_eval(bench.sh_bytes(N, 16), N, 16) == 49.5
    assert bench.sh_bytes(3_000_000, 16) == 2_376_000_000


def test_bf16_bytes():
    # K = 16, 8 cameras: bf16 lobe parameters read (16 x 22 + 24), FP32 gradients written
    bf = bench.algorithmic_bytes(N, 16, 8, lobe_bytes=bench.LOBE_BYTES_BF16)
    assert per_eval(bf, N, 8) == 162
    assert per_eval(bench.algorithmic_bytes(N, 16, 8), N, 8) == 206


def test_source_hash_ignores_comments_only():
    code = "int f(int x) {\n  return x + 1;  // one more\n}\n"
    commented = "/* header\n   text */\n" + code.replace("// one more", "// a different note") + "\n\n"
    assert bench._code_only(code) == bench._code_only(commented)
    assert bench._code_only(code) != bench._code_only(code.replace("x + 1", "x + 2"))
    h = bench.kernel_source_hash(bench.APPEARANCE_SOURCES)
    assert len(h) == 16 and h == bench.kernel_source_hash(bench.APPEARANCE_SOURCES)


def test_committed_counters_match_their_sources():
    """The counters bench.py prices the headline and compositing rooflines
    with were taken on the kernel sources as committed (else bench.py falls
    back to the HBM roofline with unknown traffic)."""
    assert bench.measured_counters("nasg_fused_k8_v16_n3000000_exact") is not None
    assert bench.measured_counters("raster_render_bwd_geom_n3000000_1920x1080",
                                   bench.RASTER_SOURCES) is not None
    for key in ("nasg_fused_k8_v1_n1048576_exact", "nasg_fused_k16_v8_n6000000_exact_bf16",
                "nasg_fused_k8_v16_n3000000_exact_angles", "nasg_batch_uneven32_exact"):
        assert bench.measured_counters(key) is not None, key


def test_counters_roofline_bounds():
    """The single-camera line stays on the HBM roof with its measured traffic;
    the VALU-bound lines (bf16 K = 16, the persistent batch) report the issue
    rate with the HBM figures beside; unknown counters give the HBM roof with
    unknown traffic."""
    ab = bench.algorithmic_bytes(1 << 20, 8, 1)
    r = bench.counters_roofline("nasg_fused_k8_v1_n1048576_exact", 0.25, ab, 1 << 20, alu=False)
    assert r["bound"] == "hbm" and r["traffic"] > ab and r["achieved"] == round(ab / 0.25 / 1e6, 1)
    r = bench.counters_roofline("nasg_batch_uneven32_exact", 13.0, 25_156_165_456, 171_865_438, alu=True)
    assert r["bound"] == "alu" and 0 < r["frac"] < 1 and r["hbm"]["algorithmic_bytes_per_launch"] > 0
    assert r["profiled_launch"] == {"tile_iters": 8, "blocks_per_cu": 4}
    r = bench.counters_roofline("no_such_key", 1.0, 1000, 10, alu=True)
    assert r["bound"] == "hbm" and r["traffic"] is None


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
