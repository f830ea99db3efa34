"""Host-side parts of bench.py: the algorithmic byte counts behind every HBM
roofline figure it reports (one eval = one primitive-view pair; each input
read once, each output written once), pinned to per-eval values worked out
by hand from the layouts (lobe parameters 44 B in FP32, 22 B in bf16;
colour and mean 24 B per primitive; 12 B per rgb or upstream-gradient
triple; 48 SH coefficients 192 B), the comment-blind source hash that ties
committed counters to kernel sources, and the one-GPU guard."""
import json
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


def test_source_hash_covers_tuning_choices_not_timings():
    """The tuning table enters the hash through its choices only: the timings
    recorded beside them change from box to box without changing a launch."""
    table = {"arch": "gfx950", "entries": {"1/8/16/0": {"lanes": 4, "views_per_lane": 4,
                                                          "block": 128, "bcast": 0,
                                                          "ms": 2.18, "n": 3000000}},
             "batch": {"tile_iters": 8, "blocks_per_cu": 4, "ms": 10.7, "scenes": 32}}
    base = bench._choices_only(json.dumps(table))
    timed = json.loads(json.dumps(table))
    timed["entries"]["1/8/16/0"]["ms"] = 2.31
    timed["batch"]["ms"] = 11.2
    assert bench._choices_only(json.dumps(timed)) == base
    chosen = json.loads(json.dumps(table))
    chosen["entries"]["1/8/16/0"]["lanes"] = 8
    assert bench._choices_only(json.dumps(chosen)) != base
    chosen = json.loads(json.dumps(table))
    chosen["batch"]["tile_iters"] = 16
    assert bench._choices_only(json.dumps(chosen)) != base


def test_counters_are_used_only_on_their_sources(tmp_path, monkeypatch):
    """Committed counters price a roofline only while the kernel sources they
    were taken on are unchanged (comment edits aside); otherwise bench.py
    reports the HBM roofline with unknown traffic."""
    import json
    h = bench.kernel_source_hash(bench.APPEARANCE_SOURCES)
    prof = tmp_path / "profiles"
    prof.mkdir()
    ent = {"source_hash": h, "bytes_per_launch": 3_500_000_000,
           "valu_wave_instructions_per_launch": 1_000_000_000, "clock_GHz": 2.1}
    (prof / "traffic.json").write_text(json.dumps({"cur": ent, "old": dict(ent, source_hash="0" * 16)}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda files=None: h)
    assert bench.measured_counters("cur") is not None
    assert bench.measured_counters("old") is None
    assert bench.measured_counters("missing") is None


def test_roofline_object():
    """frac is the algorithmic bytes against the 8 TB/s peak; the VALU issue
    rate (from counters) and the algorithmic operation rate sit beside it;
    unknown counters give unknown traffic."""
    ab = bench.algorithmic_bytes(3_000_000, 8, 16)
    ops = bench.algorithmic_ops_per_eval(8, 16)
    r = bench.roofline("no_such_key", 2.0, ab, 48_000_000, ops, ceiling=5000.0)
    assert r["bound"] == "hbm" and r["traffic"] is None
    assert r["achieved"] == round(ab / 2.0 / 1e6, 1) and r["frac"] == round(ab / 2.0 / 1e6 / 8000, 4)
    assert r["bytes_per_eval"] == 71.0 and r["frac_of_stream_ceiling"] == round(ab / 2e6 / 5000, 4)
    t = ops * 48_000_000 / 2e-3 / 1e12
    assert r["algorithmic_ops"]["frac"] == round(t / 39.3216, 4)
    assert "valu_issue" not in r and r["binding"] == "hbm"


def test_algorithmic_ops_per_eval():
    """Per primitive-view: K x 72 operations per lobe-view (26 value, 46
    gradient), K x (frame 23 + normaliser 62 EXACT / 13 APPROX + write-out 41)
    per lobe shared by the V views, 22 per view (direction, c0 and mean
    gradients); counted from the formulas of the path."""
    assert bench.algorithmic_ops_per_eval(8, 16, "exact") == 8 * 72 + 8 * 126 / 16 + 22 == 661
    assert bench.algorithmic_ops_per_eval(8, 16, "approx") == 8 * 72 + 8 * 77 / 16 + 22
    assert bench.algorithmic_ops_per_eval(8, 1, "exact") == 8 * 72 + 8 * 126 + 22


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
