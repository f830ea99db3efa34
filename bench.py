#!/usr/bin/env python3
"""Benchmark of the NASGabor appearance path on one MI355X.

Headline workload: NASGabor K = 8, fused forward+backward, 3 M primitives x
16 cameras in one launch (FP32 storage, EXACT normaliser), synthetic inputs
already resident in HBM. One step = one fused launch over the whole batch.
Prints one JSON line. Algorithmic bytes per launch: every input read once
(K x 44 B of float32 lobe parameters + 24 B of diffuse colour and mean per
primitive, 12 B of upstream gradient per primitive-view) and every output
written once (12 B of colour per primitive-view, K x 44 + 24 B of float32
gradients per primitive).

    python bench.py [--steps K] [--warmup W] [--n N] [--norm exact|approx]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "primitive-view evals/s fwd+bwd (G/s) + % HBM peak, NASGabor K=8 vs SH deg 3"
HBM_PEAK_GBS = 8000.0
LOBE_BYTES_F32 = 44          # quat 16 + shape 16 + rgbw 12
LOBE_BYTES_BF16 = 22
PRIM_BYTES = 24              # c0 12 + means 12
VIEW_BYTES = 12              # one rgb or grad_rgb triple


def algorithmic_bytes(n, k, v, *, fwd=True, bwd=True, rgb_out=True, lobe_bytes=LOBE_BYTES_F32,
                      accumulate=False):
    """HBM bytes one launch must move at minimum (each input read once, each
    output written once)."""
    rd = n * (k * lobe_bytes + PRIM_BYTES)
    b = rd
    if bwd:
        b += n * v * VIEW_BYTES                  # grad_rgb
        b += n * (k * 44 + PRIM_BYTES)           # f32 gradients of every input
        if accumulate:
            b += n * (k * 44 + PRIM_BYTES)       # read-modify-write
    if fwd and rgb_out:
        b += n * v * VIEW_BYTES                  # rgb
    return b


def sh_bytes(n, v, *, fwd=True, bwd=True):
    b = n * (192 + 12)                           # 48 coefficients + mean
    if bwd:
        b += n * v * VIEW_BYTES + n * (192 + 12)
    if fwd:
        b += n * v * VIEW_BYTES
    return b


# the sources (and launch table) each profiled kernel is built from
APPEARANCE_SOURCES = ("capi.hip", "nasg_device.hpp", "nasg_kernels.hip", "nasg_launch.hpp",
                      "nasg_skeleton.hpp", "../tuning_gfx950.json")
RASTER_SOURCES = ("capi.hip", "nasg_device.hpp", "raster.hpp", "raster_kernels.hip")
SH_SOURCES = ("capi.hip", "nasg_device.hpp", "nasg_launch.hpp", "sh3_kernels.hip",
              "../tuning_gfx950.json")


def _code_only(text: str) -> str:
    """Source text without comments and blank lines: profiles stay valid
    across edits that touch only comments."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def _choices_only(text: str) -> str:
    """A tuning table reduced to its choices (lane mappings, block sizes, batch
    tile): the timings recorded beside them do not change the launches."""
    def strip(x):
        if isinstance(x, dict):
            return {k: strip(v) for k, v in x.items() if k not in ("ms", "n", "sweep_ms")}
        return x
    return json.dumps(strip(json.loads(text)), sort_keys=True)


def kernel_source_hash(files=APPEARANCE_SOURCES):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_09794_amd", "csrc")
    for f in files:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        body = _choices_only(text) if f.endswith(".json") else _code_only(text)
        h.update(os.path.basename(f).encode() + body.encode())
    return h.hexdigest()[:16]


VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock (non-packed issue)


def measured_counters(key, files=APPEARANCE_SOURCES):
    """Per-launch counter figures (calibrated HBM bytes, VALU wave instructions)
    from the committed rocprofv3 summary, or None if missing or taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(key)
    if not ent or ent.get("source_hash") != kernel_source_hash(files):
        return None
    return ent


# Algorithmic arithmetic of the path: floating-point operations its formulas
# need (an add, multiply, fused multiply-add, reciprocal, square root or
# transcendental counts 1; no extra precision, no index or conversion work).
OPS_LOBE_VIEW = 26 + 46      # value and colour; backward partials and their sums
OPS_LOBE = {"exact": 23 + 62 + 41, "approx": 23 + 13 + 41}   # frame, normaliser, write-out
OPS_VIEW = 22                # direction, c0 and mean gradients per primitive-view


def algorithmic_ops_per_eval(k, v, norm="exact"):
    """Operations per primitive-view of the fused forward+backward."""
    return k * OPS_LOBE_VIEW + k * OPS_LOBE[norm] / v + OPS_VIEW


def roofline(key, ms, ab, evals, ops_per_eval=None, files=APPEARANCE_SOURCES, kernel=None,
             ceiling=None):
    """Roofline object of one launch: the algorithmic bytes against the HBM peak
    (`frac`), the counter-measured traffic when the committed counters match the
    kernel sources, the VALU issue rate from those counters and the algorithmic
    operation rate against the non-packed issue peak, and which roof binds."""
    ach = ab / ms / 1e6
    r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
         "algorithmic_bytes_per_launch": int(ab), "bytes_per_eval": round(ab / evals, 2)}
    if kernel:
        r["kernel"] = kernel
    if ceiling:
        r["stream_ceiling_GB_s"] = ceiling
        r["frac_of_stream_ceiling"] = round(ach / ceiling, 4)
    peak = VALU_PEAK_LANE_OPS / 1e12
    fracs = {"hbm": ach / HBM_PEAK_GBS}
    if ops_per_eval is not None:
        t = ops_per_eval * evals / (ms * 1e-3) / 1e12
        r["algorithmic_ops"] = {"ops_per_eval": round(ops_per_eval, 1), "achieved": round(t, 2),
                                "peak": round(peak, 2), "unit": "T ops/s", "frac": round(t / peak, 4)}
    c = measured_counters(key, files)
    if c is not None:
        r["traffic"] = c["bytes_per_launch"]
        lane = c["valu_wave_instructions_per_launch"] * 64
        t = lane / (ms * 1e-3) / 1e12
        r["valu_issue"] = {"lane_instructions_per_eval": round(lane / evals, 1), "achieved": round(t, 2),
                           "peak": round(peak, 2), "unit": "T VALU lane-instructions/s",
                           "frac": round(t / peak, 4)}
        if "clock_GHz" in c:
            r["valu_issue"]["profiled_clock_GHz"] = c["clock_GHz"]
        if "profiled_launch" in c:
            r["profiled_launch"] = c["profiled_launch"]
        fracs["valu"] = t / peak
    r["binding"] = max(fracs, key=fracs.get)
    return r


def parity_report(got, ref, scale):
    """max / p99 / median of the scaled error (the gate, <= 1e-5) and of the
    plain relative error per output and gradient."""
    from oracle import metrics as M
    return {k: M.report(got[k], ref[k], scale[k]) for k in got}


# ----------------------------------------------------------------- CPU oracle

_CPU_W = None   # workload shared with forked oracle workers


def _oracle_chunk(args):
    import oracle.nasg_ref as R
    import workloads as W
    lo, hi, norm = args
    w = W.take_primitives(_CPU_W, np.arange(lo, hi))
    R.forward_backward(w.quat, w.shape, w.rgbw, w.c0, w.grad_rgb, norm, means=w.means, cams=w.cams)
    return w.n * w.v


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), else the machine type."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_cores():
    """Worker processes for the CPU leg: the cores this process may run on,
    capped at the CPU share the host grants a one-GPU job (OMP_NUM_THREADS when
    set: the GPU hosts export their share there; the affinity mask there shows
    the whole machine)."""
    aff = len(os.sched_getaffinity(0))
    share = os.environ.get("OMP_NUM_THREADS", "")
    cap = int(share) if share.isdigit() and int(share) > 0 else aff
    return max(1, min(aff, cap)), aff


def cpu_baseline(w_full, prims=1_000_000, chunk=1024, norm_code=0):
    """Time the FP64 oracle (as written) on the first `prims` primitives of the
    workload, split over the host's cores (forked workers share the arrays)."""
    global _CPU_W
    _CPU_W = w_full
    cores, aff = host_cores()
    n = min(prims, w_full.n)
    ranges = [(i, min(i + chunk, n), norm_code) for i in range(0, n, chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_chunk, ranges[:cores])                   # warm the workers
        t0 = time.perf_counter()
        evals = sum(pool.map(_oracle_chunk, ranges, chunksize=1))
        dt = time.perf_counter() - t0
    _CPU_W = None
    return {"value": evals / dt / 1e9, "unit": "G evals/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 NumPy oracle, fused fwd+bwd on the first {n} of {w_full.n} primitives x "
                      f"{w_full.v} views (K={w_full.k}), {len(ranges)} chunks of {chunk} over "
                      f"{cores} processes, {dt:.1f} s wall",
            "cpu": cpu_model(), "affinity_cores": aff}


# ----------------------------------------------------------------------- GPU

def upload(w, device="cuda"):
    import torch
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
    if w.dtype == "bf16":
        lob = {k: torch.from_numpy(getattr(w, k + "_bits").view(np.int16)).to(device).view(torch.bfloat16)
               for k in ("quat", "shape", "rgbw")}
    else:
        lob = {k: t(getattr(w, k)) for k in ("quat", "shape", "rgbw")}
    return dict(lob, c0=t(w.c0), means=t(w.means), cams=t(w.cams), grad_rgb=t(w.grad_rgb),
                sh=t(w.sh))


def time_launches(fn, steps, warmup, settle=0.25):
    """Mean ms per call of fn() over `steps` calls, HIP events on the current
    stream (the stream the kernels are launched on). Before the `warmup` calls,
    fn() runs untimed for `settle` seconds: the GPU leaves its idle clock over
    the first tens of milliseconds of load (a kernel trace shows the first
    launches of a fresh run up to 25 % slower than the steady state), and every
    measurement here follows host work that lets it idle."""
    import torch
    if settle > 0:
        t0 = time.perf_counter()
        while True:
            fn()
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= settle:
                break
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def copy_ceiling(steps, mib=1024):
    """The runtime's own device-to-device copy of `mib` MiB (each byte read once
    and written once), kept beside the hand-written streaming kernels."""
    import torch
    src = torch.empty(mib << 18, device="cuda")
    dst = torch.empty_like(src)
    ms = time_launches(lambda: dst.copy_(src), steps, 1)
    cb = 2 * src.numel() * 4
    del src, dst
    return {"ms": round(ms, 4), "bytes": cb, "GB_s": round(cb / ms / 1e6, 1),
            "frac_of_peak": round(cb / ms / 1e6 / HBM_PEAK_GBS, 4)}


STREAM_GRID = (256, 512, 1024, 2048, 4096, 8192)     # 256-thread blocks (1..32 per CU)
STREAM_UNROLL = (1, 2, 4, 8)


def stream_ceiling(gib=2, reps=3):
    """Achievable HBM rate from the library's hand-written streaming kernels
    (16 B per lane): read-only, write-only and copy of `gib` GiB buffers (far
    beyond the 256 MB of last-level cache), swept over grid size, accesses in
    flight per thread and nontemporal hints; each point is the mean of `reps`
    launches after one warm-up. Returns the best point per mode and the sweep."""
    import ctypes as C

    import torch

    from paper_2606_09794_amd import _lib as L
    nbytes = gib << 30
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib = L.lib()
    out, sweep = {}, {}
    settle = 0.25      # once, before the first point: the sweep itself keeps the GPU busy
    for mode, name, moved in ((L.STREAM_READ, "read", nbytes), (L.STREAM_WRITE, "write", nbytes),
                              (L.STREAM_COPY, "copy", 2 * nbytes)):
        best = None
        for grid in STREAM_GRID:
            for unroll in STREAM_UNROLL:
                for nt in (0, 1):
                    run = lambda: L.check(lib.nasg_hbm_stream(  # noqa: E731
                        mode, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, grid,
                        unroll, nt, stream), "nasg_hbm_stream")
                    ms = time_launches(run, reps, 1, settle=settle)
                    settle = 0.0
                    gbs = moved / ms / 1e6
                    sweep[f"{name}_g{grid}_u{unroll}_nt{nt}"] = round(gbs, 1)
                    if best is None or gbs > best["GB_s"]:
                        best = {"GB_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                                "ms": round(ms, 4), "bytes": moved, "blocks": grid,
                                "unroll": unroll, "nontemporal": nt}
        out[name] = best
    del src, dst
    torch.cuda.empty_cache()
    return out, sweep


def _sampled(w, got, norm, n_sample=256, seed=0, orig=False):
    """Error of device results `got` (full tensors) on sampled primitives (all
    their views and lobes) against the oracle on the stored values: max / p99 /
    median of the scaled error (the gate) and of the plain relative error per
    output and gradient. With orig=True the oracle takes the float32 values
    before bf16 rounding instead (the quantisation cost: scaled-error summary
    and the fraction of elements within 2e-2)."""
    import workloads as W
    from oracle import metrics as M
    from oracle import nasg_paper as Pp
    from oracle import nasg_ref as R
    idx = np.sort(np.random.default_rng(seed).choice(w.n, size=min(n_sample, w.n), replace=False))
    sub = W.take_primitives(w, idx)
    src = sub.orig if orig else {"quat": sub.quat, "shape": sub.shape, "rgbw": sub.rgbw}
    if w.family != "nasgabor":
        from oracle import families as F
        code = {"nasg": F.NASG, "sg": F.SG, "sb": F.SB, "sc": F.SC, "asg": F.ASG}[w.family]
        ref, scale = F.forward_backward(code, src["quat"], src["shape"], src["rgbw"], sub.c0,
                                        sub.grad_rgb, means=sub.means, cams=sub.cams, param=w.param)
    else:
        fb = Pp.forward_backward if w.param == "angles" else R.forward_backward
        ref, scale = fb(src["quat"], src["shape"], src["rgbw"], sub.c0, sub.grad_rgb,
                        R.NORM_EXACT if norm == "exact" else R.NORM_APPROX,
                        means=sub.means, cams=sub.cams)
    ref["geom"], scale["geom"] = ref.pop("means"), scale.pop("means")
    sel = {"rgb": lambda t: t[:, idx], "quat": lambda t: t[:, idx], "shape": lambda t: t[:, idx],
           "rgbw": lambda t: t[:, :, idx], "c0": lambda t: t[idx], "geom": lambda t: t[idx]}
    out = {}
    for k, f in sel.items():
        y = f(got[k]).cpu().numpy()
        if orig:
            e = M.scaled_error(y, ref[k], scale[k])
            out[k] = dict(M.summarize(e), frac_within_2e_2=float((e <= 2e-2).mean()))
        else:
            out[k] = M.report(y, ref[k], scale[k])
    return out


def worst_scaled(rep):
    """The largest scaled error over the outputs of a parity report."""
    return max(v["scaled"]["max"] for v in rep.values())


def profile_other(args, log):
    """Counter-collection mode of the single-camera, bf16 K=16, paper-params and
    uneven-batch workloads: only the launch their bench line times (the
    persistent batch with the tuner's cached tile, or --tile-iters /
    --blocks-per-cu), --steps times."""
    import torch

    import paper_2606_09794_amd as P
    from paper_2606_09794_amd import autotune
    import workloads as W
    if args.workload in ("single-camera", "bf16-k16", "paper-params"):
        param = "angles" if args.workload == "paper-params" else "quat"
        if args.workload == "single-camera":
            w = W.config1(n=args.n)
        elif args.workload == "bf16-k16":
            w = W.config3(n=args.n)
        else:
            w = W.draw_workload(7, args.n, 8, args.views, with_sh=False, param="angles")
        d = upload(w)
        g = P.nasg_grad_buffers(w.k, w.n, "cuda")
        rgb = torch.empty((w.v, w.n, 3), device="cuda")
        for _ in range(args.steps):
            P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], means=d["means"],
                            cams=d["cams"], norm=args.norm, grads=g, rgb_out=rgb, param=param)
        lb = LOBE_BYTES_BF16 if args.workload == "bf16-k16" else LOBE_BYTES_F32
        info = {"n": w.n, "k": w.k, "v": w.v, "evals": w.n * w.v,
                "algorithmic_bytes_per_launch": algorithmic_bytes(w.n, w.k, w.v, lobe_bytes=lb)}
    elif args.workload == "uneven-batch":
        scenes = W.config4()
        dev = []
        for sc in scenes:
            dd = upload(sc.workload)
            dd["grads"] = P.nasg_grad_buffers(sc.workload.k, sc.workload.n, "cuda")
            dd["rgb"] = torch.empty((sc.workload.v, sc.workload.n, 3), device="cuda")
            dev.append(dd)
        ti, bpc = autotune.batch_defaults()
        ti = ti if args.tile_iters is None else args.tile_iters
        bpc = bpc if args.blocks_per_cu is None else args.blocks_per_cu
        plan = P.NasgBatchPlan(dev, norm=args.norm, tile_iters=ti, blocks_per_cu=bpc)
        for _ in range(args.steps):
            plan.run()
        info = {"scenes": len(scenes), "evals": sum(s.workload.n * s.workload.v for s in scenes),
                "tile_iters": ti, "blocks_per_cu": bpc,
                "algorithmic_bytes_per_launch": sum(algorithmic_bytes(s.workload.n, s.workload.k,
                                                                      s.workload.v) for s in scenes)}
    else:
        raise SystemExit("--profile: headline, single-camera, bf16-k16, paper-params or uneven-batch")
    torch.cuda.synchronize()
    print(json.dumps(dict(profile=True, workload=args.workload, launches=args.steps,
                          source_hash=kernel_source_hash(), **info)), flush=True)


def measure_single_camera(norm, steps, warmup, log, n=1 << 20, ceiling=None):
    """K = 8, 1 M primitives x one camera, fused forward+backward (FP32
    storage), with the degree-3 SH fused launch on the same inputs."""
    import torch

    import paper_2606_09794_amd as P
    import workloads as W
    t0 = time.perf_counter()
    w = W.config1(n=n)
    log(f"single camera: generated N={w.n} K={w.k} in {time.perf_counter() - t0:.1f}s")
    d = upload(w)
    n, k, v = w.n, w.k, w.v
    g = P.nasg_grad_buffers(k, n, "cuda")
    rgb = torch.empty((v, n, 3), device="cuda")
    fn = lambda: P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"],  # noqa: E731
                                 means=d["means"], cams=d["cams"], norm=norm, grads=g, rgb_out=rgb)
    ms = time_launches(fn, steps, warmup)
    ab = algorithmic_bytes(n, k, v)
    gsh = {"sh": torch.empty_like(d["sh"]), "geom": torch.empty((n, 3), device="cuda")}
    rsh = torch.empty_like(rgb)
    msh = time_launches(lambda: P.sh3_eval_bwd(d["sh"], d["grad_rgb"], means=d["means"], cams=d["cams"],
                                               grads=gsh, rgb_out=rsh), steps, warmup)
    fn()
    torch.cuda.synchronize()
    par = _sampled(w, dict(g, rgb=rgb), norm)
    log(f"single camera: {ms:.4f} ms, parity worst scaled {worst_scaled(par):.2e}")
    sb = sh_bytes(n, v)
    return {"workload": f"NASGabor K={k} fused fwd+bwd, {n} primitives x 1 camera, FP32, {norm} normaliser",
            "ms": round(ms, 4), "G_evals_s": round(n * v / ms / 1e6, 4),
            "roofline": roofline(f"nasg_fused_k{k}_v{v}_n{n}_{norm}", ms, ab, n * v,
                                 algorithmic_ops_per_eval(k, v, norm), ceiling=ceiling,
                                 kernel="nasg_kernel (fused forward+backward, one view)"),
            "sh3_fused": {"ms": round(msh, 4), "G_evals_s": round(n * v / msh / 1e6, 4),
                          "GB_s": round(sb / msh / 1e6, 1), "hbm_frac": round(sb / msh / 1e6 / HBM_PEAK_GBS, 4)},
            "parity_sampled": par}


def measure_bf16_k16(norm, steps, warmup, log, n=6_000_000, ceiling=None):
    """K = 16, 6 M primitives x 8 cameras with bf16 lobe storage, beside the
    same values in FP32 storage; parity against the dequantised values (the
    gate) and the quantisation cost against the FP32 values before rounding."""
    import torch

    import paper_2606_09794_amd as P
    import workloads as W
    t0 = time.perf_counter()
    w = W.config3(n=n)
    log(f"bf16 K=16: generated N={w.n} K={w.k} V={w.v} in {time.perf_counter() - t0:.1f}s")
    d = upload(w)
    n, k, v = w.n, w.k, w.v
    g = P.nasg_grad_buffers(k, n, "cuda")
    rgb = torch.empty((v, n, 3), device="cuda")
    fn = lambda dd: P.nasg_eval_bwd(dd["quat"], dd["shape"], dd["rgbw"], dd["c0"], dd["grad_rgb"],  # noqa: E731
                                    means=dd["means"], cams=dd["cams"], norm=norm, grads=g, rgb_out=rgb)
    ms = time_launches(lambda: fn(d), steps, warmup)
    fn(d)
    torch.cuda.synchronize()
    par = _sampled(w, dict(g, rgb=rgb), norm)
    qcost = _sampled(w, dict(g, rgb=rgb), norm, orig=True)
    d32 = dict(d, quat=d["quat"].float(), shape=d["shape"].float(), rgbw=d["rgbw"].float())
    ms32 = time_launches(lambda: fn(d32), steps, warmup)
    fn(d32)
    torch.cuda.synchronize()
    par32 = _sampled(w, dict(g, rgb=rgb), norm)
    log(f"bf16 K=16: {ms:.3f} ms (fp32 storage {ms32:.3f} ms), parity worst scaled "
        f"{worst_scaled(par):.2e}")
    ab = algorithmic_bytes(n, k, v, lobe_bytes=LOBE_BYTES_BF16)
    ab32 = algorithmic_bytes(n, k, v)
    return {"workload": f"NASGabor K={k} fused fwd+bwd, {n} primitives x {v} cameras, lobe parameters "
                        f"stored in bf16, {norm} normaliser",
            "ms": round(ms, 4), "G_evals_s": round(n * v / ms / 1e6, 4),
            "roofline": roofline(f"nasg_fused_k{k}_v{v}_n{n}_{norm}_bf16", ms, ab, n * v,
                                 algorithmic_ops_per_eval(k, v, norm), ceiling=ceiling,
                                 kernel="nasg_kernel (fused forward+backward, bf16 lobes)"),
            "fp32_storage_same_values": {
                "ms": round(ms32, 4), "G_evals_s": round(n * v / ms32 / 1e6, 4),
                "hbm_frac": round(ab32 / ms32 / 1e6 / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_launch": ab32, "parity_sampled": par32},
            "parity_sampled": par,
            "bf16_quantisation_cost_vs_fp32_values": qcost}


def measure_uneven_batch(norm, steps, warmup, log, ceiling=None, tune=True, n_scenes=32,
                         scale=1.0, parity_every=4):
    """`n_scenes` scenes (N log-uniform in [5e4, 2e6] times `scale`, K in
    {4, 8, 16}, V in {1, 4, 16}) in one persistent fused launch with the
    tuner's (tile passes, blocks per CU), its hipGraph replay and per-scene
    launches; sampled parity on every `parity_every`-th scene."""
    import torch

    import paper_2606_09794_amd as P
    import workloads as W
    from paper_2606_09794_amd import autotune
    t0 = time.perf_counter()
    scenes = W.config4(n_scenes=n_scenes, scale=scale)
    tag = f"uneven batch ({len(scenes)} scenes)"
    log(f"{tag}: generated {len(scenes)} scenes, {sum(s.workload.n for s in scenes)} primitives "
        f"in {time.perf_counter() - t0:.1f}s")
    dev = []
    for sc in scenes:
        w = sc.workload
        dd = upload(w)
        dd["grads"] = P.nasg_grad_buffers(w.k, w.n, "cuda")
        dd["rgb"] = torch.empty((w.v, w.n, 3), device="cuda")
        dev.append(dd)
    evals = sum(sc.workload.n * sc.workload.v for sc in scenes)
    ab = sum(algorithmic_bytes(sc.workload.n, sc.workload.k, sc.workload.v) for sc in scenes)
    ops = sum(algorithmic_ops_per_eval(sc.workload.k, sc.workload.v, norm) * sc.workload.n * sc.workload.v
              for sc in scenes) / evals
    if tune:
        choice = autotune.tune_batch(dev, norm=norm, save=False, verbose=False)
        ti, bpc, sweep = choice["tile_iters"], choice["blocks_per_cu"], choice["sweep_ms"]
    else:
        ti, bpc = autotune.batch_defaults()
        sweep = None
    plan = P.NasgBatchPlan(dev, norm=norm, tile_iters=ti, blocks_per_cu=bpc)
    ms = time_launches(plan.run, steps, warmup)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        plan.run()
    ms_graph = time_launches(graph.replay, steps, warmup)

    def per_scene():
        for dd in dev:
            P.nasg_eval_bwd(dd["quat"], dd["shape"], dd["rgbw"], dd["c0"], dd["grad_rgb"],
                            means=dd["means"], cams=dd["cams"], norm=norm, grads=dd["grads"],
                            rgb_out=dd["rgb"])
    ms_sep = time_launches(per_scene, steps, warmup)
    graph.replay()
    torch.cuda.synchronize()
    worst = {}
    for sc, dd in zip(scenes[::parity_every], dev[::parity_every]):
        rep = _sampled(sc.workload, dict(dd["grads"], rgb=dd["rgb"]), norm, n_sample=64)
        for kk, vv in rep.items():
            cur = worst.get(kk)
            if cur is None or vv["scaled"]["max"] > cur["scaled"]["max"]:
                worst[kk] = vv
    log(f"{tag}: persistent {ms:.3f} ms, graph {ms_graph:.3f} ms, per-scene {ms_sep:.3f} ms "
        f"(tile {ti}, {bpc} blocks/CU), parity worst scaled {worst_scaled(worst):.2e}")
    del graph, plan, dev
    torch.cuda.empty_cache()
    lo, hi = (f"{x:.0e}".replace("e+0", "e") for x in (5e4 * scale, 2e6 * scale))
    return {"workload": f"{len(scenes)} scenes (N log-uniform in [{lo}, {hi}], K in {{4,8,16}}, "
                        f"V in {{1,4,16}}), one persistent fused fwd+bwd launch, {norm} normaliser",
            "scenes": len(scenes), "primitives": sum(s.workload.n for s in scenes), "evals": evals,
            "tile_iters": ti, "blocks_per_cu": bpc,
            "ms": round(ms, 4), "G_evals_s": round(evals / ms / 1e6, 4),
            "roofline": roofline(f"nasg_batch_uneven{len(scenes)}_{norm}", ms, ab, evals, ops,
                                 ceiling=ceiling, kernel="nasg_batched_kernel (persistent)"),
            "graph_replay": {"ms": round(ms_graph, 4), "G_evals_s": round(evals / ms_graph / 1e6, 4)},
            "per_scene_launches": {"ms": round(ms_sep, 4), "G_evals_s": round(evals / ms_sep / 1e6, 4)},
            "tuner_sweep_ms": sweep,
            "parity_sampled_worst_scene": worst}


def bench_other(args, log):
    """Workloads other than the headline, each as its own JSON line."""
    import torch

    import paper_2606_09794_amd as P
    import workloads as W
    if args.profile:
        profile_other(args, log)
        return
    res = {"metric": METRIC, "unit": "G evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic"}

    def line(m, dtype, **cfg):
        res.update(value=m["G_evals_s"], ms_per_step=m["ms"], dtype=dtype,
                   config=dict({"workload": m["workload"]}, **cfg), roofline=m["roofline"],
                   detail={k: v for k, v in m.items() if k not in ("roofline", "workload")})

    if args.workload == "single-camera":
        line(measure_single_camera(args.norm, args.steps, args.warmup, log, n=args.n), "f32",
             primitives=args.n, lobes=8, views=1)
    elif args.workload == "bf16-k16":
        line(measure_bf16_k16(args.norm, args.steps, args.warmup, log, n=args.n), "f32 (bf16 storage)",
             primitives=args.n, lobes=16, views=8)
    elif args.workload == "uneven-batch":
        line(measure_uneven_batch(args.norm, args.steps, args.warmup, log), "f32", scenes=32)
    elif args.workload == "paper-params":
        t0 = time.perf_counter()
        w = W.draw_workload(7, args.n, 8, args.views, with_sh=False, param="angles")
        log(f"generated N={w.n} K={w.k} V={w.v} (raw values) in {time.perf_counter() - t0:.1f}s")
        d = upload(w)
        n, k, v = w.n, w.k, w.v
        g = P.nasg_grad_buffers(k, n, "cuda")
        rgb = torch.empty((v, n, 3), device="cuda")
        fn = lambda dd, par: P.nasg_eval_bwd(dd["quat"], dd["shape"], dd["rgbw"], dd["c0"],  # noqa: E731
                                             dd["grad_rgb"], means=dd["means"], cams=dd["cams"],
                                             norm=args.norm, grads=g, rgb_out=rgb, param=par)
        ms = time_launches(lambda: fn(d, "angles"), args.steps, args.warmup)
        fn(d, "angles")
        torch.cuda.synchronize()
        par = _sampled(w, dict(g, rgb=rgb), args.norm)
        del d
        wq = W.draw_workload(7, n, k, v, with_sh=False)
        dq = upload(wq)
        msq = time_launches(lambda: fn(dq, "quat"), args.steps, args.warmup)
        ab = algorithmic_bytes(n, k, v)
        res.update(value=round(n * v / ms / 1e6, 4), ms_per_step=round(ms, 4), dtype="f32",
                   config={"workload": f"NASGabor K={k} fused fwd+bwd, {n} primitives x {v} cameras, "
                                       f"the paper's raw lobe values (three frame cosines and "
                                       f"activations), FP32, {args.norm} normaliser",
                           "primitives": n, "lobes": k, "views": v, "param": "angles"},
                   roofline=roofline(f"nasg_fused_k{k}_v{v}_n{n}_{args.norm}_angles", ms, ab, n * v,
                                     kernel="nasg_kernel (fused, the paper's raw values)"),
                   compare={"quaternion_parametrisation_same_sizes": {
                       "ms": round(msq, 4), "G_evals_s": round(n * v / msq / 1e6, 4)}},
                   parity_sampled=par)
    elif args.workload == "families":
        per = {}
        n, k, v = args.n, 8, args.views
        ab = algorithmic_bytes(n, k, v)
        g = P.nasg_grad_buffers(k, n, "cuda")
        rgb = torch.empty((v, n, 3), device="cuda")
        for fam in ("nasgabor", "nasg", "sg", "sb", "sc", "asg"):
            t0 = time.perf_counter()
            w = W.draw_workload(11, n, k, v, with_sh=False, family=fam)
            log(f"generated {fam} N={n} K={k} V={v} in {time.perf_counter() - t0:.1f}s")
            d = upload(w)
            fn = lambda: P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"],  # noqa: E731
                                         d["grad_rgb"], means=d["means"], cams=d["cams"],
                                         norm=args.norm, grads=g, rgb_out=rgb, family=fam)
            ms = time_launches(fn, args.steps, args.warmup)
            fn()
            torch.cuda.synchronize()
            rep = _sampled(w, dict(g, rgb=rgb), args.norm, n_sample=128)
            per[fam] = {"ms": round(ms, 4), "G_evals_s": round(n * v / ms / 1e6, 4),
                        "hbm_frac": round(ab / ms / 1e6 / HBM_PEAK_GBS, 4),
                        "parity_sampled_max_scaled_error": worst_scaled(rep)}
            del d
        best = per["nasgabor"]
        res.update(value=best["G_evals_s"], ms_per_step=best["ms"], dtype="f32",
                   config={"workload": f"lobe families of the distribution table, K={k} fused fwd+bwd, "
                                       f"{n} primitives x {v} cameras each, FP32; value = NASGabor",
                           "primitives": n, "lobes": k, "views": v},
                   # the NASGabor launch is the headline's kernel at the headline's sizes
                   roofline=roofline(f"nasg_fused_k{k}_v{v}_n{n}_{args.norm}", best["ms"], ab, n * v,
                                     algorithmic_ops_per_eval(k, v, args.norm),
                                     kernel="nasg_kernel (fused forward+backward)"),
                   families=per)
    elif args.workload == "training-view":
        res.update(_training_view(args, log))
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    print(json.dumps(res), flush=True)


def _training_view(args, log):
    """One training view: NASGabor colours of every primitive along its
    central ray for one camera, compositing into a 1920 x 1080 image, the
    compositing backward (colours, opacities, means, scales, quaternions) and
    the appearance backward on its colour gradients. One step = those four
    calls."""
    import torch

    import paper_2606_09794_amd as P
    import workloads as W
    from oracle import metrics as M
    from oracle import nasg_ref as R
    from oracle import raster_ref as RR
    n, k, width, height, cap = args.n, 8, 1920, 1080, 4096
    t0 = time.perf_counter()
    sc = W.draw_splat_scene(12, n, width, height)
    w = W.draw_workload(12, n, k, 1, with_grad=False, with_sh=False)
    log(f"generated scene N={n} {width}x{height}, K={k} lobes in {time.perf_counter() - t0:.1f}s")
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    means, scales, rots, opac = dv(sc.means), dv(sc.scales), dv(sc.rots), dv(sc.opac)
    quat, shape, rgbw, c0 = dv(w.quat), dv(w.shape), dv(w.rgbw), dv(w.c0)
    cam = P.Camera(sc.cam["R"], sc.cam["t"], sc.cam["fx"], sc.cam["fy"], sc.cam["cx"], sc.cam["cy"],
                   width, height)
    cams = cam.centre("cuda")
    gimg = dv(sc.grad_image)
    rgb = torch.empty((1, n, 3), device="cuda")
    ws = torch.empty(P.raster_workspace_bytes(n, cam, cap), dtype=torch.uint8, device="cuda")
    g = P.nasg_grad_buffers(k, n, "cuda")
    state = {}

    def app_fwd():
        P.nasg_eval_fwd(quat, shape, rgbw, c0, means=means, cams=cams, norm=args.norm, out=rgb)

    def ras_fwd():
        state["img"], _ = P.raster_fwd(means, scales, rots, opac, rgb[0], cam, cap, workspace=ws,
                                       check_overflow=False)

    def ras_bwd():
        (state["gc"], state["go"], state["gm"], state["gs"],
         state["gr"]) = P.raster_bwd(means, scales, rots, opac, rgb[0], cam, ws, gimg, cap,
                                     geometry=True)

    def ras_bwd_colour_only():
        P.raster_bwd(means, scales, rots, opac, rgb[0], cam, ws, gimg, cap)

    def app_bwd():
        P.nasg_eval_bwd(quat, shape, rgbw, c0, state["gc"][None], means=means, cams=cams,
                        norm=args.norm, grads=g)

    def step():
        app_fwd()
        ras_fwd()
        ras_bwd()
        app_bwd()

    ms = time_launches(step, args.steps, args.warmup)
    parts = {name: round(time_launches(f, args.steps, 1), 4)
             for name, f in (("appearance_fwd", app_fwd), ("raster_fwd", ras_fwd),
                             ("raster_bwd", ras_bwd), ("appearance_bwd", app_bwd),
                             ("raster_bwd_colour_opacity_only", ras_bwd_colour_only))}
    step()
    torch.cuda.synchronize()
    if int(ws[:4].view(torch.int32).item()) != 0:
        raise SystemExit("a tile list overflowed; the measurement would miss primitives")
    log(f"training view {ms:.3f} ms/step, parts {parts}")
    # parity: a window of the image and the colour / opacity gradients of its
    # primitives against the oracle (upstream gradient restricted to the window
    # in a separate, untimed backward), and the appearance stage on sampled
    # primitives against the oracle with the device's colour gradients as input
    x0, y0, ww, hh = 900, 500, 32, 24
    gwin = torch.zeros_like(gimg)
    gwin[y0:y0 + hh, x0:x0 + ww] = gimg[y0:y0 + hh, x0:x0 + ww]
    gcw, gow, gmw, gsw, grw = P.raster_bwd(means, scales, rots, opac, rgb[0], cam, ws, gwin, cap,
                                           geometry=True)
    rgb_np = rgb[0].cpu().numpy()
    p = RR.project(sc.means, sc.scales, sc.rots, sc.cam)
    ex = 3 * np.sqrt(p["cov2"][:, 0, 0]) + 1
    ey = 3 * np.sqrt(p["cov2"][:, 1, 1]) + 1
    keep = p["vis"] & (p["u"] + ex >= x0) & (p["u"] - ex <= x0 + ww) & \
        (p["v"] + ey >= y0) & (p["v"] - ey <= y0 + hh)
    idx = np.nonzero(keep)[0]
    wcam = dict(sc.cam, cx=sc.cam["cx"] - x0, cy=sc.cam["cy"] - y0, width=ww, height=hh)
    ref, scale = RR.render(sc.means[idx], sc.scales[idx], sc.rots[idx], sc.opac[idx], rgb_np[idx],
                           wcam, grad_image=sc.grad_image[y0:y0 + hh, x0:x0 + ww], geometry=True)
    img = state["img"].cpu().numpy()
    par = {"image_window": float(M.scaled_error(img[y0:y0 + hh, x0:x0 + ww], ref["image"],
                                                scale["image"]).max()),
           "grad_colors_window": float(M.scaled_error(gcw.cpu().numpy()[idx], ref["colors"],
                                                      scale["colors"]).max()),
           "grad_opac_window": float(M.scaled_error(gow.cpu().numpy()[idx], ref["opac"],
                                                    scale["opac"]).max()),
           "grad_means_window": float(M.scaled_error(gmw.cpu().numpy()[idx], ref["means"],
                                                     scale["means"]).max()),
           "grad_scales_window": float(M.scaled_error(gsw.cpu().numpy()[idx], ref["scales"],
                                                      scale["scales"]).max()),
           "grad_rots_window": float(M.scaled_error(grw.cpu().numpy()[idx], ref["rots"],
                                                    scale["rots"]).max()),
           "window_primitives": int(len(idx))}
    sidx = np.sort(np.random.default_rng(0).choice(n, size=256, replace=False))
    sub = W.take_primitives(w, sidx)
    gc_np = state["gc"].cpu().numpy()[sidx][None]
    o = cams.cpu().numpy()
    code = R.NORM_EXACT if args.norm == "exact" else R.NORM_APPROX
    aref, ascale = R.forward_backward(sub.quat, sub.shape, sub.rgbw, sub.c0, gc_np, code,
                                      means=sc.means[sidx], cams=o)
    got = {"rgb": rgb[:, sidx].cpu().numpy(), "quat": g["quat"][:, sidx].cpu().numpy(),
           "shape": g["shape"][:, sidx].cpu().numpy(), "rgbw": g["rgbw"][:, :, sidx].cpu().numpy(),
           "c0": g["c0"][sidx].cpu().numpy(), "means": g["geom"][sidx].cpu().numpy()}
    for key_, v_ in got.items():
        par[f"appearance_{key_}"] = float(M.scaled_error(v_, aref[key_], ascale[key_]).max())
    log(f"parity {par}")
    tiles = ((width + 15) // 16) * ((height + 15) // 16)
    # dominant kernel: the compositing backward (raster_bwd = accumulator clear,
    # raster_render_bwd, rounding to float32; the two small kernels take ~0.5 %)
    counters = measured_counters(f"raster_render_bwd_geom_n{n}_{width}x{height}", RASTER_SOURCES)
    roofline = None
    if counters is not None:
        lane_ops = counters["valu_wave_instructions_per_launch"] * 64
        ach = lane_ops / (parts["raster_bwd"] * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(ach, 2),
                    "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
                    "unit": "T VALU lane-instructions/s",
                    "frac": round(ach * 1e12 / VALU_PEAK_LANE_OPS, 4),
                    "traffic": counters["bytes_per_launch"],
                    "kernel": "raster_render_bwd (compositing backward with geometry)"}
    return dict(value=round(n / ms / 1e6, 4), ms_per_step=round(ms, 4), dtype="f32 (f64 compositing sums)",
                config={"workload": f"one training view: NASGabor K={k} colours of {n} primitives for "
                                    f"one camera, composited into {width}x{height}, compositing "
                                    f"backward (colour, opacity and geometry gradients) and "
                                    f"appearance backward ({args.norm} normaliser)",
                        "primitives": n, "lobes": k, "views": 1, "width": width, "height": height,
                        "tile_capacity": cap, "tiles": tiles},
                roofline=roofline, parts_ms=parts, parity_max_scaled_error=par)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=3_000_000)
    ap.add_argument("--views", type=int, default=16)
    ap.add_argument("--norm", choices=["exact", "approx"], default="exact")
    ap.add_argument("--quick", action="store_true", help="headline only (no comparisons, no CPU leg)")
    ap.add_argument("--cpu-prims", type=int, default=3_000_000,
                    help="primitives in the CPU-oracle timing sample")
    ap.add_argument("--profile-kernel", choices=["nasg", "sh3"], default="nasg",
                    help="with --profile: the headline NASGabor launch (plus the copy "
                         "calibration) or the degree-3 SH fused launch on the same inputs")
    ap.add_argument("--profile", action="store_true",
                    help="counter-collection mode: a few headline launches plus a plain "
                         "device copy of --copy-mib MiB for calibrating byte counters; with "
                         "--workload single-camera, bf16-k16, paper-params or uneven-batch, "
                         "that workload's timed launch only")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--tile-iters", type=int, default=None,
                    help="with --profile --workload uneven-batch: tile passes per work item "
                         "(default: the tuner's cached choice, as the bench line uses)")
    ap.add_argument("--blocks-per-cu", type=int, default=None,
                    help="with --profile --workload uneven-batch: persistent blocks per CU "
                         "(default: the tuner's cached choice)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "single-camera", "bf16-k16", "uneven-batch", "paper-params",
                             "families", "training-view"],
                    help="headline: K=8, 3 M primitives x 16 cameras; single-camera: K=8, 1 M x 1; "
                         "bf16-k16: K=16, 6 M x 8, bf16 storage; uneven-batch: 32 scenes in one "
                         "persistent launch; paper-params: the headline sizes with the paper's raw "
                         "lobe values; families: every lobe family at the headline sizes; "
                         "training-view: K=8 colours of 3 M primitives for one camera composited "
                         "into 1920x1080, with both backwards")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; the path shards by primitive with no "
              "exchange, so --gpus N > 1 is not run", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2606_09794_amd as P
    import workloads as W
    from paper_2606_09794_amd import autotune

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    autotune.load_cache()
    if args.workload != "headline":
        if args.n == 3_000_000:
            args.n = {"single-camera": 1 << 20, "bf16-k16": 6_000_000}.get(args.workload, args.n)
        bench_other(args, log)
        return
    t0 = time.perf_counter()
    w = W.config2(n=args.n, v=args.views)
    log(f"generated N={w.n} K={w.k} V={w.v} in {time.perf_counter() - t0:.1f}s")
    d = upload(w)
    n, k, v = w.n, w.k, w.v
    g = P.nasg_grad_buffers(k, n, "cuda")
    rgb = torch.empty((v, n, 3), device="cuda")

    def fused():
        P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], means=d["means"],
                        cams=d["cams"], norm=args.norm, grads=g, rgb_out=rgb)

    if args.profile:
        if args.profile_kernel == "sh3":
            gsh = {"sh": torch.empty_like(d["sh"]), "geom": torch.empty((n, 3), device="cuda")}
            for _ in range(args.steps):
                P.sh3_eval_bwd(d["sh"], d["grad_rgb"], means=d["means"], cams=d["cams"], grads=gsh,
                               rgb_out=rgb)
            torch.cuda.synchronize()
            print(json.dumps({"profile": True, "kernel": "sh3 fused", "launches": args.steps,
                              "n": n, "v": v, "algorithmic_bytes_per_launch": sh_bytes(n, v),
                              "source_hash": kernel_source_hash(SH_SOURCES)}), flush=True)
            return
        for _ in range(args.steps):
            fused()
        src = torch.empty(args.copy_mib << 18, device="cuda")        # float32 elements
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": True, "fused_launches": args.steps, "n": n, "k": k, "v": v,
                          "copy_bytes": src.numel() * 4, "copies": 3,
                          "algorithmic_bytes_per_launch": algorithmic_bytes(n, k, v),
                          "source_hash": kernel_source_hash()}), flush=True)
        return

    ms = time_launches(fused, args.steps, args.warmup)
    evals = n * v
    value = evals / (ms * 1e-3) / 1e9
    abytes = algorithmic_bytes(n, k, v)
    log(f"fused fwd+bwd {ms:.3f} ms/step, {value:.2f} G evals/s, "
        f"{abytes / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic")
    ceiling, stream = None, None
    if not args.quick:
        stream, stream_sweep = stream_ceiling()
        ceiling = stream["copy"]["GB_s"]
        log(f"streaming ceiling: read {stream['read']['GB_s']} write {stream['write']['GB_s']} "
            f"copy {stream['copy']['GB_s']} GB/s")
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "G evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"NASGabor K={k} fused fwd+bwd, {n} primitives x {v} cameras, "
                               f"one launch, FP32 storage, {args.norm} normaliser",
                   "primitives": n, "lobes": k, "views": v, "norm": args.norm},
        "roofline": roofline(f"nasg_fused_k{k}_v{v}_n{n}_{args.norm}", ms, abytes, evals,
                             algorithmic_ops_per_eval(k, v, args.norm), ceiling=ceiling,
                             kernel="nasg_kernel (fused forward+backward)"),
    }

    if not args.quick:
        cmp = {}
        steps = max(3, args.steps // 2)

        def sep():
            P.nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], means=d["means"],
                            cams=d["cams"], norm=args.norm, out=rgb)
            P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"],
                            means=d["means"], cams=d["cams"], norm=args.norm, grads=g)
        m = time_launches(sep, steps, 1)
        cmp["nasg_separate_fwd_then_bwd"] = {"ms": round(m, 4), "G_evals_s": round(evals / m / 1e6, 4)}
        # 16 single-view launches, gradients accumulated
        cams1 = [d["cams"][i:i + 1].contiguous() for i in range(v)]
        gr1 = [d["grad_rgb"][i:i + 1].contiguous() for i in range(v)]
        rgb1 = torch.empty((1, n, 3), device="cuda")

        def single():
            for i in range(v):
                P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], gr1[i], means=d["means"],
                                cams=cams1[i], norm=args.norm, grads=g, accumulate=i > 0, rgb_out=rgb1)
        m = time_launches(single, max(2, steps // 4), 1)
        cmp["nasg_16_single_view_launches"] = {"ms": round(m, 4), "G_evals_s": round(evals / m / 1e6, 4)}
        other = "approx" if args.norm == "exact" else "exact"

        def fused_other():
            P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], means=d["means"],
                            cams=d["cams"], norm=other, grads=g, rgb_out=rgb)
        m = time_launches(fused_other, steps, 1)
        cmp[f"nasg_fused_{other}_normaliser"] = {"ms": round(m, 4), "G_evals_s": round(evals / m / 1e6, 4)}
        # SH degree 3, same means / cameras / upstream gradient
        gsh = {"sh": torch.empty_like(d["sh"]), "geom": torch.empty((n, 3), device="cuda")}
        rsh = torch.empty_like(rgb)

        def sh():
            P.sh3_eval_bwd(d["sh"], d["grad_rgb"], means=d["means"], cams=d["cams"], grads=gsh,
                           rgb_out=rsh)
        m = time_launches(sh, steps, 1)
        sb = sh_bytes(n, v)
        cmp["sh3_fused"] = {"ms": round(m, 4), "G_evals_s": round(evals / m / 1e6, 4),
                            "roofline": roofline(f"sh3_fused_n{n}_v{v}", m, sb, evals, files=SH_SOURCES,
                                                 ceiling=ceiling, kernel="sh3_kernel (fused)")}
        # plain FP32 single-view path on the same primitives (first camera)
        def plain():
            P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], gr1[0], means=d["means"],
                            cams=cams1[0], norm=args.norm, grads=g, rgb_out=rgb1)
        m = time_launches(plain, steps, 1)
        pb = algorithmic_bytes(n, k, 1)
        cmp["nasg_plain_single_view"] = {"ms": round(m, 4), "G_evals_s": round(n / m / 1e6, 4),
                                         "GB_s": round(pb / m / 1e6, 1),
                                         "hbm_frac": round(pb / m / 1e6 / HBM_PEAK_GBS, 4)}
        cmp["hbm_stream_ceiling"] = dict(stream, runtime_copy=copy_ceiling(steps), sweep_GB_s=stream_sweep)
        # sampled parity of the timed configuration (rerun the headline once)
        fused()
        torch.cuda.synchronize()
        out["parity_sampled"] = _sampled(w, dict(g, rgb=rgb), args.norm, n_sample=512)
        log(f"parity: worst scaled error {worst_scaled(out['parity_sampled']):.2e}")
        del d, g, rgb, gsh, rsh, rgb1, cams1, gr1
        torch.cuda.empty_cache()
        # the other workloads, each at its own full size in its benchmarked launch
        cmp["single_camera_1M"] = measure_single_camera(args.norm, args.steps, args.warmup, log,
                                                        ceiling=ceiling)
        torch.cuda.empty_cache()
        cmp["bf16_k16_6M_x8"] = measure_bf16_k16(args.norm, args.steps, args.warmup, log, ceiling=ceiling)
        torch.cuda.empty_cache()
        cmp["uneven_batch_32_scenes"] = measure_uneven_batch(args.norm, args.steps, args.warmup, log,
                                                             ceiling=ceiling)
        torch.cuda.empty_cache()
        # the case a single persistent launch is for: many small scenes
        cmp["uneven_batch_256_small_scenes"] = measure_uneven_batch(
            args.norm, args.steps, args.warmup, log, ceiling=ceiling, n_scenes=256, scale=0.02,
            parity_every=16)
        out["compare"] = cmp
        out["cpu_baseline"] = cpu_baseline(w, prims=args.cpu_prims,
                                           norm_code=0 if args.norm == "exact" else 1)
        log(f"cpu baseline {out['cpu_baseline']['value'] * 1e3:.3f} M evals/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
