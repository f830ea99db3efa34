"""Launch-shape autotuner for libnasg.

For a key (kernel, K, V, storage dtype) it times every compiled
(lanes per primitive, views per lane) mapping and block size on synthetic
device inputs of the requested size, installs the fastest in the library's
tuning table (``nasg_set_tuning``) and records it in a JSON cache, which
``load_cache`` replays at start-up.

    python -m paper_2606_09794_amd.autotune --k 8 --v 16 --n 3000000
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, List, Tuple

from . import _lib as L
from .api import (get_tuning, nasg_eval_bwd, nasg_eval_fwd, nasg_grad_buffers, set_tuning,
                  sh3_eval_bwd, sh3_eval_fwd)

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
MAPPINGS: List[Tuple[int, int]] = [(1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2),
                                   (4, 4), (8, 1), (8, 2), (16, 1)]
# the broadcast-view mappings (NASGabor kernels only)
BCAST_MAPPINGS: List[Tuple[int, int]] = [(4, 1), (8, 1), (16, 1), (8, 2), (8, 4)]
BLOCKS = (64, 128, 256)
KERNELS = {"nasg_fwd": L.KERNEL_NASG_FWD, "nasg_bwd": L.KERNEL_NASG_BWD,
           "sh_fwd": L.KERNEL_SH_FWD, "sh_bwd": L.KERNEL_SH_BWD}


def _key(kernel: int, k: int, v: int, dtype: int) -> str:
    return f"{kernel}/{k}/{v}/{dtype}"


def load_cache(path: str = CACHE) -> int:
    """Install every cached choice into the library; returns how many."""
    if not os.path.exists(path):
        return 0
    with open(path) as fh:
        data = json.load(fh)
    count = 0
    for key, ent in data.get("entries", {}).items():
        kernel, k, v, dtype = (int(x) for x in key.split("/"))
        set_tuning(kernel, k, v, dtype, ent["lanes"], ent["views_per_lane"], ent["block"],
                   ent.get("bcast", 0))
        count += 1
    return count


def save_entry(kernel: int, k: int, v: int, dtype: int, choice: Dict, path: str = CACHE) -> None:
    data = {"arch": "gfx950", "entries": {}}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data["entries"][_key(kernel, k, v, dtype)] = choice
    with open(path + ".tmp", "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)


def _inputs(k: int, v: int, n: int, bf16: bool, seed: int = 0):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    f = dict(device="cuda", generator=g)
    quat = torch.randn((k, n, 4), **f)
    lam = torch.exp(torch.rand((k, n), **f) * 6.9078)
    a = torch.exp(torch.rand((k, n), **f) * 6.9078)
    kk = torch.rand((k, n), **f) * 16
    zeta = torch.rand((k, n), **f) * 6.2832
    shape = torch.stack([lam, a, kk, zeta], -1).contiguous()
    rgbw = torch.randn((k, 3, n), **f) * 0.5
    if bf16:
        quat, shape, rgbw = (t.to(torch.bfloat16) for t in (quat, shape, rgbw))
    c0 = torch.randn((n, 3), **f) * 0.5
    means = torch.rand((n, 3), **f) * 10 - 5
    cams = torch.nn.functional.normalize(torch.randn((v, 3), **f), dim=1) * 10
    grad = torch.randn((v, n, 3), **f)
    sh = torch.randn((16, 3, n), **f) * 0.3
    return dict(quat=quat, shape=shape, rgbw=rgbw, c0=c0, means=means, cams=cams, grad_rgb=grad, sh=sh)


def tune(kernel: int, k: int, v: int, dtype: int, n: int, steps: int = 5, norm: str = "exact",
         save: bool = True, verbose: bool = True, cache: str = CACHE) -> Dict:
    """Time every mapping for one key and install the fastest."""
    import torch
    d = _inputs(k, v, n, dtype == L.NASG_BF16)
    out = torch.empty((v, n, 3), device="cuda")
    grads = nasg_grad_buffers(k, n, "cuda") if kernel == L.KERNEL_NASG_BWD else None
    gsh = {"sh": torch.empty_like(d["sh"]), "geom": torch.empty((n, 3), device="cuda")}

    def call():
        if kernel == L.KERNEL_NASG_FWD:
            nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], means=d["means"], cams=d["cams"],
                          norm=norm, out=out)
        elif kernel == L.KERNEL_NASG_BWD:
            nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], means=d["means"],
                          cams=d["cams"], norm=norm, grads=grads, rgb_out=out)
        elif kernel == L.KERNEL_SH_FWD:
            sh3_eval_fwd(d["sh"], means=d["means"], cams=d["cams"], out=out)
        else:
            sh3_eval_bwd(d["sh"], d["grad_rgb"], means=d["means"], cams=d["cams"], grads=gsh, rgb_out=out)

    def timed(steps_):
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps_):
            call()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps_

    # warm the clocks on the built-in choice before the sweep
    set_tuning(kernel, k, v, dtype, 0, 0)
    timed(4 * steps)
    results = []
    cands = [(lanes, vpl, 0) for lanes, vpl in MAPPINGS
             if lanes <= max(1, v) and lanes * vpl <= 4 * max(v, 1)]
    if kernel in (L.KERNEL_NASG_FWD, L.KERNEL_NASG_BWD):
        # broadcast views: lanes up to the lobe count, views per lane up to V
        cands += [(lanes, vpl, 1) for lanes, vpl in BCAST_MAPPINGS
                  if lanes <= max(4, k) and vpl <= max(1, v)]
    for lanes, vpl, bc in cands:
        for block in BLOCKS:
            set_tuning(kernel, k, v, dtype, lanes, vpl, block, bc)
            ms = timed(steps)
            results.append((ms, lanes, vpl, block, bc))
            if verbose:
                print(f"  kernel={kernel} K={k} V={v} dtype={dtype} lanes={lanes} vpl={vpl} "
                      f"bcast={bc} block={block}: {ms:.3f} ms", flush=True)
    # confirm: the fastest few again, interleaved, with four times the steps
    top = sorted(results)[:4]
    best = {c[1:]: [] for c in top}
    for _ in range(2):
        for c in top:
            set_tuning(kernel, k, v, dtype, *c[1:])
            best[c[1:]].append(timed(2 * steps))
    ms, (lanes, vpl, block, bc) = min((min(t), c) for c, t in best.items())
    set_tuning(kernel, k, v, dtype, lanes, vpl, block, bc)
    choice = {"lanes": lanes, "views_per_lane": vpl, "block": block, "bcast": bc,
              "ms": round(ms, 4), "n": n}
    if save:
        save_entry(kernel, k, v, dtype, choice, path=cache)
    assert get_tuning(kernel, k, v, dtype) == (lanes, vpl, block, bc)
    return choice


# ---------------------------------------------------------------- batches
# The persistent multi-scene launch has its own launch shape: the 256-thread
# block passes per work item (tile size) and the persistent blocks per compute
# unit. It is tuned on a whole batch and cached under the key "batch".
BATCH_TILE_ITERS = (1, 2, 4, 8, 16)
BATCH_BLOCKS_PER_CU = (1, 2, 3, 4)
BATCH_FALLBACK = (4, 2)


def batch_defaults(path: str = CACHE) -> Tuple[int, int]:
    """(tile_iters, blocks_per_cu) from the cache's batch entry, else the
    built-in (4, 2)."""
    if os.path.exists(path):
        with open(path) as fh:
            ent = json.load(fh).get("batch")
        if ent:
            return int(ent["tile_iters"]), int(ent["blocks_per_cu"])
    return BATCH_FALLBACK


def tune_batch(scenes, norm: str = "exact", steps: int = 3, save: bool = True,
               verbose: bool = True, path: str = CACHE) -> Dict:
    """Time a persistent plan of `scenes` (the list NasgBatchPlan takes) for
    every (tile_iters, blocks_per_cu) pair; the fastest is returned and, with
    `save`, recorded as the cache's batch entry."""
    import torch

    from .api import NasgBatchPlan
    results = []
    for ti in BATCH_TILE_ITERS:
        for bpc in BATCH_BLOCKS_PER_CU:
            plan = NasgBatchPlan(scenes, norm=norm, tile_iters=ti, blocks_per_cu=bpc)
            plan.run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                plan.run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            results.append((ms, ti, bpc))
            if verbose:
                print(f"  batch tile_iters={ti} blocks_per_cu={bpc}: {ms:.3f} ms", flush=True)
    ms, ti, bpc = min(results)
    choice = {"tile_iters": ti, "blocks_per_cu": bpc, "ms": round(ms, 4), "scenes": len(scenes),
              "sweep_ms": {f"tile{t_}_bpc{b_}": round(m_, 4) for m_, t_, b_ in results}}
    if save:
        data = {"arch": "gfx950", "entries": {}}
        if os.path.exists(path):
            with open(path) as fh:
                data = json.load(fh)
        data["batch"] = {k: v for k, v in choice.items() if k != "sweep_ms"}
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    return choice


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernels", default="nasg_fwd,nasg_bwd,sh_fwd,sh_bwd")
    ap.add_argument("--k", type=int, nargs="+", default=[8])
    ap.add_argument("--v", type=int, nargs="+", default=[16])
    ap.add_argument("--dtype", type=int, nargs="+", default=[0])
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--cache", default=CACHE, help="JSON file the choices are written to")
    ap.add_argument("--batch", action="store_true",
                    help="tune the persistent launch on the 32-scene uneven batch instead")
    args = ap.parse_args()
    if args.batch:
        import sys

        import torch
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import workloads as W
        from .api import nasg_grad_buffers as bufs
        dev = []
        for sc in W.config4():
            w = sc.workload
            t = {k: torch.from_numpy(getattr(w, k)).cuda()
                 for k in ("quat", "shape", "rgbw", "c0", "means", "cams", "grad_rgb")}
            t["grads"] = bufs(w.k, w.n, "cuda")
            t["rgb"] = torch.empty((w.v, w.n, 3), device="cuda")
            dev.append(t)
        print(f"batch: {tune_batch(dev, path=args.cache)}", flush=True)
        return
    for name in args.kernels.split(","):
        kern = KERNELS[name]
        for k in (args.k if kern < 2 else [0]):
            for v in args.v:
                for dt in (args.dtype if kern < 2 else [0]):
                    c = tune(kern, k, v, dt, args.n, args.steps, cache=args.cache)
                    print(f"{name} K={k} V={v} dtype={dt}: {c}", flush=True)


if __name__ == "__main__":
    main()
