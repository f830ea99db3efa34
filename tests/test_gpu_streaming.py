"""GPU parity around the appearance kernels' streaming flavour.

A launch with one lane per primitive whose views fit in one chunk and which
does not accumulate reads every lobe record and writes every output once and
takes the kernel flavour with nontemporal accesses; a launch with more view
chunks, or one adding onto earlier gradients, takes the plain one. Each
mapping with one lane per primitive runs on both sides of that line (V from
1 to views-per-lane + 1, FP32 and bf16 storage), into output buffers filled
beforehand: with NaN when the launch overwrites (every output must be
written), with known values when it accumulates (the result must be those
values plus the oracle's gradients). Bar: the FP32 bar of the other parity
tests, 1e-5 on the scaled error.
"""
import numpy as np
import pytest
import torch

import paper_2606_09794_amd as P
import workloads as W
from gpu_util import compare, dgeo, oracle_nasg, upload

pytestmark = pytest.mark.gpu
TOL = 1e-5
GRADS = ("quat", "shape", "rgbw", "c0", "geom")


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for kern in (0, 1):
        for v in range(1, 6):
            for dt in (0, 1):
                P.set_tuning(kern, 5, v, dt, 0, 0)


def _buffers(k, n, fill):
    g = P.nasg_grad_buffers(k, n, "cuda")
    for t in g.values():
        t.copy_(fill(t.shape))
    return g


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("vpl", [1, 2, 4])
def test_one_lane_mappings_across_the_chunk_line(vpl, dtype):
    dt = 1 if dtype == "bf16" else 0
    for v in range(1, vpl + 2):
        print(f"vpl={vpl} V={v} {dtype}", flush=True)
        w = W.draw_workload(400 + 10 * vpl + v, 777, 5, v, dtype=dtype)
        for kern in (0, 1):
            P.set_tuning(kern, 5, v, dt, 1, vpl)
        d = upload(w)
        ref, scale = oracle_nasg(w, "exact")
        nan = lambda shape: torch.full(shape, float("nan"), device="cuda")  # noqa: E731
        # overwrite: every output written (single chunk: the streaming flavour)
        g = _buffers(5, w.n, nan)
        rgb = torch.full((v, w.n, 3), float("nan"), device="cuda")
        P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], norm="exact",
                        grads=g, rgb_out=rgb, **dgeo(d))
        fwd = torch.full((v, w.n, 3), float("nan"), device="cuda")
        P.nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], norm="exact", out=fwd,
                        **dgeo(d))
        torch.cuda.synchronize()
        compare(rgb.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb (fused)", TOL)
        compare(fwd.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb", TOL)
        for name in GRADS:
            compare(g[name].cpu().numpy(), ref[name], scale[name], name, TOL)
        # accumulate onto known values: the plain flavour, whatever the chunking
        gen = torch.Generator(device="cuda").manual_seed(v)
        rnd = lambda shape: torch.randn(shape, device="cuda", generator=gen)  # noqa: E731
        g = _buffers(5, w.n, rnd)
        base = {k: t.clone() for k, t in g.items()}
        P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], norm="exact",
                        grads=g, accumulate=True, **dgeo(d))
        torch.cuda.synchronize()
        for name in GRADS:
            got = g[name].double().cpu().numpy() - base[name].double().cpu().numpy()
            # the stored sum rounds base + grad once: allow that rounding beside the bar
            slack = np.abs(base[name].double().cpu().numpy()) * 2.0 ** -23
            err = np.abs(got - ref[name]) - slack
            assert np.all(err <= TOL * np.maximum(scale[name], 1e-30)), name
