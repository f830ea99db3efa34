"""GPU parity in the edge regions of the NASGabor lobe (Section 5.1 definition
and closed-form integral): designed inputs from ``workloads.edges``, run
through the C ABI, against the FP64 oracle on the same stored values.

* the fixed edge grid: k = Lam exactly and Lam^2 - k^2 in {+-0.5, +-1, +-1.5}
  (the series branch of the normaliser's sinhc and its boundaries), k > Lam
  with small Lam (the sine branch), zeta = pi +- 1e-2 / 1e-4 with
  k in {0, 1e-4, 1e-2} (1 + cos(zeta) Psi near zero), views 1e-7 .. 1e-1 rad
  from +z and from -z (sharp and broad lobes, d.x largest and d.x = 0),
  Lam in {1e2, 1e4, 1e6} viewed at 0.1, 1 and 3 peak widths, k = 0;
* seeded draws in every region (the regions the oracle's Hypothesis tests
  sweep against 50-digit values), through several lane mappings;
* camera-mode workloads whose sharp lobes (Lam up to 1e6) are aimed at the
  cameras, at the tuned 16-view mapping;
* lobes on both sides of lam = 1/2 and Lam = 3/2, where the normaliser
  changes between its FP32 and FP64 code;
each in float32 and bfloat16 storage (the oracle sees the dequantised
values) and with both normalisers. Bar: scaled error <= 1e-5 element-wise on
every output and gradient; the plain relative error is printed beside it.
"""
import numpy as np
import pytest
import torch

import paper_2606_09794_amd as P
from gpu_util import compare, dgeo, oracle_nasg, upload
from workloads import edges as E

pytestmark = pytest.mark.gpu
TOL = 1e-5
OUTPUTS = ("quat", "shape", "rgbw", "c0", "geom")


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for kern in (0, 1):
        for k in (1, 8):
            for v in (1, 16):
                for dt in (0, 1):
                    P.set_tuning(kern, k, v, dt, 0, 0)


def _run_and_check(w, norm, label):
    print(f"\n[{label}] n={w.n} k={w.k} v={w.v} {w.dtype} {norm}", flush=True)
    d = upload(w)
    rgb = P.nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], norm=norm, **dgeo(d))
    rgb_f = torch.empty_like(rgb)
    g = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], norm=norm,
                        rgb_out=rgb_f, **dgeo(d))
    torch.cuda.synchronize()
    ref, scale = oracle_nasg(w, norm)
    compare(rgb.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb", TOL)
    compare(rgb_f.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb (fused)", TOL)
    for name in OUTPUTS:
        compare(g[name].cpu().numpy(), ref[name], scale[name], name, TOL)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("norm", ["exact", "approx"])
def test_edge_grid(dtype, norm):
    """Every named edge point, one lobe and one raw view each."""
    _run_and_check(E.edge_grid(dtype), norm, "edge grid")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("norm", ["exact", "approx"])
@pytest.mark.parametrize("region", E.REGIONS)
def test_edge_region_draws(region, norm, dtype):
    """64 seeded draws in one region."""
    seed = 1000 + E.REGIONS.index(region) + (50 if dtype == "bf16" else 0)
    _run_and_check(E.edge_workload(seed, 64, regions=(region,), dtype=dtype), norm, region)


@pytest.mark.parametrize("lanes,vpl", [(2, 2), (8, 2), (16, 1)])
def test_edge_draws_every_region_other_mappings(lanes, vpl):
    """All regions in one launch through mappings that spread a primitive
    over several lanes (its single view slot travels round the group)."""
    for kern in (0, 1):
        P.set_tuning(kern, 1, 1, 0, lanes, vpl)
    _run_and_check(E.edge_workload(77, 24), "exact", f"all regions, {lanes}x{vpl}")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("norm", ["exact", "approx"])
def test_sharp_lobes_aimed_at_cameras(dtype, norm):
    """K = 8 sharp lobes (Lam log-uniform in [1e2, 1e6]) aimed 1e-5 .. 3e-2 rad
    off the direction to one of 16 cameras: every lobe meets one view next to
    its peak and fifteen far from it, at the tuned 16-view mapping."""
    _run_and_check(E.aimed_workload(21 + (dtype == "bf16"), 1501, 8, 16, dtype), norm,
                   "aimed sharp lobes")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("norm", ["exact", "approx"])
def test_normaliser_precision_switch(dtype, norm):
    """Lobes on both sides of lam = 1/2 and Lam = 3/2, where the kernel moves
    between its FP32 and FP64 normaliser, in every branch of Psi and with
    zeta at 0, pi/2 and next to pi."""
    _run_and_check(E.switch_grid(dtype), norm, "precision switch")


def test_aimed_single_camera():
    """The single-camera mapping on aimed lobes (every lobe of a primitive
    aimed at the one camera)."""
    _run_and_check(E.aimed_workload(23, 2049, 8, 1), "exact", "aimed, one camera")


def test_edge_grid_is_deterministic():
    w = E.edge_grid()
    d = upload(w)
    outs = []
    for _ in range(2):
        rgb = torch.empty_like(d["grad_rgb"])
        g = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"],
                            dirs=d["dirs"], rgb_out=rgb)
        torch.cuda.synchronize()
        outs.append([rgb.clone()] + [g[k].clone() for k in OUTPUTS])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    assert np.isfinite(outs[0][0].cpu().numpy()).all()
