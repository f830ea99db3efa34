"""GPU parity for the other lobe families of the paper's distribution table
(Supplementary A): NASG (Supplementary E), spherical Gaussian, spherical beta,
spherical Cauchy and anisotropic spherical Gaussian, through the C ABI against
the FP64 oracle on the same seeded values, FP32 bar 1e-5 on the scaled error."""
import pytest
import torch

import paper_2606_09794_amd as P
import workloads as W
from gpu_util import compare, dgeo, oracle_nasg, upload

pytestmark = pytest.mark.gpu
TOL = 1e-5
FAMS = ["nasg", "sg", "sb", "sc", "asg"]


def _check(w, tol=TOL):
    d = upload(w)
    kw = dict(param=w.param, family=w.family, **dgeo(d))
    rgb = P.nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], **kw)
    rgb_f = torch.empty_like(rgb)
    g = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], rgb_out=rgb_f, **kw)
    torch.cuda.synchronize()
    ref, scale = oracle_nasg(w, "exact")
    compare(rgb.cpu().numpy(), ref["rgb"], scale["rgb"], f"{w.family} rgb", tol)
    compare(rgb_f.cpu().numpy(), ref["rgb"], scale["rgb"], f"{w.family} rgb (fused)", tol)
    for name in ("quat", "shape", "rgbw", "c0", "geom"):
        compare(g[name].cpu().numpy(), ref[name], scale[name], f"{w.family} {name}", tol)
    return g


@pytest.mark.parametrize("fam", FAMS)
def test_sixteen_views_k8(fam):
    """(8 lanes, 2 views) mapping; 1200 primitives."""
    _check(W.draw_workload(80 + FAMS.index(fam), 1200, 8, 16, family=fam))


@pytest.mark.parametrize("fam", FAMS)
def test_single_camera_ragged(fam):
    """(1, 1) mapping, 2001 primitives."""
    _check(W.draw_workload(90 + FAMS.index(fam), 2001, 8, 1, family=fam))


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("v", [3, 5, 37])
def test_other_view_counts(fam, v):
    """(2, 2) at V = 3, (4, 2) at V = 5 with K = 3 (a lane without a lobe in
    every chunk), and V = 37 (view chunks accumulating in place)."""
    _check(W.draw_workload(100 + 7 * FAMS.index(fam) + v, 257, 3, v, family=fam))


@pytest.mark.parametrize("fam", FAMS)
def test_bf16_storage(fam):
    _check(W.draw_workload(110 + FAMS.index(fam), 600, 4, 8, family=fam, dtype="bf16"))


def test_nasg_with_the_papers_raw_values():
    w = W.draw_workload(120, 900, 8, 16, param="angles")
    w.family = "nasg"
    g = _check(w)
    assert torch.all(g["shape"][..., 2:] == 0)


def test_nasg_equals_nasgabor_without_carrier():
    """NASG lobes equal NASGabor lobes with k = zeta = 0 and the NASG
    normaliser, computed by the NASGabor kernel (two different kernels)."""
    w = W.draw_workload(121, 700, 8, 16, family="nasg")
    d = upload(w)
    a = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], means=d["means"],
                        cams=d["cams"], rgb_out=torch.empty((16, 700, 3), device="cuda"),
                        family="nasg")
    ga = {k: v.clone() for k, v in a.items()}
    b = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], means=d["means"],
                        cams=d["cams"], norm="approx")
    torch.cuda.synchronize()
    ref, scale = oracle_nasg(w, "exact")
    for name in ("quat", "rgbw", "c0", "geom"):
        compare(ga[name].cpu().numpy(), b[name].cpu().numpy(), scale[name], name, 2 * TOL)
    compare(ga["shape"][..., :2].cpu().numpy(), b["shape"][..., :2].cpu().numpy(),
            scale["shape"][..., :2], "shape", 2 * TOL)
