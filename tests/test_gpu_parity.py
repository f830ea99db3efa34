"""GPU parity: the HIP kernels (through the C ABI) against the FP64 oracle on
the same seeded inputs. Error metric: |y - y_ref| / S with S the sum of the
absolute elementary terms of y_ref (oracle.metrics); FP32 bar 1e-5."""
import numpy as np
import pytest
import torch

import paper_2606_09794_amd as P
import workloads as W
from gpu_util import compare, dgeo, oracle_nasg, oracle_sh, upload

pytestmark = pytest.mark.gpu
TOL = 1e-5
CONFIGS = [(1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2), (4, 4), (8, 1), (8, 2),
           (16, 1)]


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for kern in range(4):
        for k in (0, 4, 8, 16):
            for v in (1, 2, 3, 4, 5, 8, 16, 37):
                for dt in (0, 1):
                    P.set_tuning(kern, k, v, dt, 0, 0)


def _run_nasg(d, norm, fused=True):
    g = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], norm=norm,
                        rgb_out=torch.empty_like(d["grad_rgb"]) if fused else None, **dgeo(d))
    torch.cuda.synchronize()
    return g


def _check_nasg(w, norm, tol=TOL, fused=True):
    d = upload(w)
    rgb = P.nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], norm=norm, **dgeo(d))
    rgb_f = torch.empty_like(rgb)
    g = P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"], norm=norm,
                        rgb_out=rgb_f if fused else None, **dgeo(d))
    torch.cuda.synchronize()
    ref, scale = oracle_nasg(w, norm)
    rep = {"rgb": compare(rgb.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb", tol)}
    if fused:
        compare(rgb_f.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb (fused)", tol)
    for name in ("quat", "shape", "rgbw", "c0", "geom"):
        rep[name] = compare(g[name].cpu().numpy(), ref[name], scale[name], name, tol)
    return rep


@pytest.mark.parametrize("norm", ["exact", "approx"])
def test_config0_forward_and_backward(norm):
    """4096 primitives, K = 4, one raw direction each (seed 0)."""
    _check_nasg(W.config0(), norm)


@pytest.mark.parametrize("norm", ["exact", "approx"])
def test_single_camera_k8_ragged(norm):
    """Config-1 shape at a ragged size: K = 8, one camera, 3001 primitives."""
    _check_nasg(W.draw_workload(1, 3001, 8, 1), norm)


@pytest.mark.parametrize("norm", ["exact", "approx"])
def test_sixteen_views_k8(norm):
    """Config-2 shape at 1500 primitives: K = 8, V = 16 in one launch."""
    _check_nasg(W.draw_workload(2, 1500, 8, 16), norm)


@pytest.mark.parametrize("lanes,vpl", CONFIGS)
def test_every_lane_mapping(lanes, vpl):
    """Each compiled (lanes, views-per-lane) pair, with V = 5 (ragged against
    every mapping and, for small lanes*vpl, several view chunks)."""
    w = W.draw_workload(30 + lanes * 10 + vpl, 333, 3, 5)
    for kern in (0, 1):
        P.set_tuning(kern, 3, 5, 0, lanes, vpl)
    _check_nasg(w, "exact")


def test_many_views_chunked():
    """V = 37 > lanes * views-per-lane: view chunks accumulate in place."""
    _check_nasg(W.draw_workload(7, 200, 4, 37), "exact")


def test_bf16_storage_against_dequantised_oracle():
    """Lobe parameters stored as bfloat16 (K = 16, V = 8): the oracle sees the
    dequantised values; FP32 arithmetic gives the FP32 bar."""
    w = W.draw_workload(3, 700, 16, 8, dtype="bf16")
    _check_nasg(w, "exact")
    _check_nasg(w, "approx")


def test_accumulate_and_view_split_equivalence():
    """16 single-view launches in ACCUMULATE mode equal one 16-view launch."""
    w = W.draw_workload(5, 900, 8, 16)
    d = upload(w)
    full = _run_nasg(d, "exact", fused=False)
    acc = P.nasg_grad_buffers(8, w.n, "cuda")
    for t in acc.values():
        t.zero_()
    for v in range(16):
        P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"][v:v + 1].contiguous(),
                        means=d["means"], cams=d["cams"][v:v + 1].contiguous(), norm="exact",
                        grads=acc, accumulate=True)
    torch.cuda.synchronize()
    ref, scale = oracle_nasg(w, "exact")
    for name in ("quat", "shape", "rgbw", "c0", "geom"):
        compare(acc[name].cpu().numpy(), ref[name], scale[name], name, TOL)
        compare(acc[name].cpu().numpy(), full[name].cpu().numpy(), scale[name], name, 2 * TOL)


def test_deterministic():
    w = W.draw_workload(6, 2000, 8, 16)
    d = upload(w)
    a = {k: v.clone() for k, v in _run_nasg(d, "exact").items()}
    b = _run_nasg(d, "exact")
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_poles_exact():
    """d = +z gives N (1 + cos zeta)/2; d = -z gives 0 with zero gradients."""
    w = W.draw_workload(8, 4, 1, 1, dirs_mode=True)
    w.quat[:] = np.array([1, 0, 0, 0], np.float32)
    w.dirs[:] = np.array([[0, 0, 2], [0, 0, -3], [0, 0, 1], [0, 0, -1]], np.float32)
    _check_nasg(w, "exact")
    _check_nasg(w, "approx")


def test_empty_input_is_noop():
    w = W.draw_workload(9, 5, 2, 3)
    d = upload(w)
    e = {k: (v[..., :0] if k in ("rgbw",) else v[:, :0] if k in ("quat", "shape") else
             v[:0] if k in ("c0", "means") else v) for k, v in d.items() if v is not None}
    out = torch.full((3, 0, 3), 7.0, device="cuda")
    P.nasg_eval_fwd(e["quat"].contiguous(), e["shape"].contiguous(), e["rgbw"].contiguous(),
                    e["c0"].contiguous(), means=e["means"].contiguous(), cams=e["cams"], out=out)
    torch.cuda.synchronize()


@pytest.mark.parametrize("lanes,vpl", [(1, 1), (4, 4), (16, 1)])
def test_sh3_forward_backward(lanes, vpl):
    w = W.draw_workload(10, 1234, 1, 16)
    for kern in (2, 3):
        P.set_tuning(kern, 0, 16, 0, lanes, vpl)
    d = upload(w)
    rgb = P.sh3_eval_fwd(d["sh"], means=d["means"], cams=d["cams"])
    rgb_f = torch.empty_like(rgb)
    g = P.sh3_eval_bwd(d["sh"], d["grad_rgb"], means=d["means"], cams=d["cams"], rgb_out=rgb_f)
    torch.cuda.synchronize()
    ref, scale = oracle_sh(w)
    compare(rgb.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb", TOL)
    # the fused kernel is a different instruction stream: equal up to rounding
    compare(rgb_f.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb (fused)", TOL)
    compare(rgb_f.cpu().numpy(), rgb.cpu().numpy(), scale["rgb"], "rgb fused vs forward", 2 * TOL)
    compare(g["sh"].cpu().numpy(), ref["sh"], scale["sh"], "sh", TOL)
    compare(g["geom"].cpu().numpy(), ref["geom"], scale["geom"], "geom", TOL)


def test_sh3_config0_directions():
    w = W.config0()
    d = upload(w)
    g = P.sh3_eval_bwd(d["sh"], d["grad_rgb"], dirs=d["dirs"], rgb_out=torch.empty_like(d["grad_rgb"]))
    rgb = P.sh3_eval_fwd(d["sh"], dirs=d["dirs"])
    torch.cuda.synchronize()
    ref, scale = oracle_sh(w)
    compare(rgb.cpu().numpy(), ref["rgb"], scale["rgb"], "rgb", TOL)
    compare(g["sh"].cpu().numpy(), ref["sh"], scale["sh"], "sh", TOL)
    compare(g["geom"].cpu().numpy(), ref["geom"], scale["geom"], "geom", TOL)


def test_autograd_function():
    w = W.draw_workload(12, 300, 4, 4)
    d = upload(w)
    leaves = {k: d[k].clone().requires_grad_(True) for k in ("quat", "shape", "rgbw", "c0", "means")}
    rgb = P.NasgEval.apply(leaves["quat"], leaves["shape"], leaves["rgbw"], leaves["c0"],
                           leaves["means"], d["cams"], None, "exact")
    (rgb * d["grad_rgb"]).sum().backward()
    ref, scale = oracle_nasg(w, "exact")
    for k in ("quat", "shape", "rgbw", "c0"):
        compare(leaves[k].grad.cpu().numpy(), ref[k], scale[k], k, TOL)
    compare(leaves["means"].grad.cpu().numpy(), ref["geom"], scale["geom"], "means", TOL)


def test_eval_calls_replay_from_a_graph():
    """The single-scene calls allocate, copy and synchronise nothing:
    nasg_eval_fwd, nasg_eval_bwd (fused) and the SH pair captured into one
    graph replay bitwise equal to the eager run (they use no atomics), with
    eager work and poisoned outputs between replays."""
    w = W.draw_workload(61, 3000, 8, 16)
    d = upload(w)
    g = P.nasg_grad_buffers(w.k, w.n, "cuda")
    rgb = torch.empty_like(d["grad_rgb"])
    rgb2 = torch.empty_like(d["grad_rgb"])
    rgb_sh = torch.empty_like(d["grad_rgb"])
    gsh = {"sh": torch.empty_like(d["sh"]), "geom": torch.empty((w.n, 3), device="cuda")}
    outs = [rgb, rgb2, rgb_sh, *g.values(), *gsh.values()]

    def run():
        P.nasg_eval_fwd(d["quat"], d["shape"], d["rgbw"], d["c0"], means=d["means"],
                        cams=d["cams"], out=rgb)
        P.nasg_eval_bwd(d["quat"], d["shape"], d["rgbw"], d["c0"], d["grad_rgb"],
                        means=d["means"], cams=d["cams"], grads=g, rgb_out=rgb2)
        P.sh3_eval_bwd(d["sh"], d["grad_rgb"], means=d["means"], cams=d["cams"], grads=gsh,
                       rgb_out=rgb_sh)

    run()
    torch.cuda.synchronize()
    eager = [t.clone() for t in outs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for k, (t, e) in enumerate(zip(outs, eager)):
            assert torch.equal(t, e), (rep, k)


def test_sh3_autograd_function():
    """SH3Eval: forward through sh3_eval_fwd, backward through sh3_eval_bwd,
    in camera mode (gradient to sh and means) and direction mode (sh, dirs)."""
    w = W.draw_workload(14, 400, 1, 4)
    d = upload(w)
    sh = d["sh"].clone().requires_grad_(True)
    means = d["means"].clone().requires_grad_(True)
    rgb = P.SH3Eval.apply(sh, means, d["cams"], None)
    (rgb * d["grad_rgb"]).sum().backward()
    ref, scale = oracle_sh(w)
    compare(rgb.detach().cpu().numpy(), ref["rgb"], scale["rgb"], "rgb", TOL)
    compare(sh.grad.cpu().numpy(), ref["sh"], scale["sh"], "sh", TOL)
    compare(means.grad.cpu().numpy(), ref["geom"], scale["geom"], "means", TOL)
    w0 = W.config0()
    d0 = upload(w0)
    sh0 = d0["sh"].clone().requires_grad_(True)
    dirs = d0["dirs"].clone().requires_grad_(True)
    rgb0 = P.SH3Eval.apply(sh0, None, None, dirs)
    (rgb0 * d0["grad_rgb"]).sum().backward()
    ref0, scale0 = oracle_sh(w0)
    compare(sh0.grad.cpu().numpy(), ref0["sh"], scale0["sh"], "sh (dirs)", TOL)
    compare(dirs.grad.cpu().numpy(), ref0["geom"], scale0["geom"], "dirs", TOL)


def test_output_buffers_are_shape_checked():
    """Caller-supplied outputs of the wrong shape, dtype or device are refused
    on the host before any launch."""
    w = W.draw_workload(15, 64, 2, 3)
    d = upload(w)
    base = dict(means=d["means"], cams=d["cams"])
    lob = (d["quat"], d["shape"], d["rgbw"], d["c0"])
    with pytest.raises(ValueError):
        P.nasg_eval_fwd(*lob, out=torch.empty((1, 64, 3), device="cuda"), **base)
    with pytest.raises(ValueError):
        P.nasg_eval_fwd(*lob, out=torch.empty((3, 64, 3), device="cuda", dtype=torch.float64), **base)
    with pytest.raises(ValueError):
        P.nasg_eval_fwd(*lob, out=torch.empty((3, 64, 3)), **base)
    g = P.nasg_grad_buffers(2, 64, "cuda")
    bad = dict(g, quat=torch.empty((2, 63, 4), device="cuda"))
    with pytest.raises(ValueError):
        P.nasg_eval_bwd(*lob, d["grad_rgb"], grads=bad, **base)
    bad = dict(g, rgbw=torch.empty((2, 64, 3), device="cuda"))
    with pytest.raises(ValueError):
        P.nasg_eval_bwd(*lob, d["grad_rgb"], grads=bad, **base)
    with pytest.raises(ValueError):
        P.nasg_eval_bwd(*lob, d["grad_rgb"], grads=g, rgb_out=torch.empty((1, 64, 3), device="cuda"),
                        **base)
    with pytest.raises(ValueError):
        P.sh3_eval_bwd(d["sh"], d["grad_rgb"], grads={"sh": torch.empty((16, 3, 63), device="cuda")},
                       **base)
    with pytest.raises(ValueError):
        P.sh3_eval_bwd(d["sh"], d["grad_rgb"], grads={"geom": torch.empty((64, 3))}, **base)
    with pytest.raises(ValueError):
        P.sh3_eval_bwd(d["sh"][:15].contiguous(), d["grad_rgb"], **base)
    with pytest.raises(ValueError):
        P.sh3_eval_fwd(d["sh"], out=torch.empty((3, 64, 2), device="cuda"), **base)
    sc = dict(d, grads=dict(g, c0=torch.empty((65, 3), device="cuda")), rgb=None)
    with pytest.raises(ValueError):
        P.NasgBatchPlan([sc])
    sc = dict(d, grads=g, rgb=torch.empty((2, 64, 3), device="cuda"))
    with pytest.raises(ValueError):
        P.NasgBatchPlan([sc])
    torch.cuda.synchronize()
