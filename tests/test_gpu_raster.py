"""GPU parity of the compositing path (Section 3.1: C = sum_i T_i alpha_i c_i
over depth-sorted projected Gaussians) and of its colour / opacity gradients,
through the C ABI against the FP64 oracle on the same seeded scenes. Bar:
scaled error <= 1e-5 (the FP32 bar of the appearance path); the kernels keep
transmittance and colour sums in FP64 and evaluate rho in FP32, so the
expected error is a few float32 ulps of the scale."""
import numpy as np
import pytest
import torch

import paper_2606_09794_amd as P
import workloads as W
from gpu_util import compare
from oracle import raster_ref as RR

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _camera(cam):
    return P.Camera(cam["R"], cam["t"], cam["fx"], cam["fy"], cam["cx"], cam["cy"],
                    cam["width"], cam["height"])


def _dev(sc):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    return [t(sc.means), t(sc.scales), t(sc.rots), t(sc.opac), t(sc.colors)]


GEOM = ("means", "scales", "rots")


def _gpu(sc, cap=1024, grad_image=None, geometry=False):
    """image, grad colours, grad opacities (and, with geometry, grad means,
    scales, rots) as numpy arrays."""
    d = _dev(sc)
    cam = _camera(sc.cam)
    img, ws = P.raster_fwd(*d, cam, cap)
    gi = torch.from_numpy(np.ascontiguousarray(sc.grad_image if grad_image is None else grad_image)).cuda()
    out = P.raster_bwd(*d, cam, ws, gi, cap, geometry=geometry)
    torch.cuda.synchronize()
    return (img.cpu().numpy(), *(t.cpu().numpy() for t in out))


def _check(sc, cap=1024, tol=TOL):
    img, gc, go, gm, gs, gr = _gpu(sc, cap, geometry=True)
    ref, scale = RR.render(sc.means, sc.scales, sc.rots, sc.opac, sc.colors, sc.cam,
                           grad_image=sc.grad_image, geometry=True)
    compare(img, ref["image"], scale["image"], "image", tol)
    compare(gc, ref["colors"], scale["colors"], "grad colors", tol)
    compare(go, ref["opac"], scale["opac"], "grad opac", tol)
    for name, v in zip(GEOM, (gm, gs, gr)):
        compare(v, ref[name], scale[name], f"grad {name}", tol)
    return img, ref


def test_ragged_image_several_tiles():
    """70 x 45 pixels: 5 x 3 tiles, the last column and row partial."""
    sc = W.draw_splat_scene(1, 400, 70, 45, scale=(0.05, 0.5))
    img, ref = _check(sc)
    assert (ref["image"] != 0).mean() > 0.5


def test_deep_overlap():
    """Large primitives: every pixel composites tens to hundreds of layers and
    the transmittance falls by many orders of magnitude."""
    sc = W.draw_splat_scene(2, 300, 48, 40, scale=(0.3, 1.0), depth=(3.0, 6.0), behind=0.0)
    p = RR.project(sc.means, sc.scales, sc.rots, sc.cam)
    yy, xx = np.mgrid[0:40, 0:48] + 0.5
    dx = xx.ravel()[:, None] - p["u"][None]
    dy = yy.ravel()[:, None] - p["v"][None]
    q = p["a"] * dx * dx + 2 * p["b"] * dx * dy + p["c"] * dy * dy
    assert (q <= 9).sum(1).max() > 100
    _check(sc)


def test_opacities_at_the_clamp():
    """Opacities near 1: alpha clamps at 0.99 near the centres, where the
    opacity gradient is zero."""
    sc = W.draw_splat_scene(3, 150, 40, 33, scale=(0.1, 0.4), opac=(0.95, 1.0))
    _check(sc)


def test_zero_and_tiny_opacities():
    """A fifth of the primitives have opacity 0 and a fifth 1e-30 (alpha is
    zero or far below every other layer): they add nothing to the image, yet
    their opacity gradient, T rho times dL/dalpha summed over their pixels, is
    of the usual size and must match the oracle, as must everything behind
    and in front of them."""
    sc = W.draw_splat_scene(4, 400, 48, 40, scale=(0.05, 0.4))
    rng = np.random.default_rng(40)
    k = rng.permutation(sc.n)
    sc.opac[k[: sc.n // 5]] = 0.0
    sc.opac[k[sc.n // 5: 2 * sc.n // 5]] = 1e-30
    img, ref = _check(sc)
    gc, go = _gpu(sc)[1:3]
    assert np.abs(go[k[: 2 * sc.n // 5]]).max() > 1e-3    # nonzero at alpha = 0


def test_nothing_visible():
    """All primitives behind the near plane: black image, zero gradients."""
    sc = W.draw_splat_scene(4, 64, 40, 30, scale=(0.1, 0.4), behind=1.0)
    img, *grads = _gpu(sc, geometry=True)
    assert np.all(img == 0) and all(np.all(v == 0) for v in grads)


def test_empty_scene():
    sc = W.draw_splat_scene(5, 0, 33, 17)
    img, gc, go, gm, gs, gr = _gpu(sc, geometry=True)
    assert img.shape == (17, 33, 3) and np.all(img == 0)
    assert gc.shape == (0, 3) and go.shape == (0,) and gr.shape == (0, 4)


def test_tile_overflow_is_reported():
    sc = W.draw_splat_scene(6, 200, 32, 32, scale=(0.3, 1.0), behind=0.0)
    d = _dev(sc)
    with pytest.raises(P.NasgError, match="tile"):
        P.raster_fwd(*d, _camera(sc.cam), 8)


def test_backward_repeats_and_matches_autograd():
    """The backward may be called again on the same workspace; the autograd
    wrapper returns the same gradients."""
    sc = W.draw_splat_scene(7, 300, 64, 48, scale=(0.05, 0.5))
    d = _dev(sc)
    cam = _camera(sc.cam)
    img, ws = P.raster_fwd(*d, cam)
    gi = torch.from_numpy(sc.grad_image).cuda()
    a = P.raster_bwd(*d, cam, ws, gi)
    b = P.raster_bwd(*d, cam, ws, gi)
    op = d[3].clone().requires_grad_(True)
    col = d[4].clone().requires_grad_(True)
    geo = [t.clone().requires_grad_(True) for t in d[:3]]
    out = P.Rasterize.apply(*geo, op, col, cam)
    (out * gi).sum().backward()
    ag = P.raster_bwd(*d, cam, ws, gi, geometry=True)
    torch.cuda.synchronize()
    assert torch.equal(out, img)
    for x, y in ((a[0], b[0]), (a[1], b[1]), (a[0], col.grad), (a[1], op.grad), (ag[0], a[0]),
                 (ag[2], geo[0].grad), (ag[3], geo[1].grad), (ag[4], geo[2].grad)):
        assert torch.allclose(x, y, rtol=1e-6, atol=1e-7)


def _window_oracle(sc, x0, y0, w, h):
    """The oracle on a window of the image: a camera with the principal point
    shifted, over the primitives whose 3-sigma box (plus one pixel) meets the
    window; the others have q > 9 on every window pixel and add nothing."""
    p = RR.project(sc.means, sc.scales, sc.rots, sc.cam)
    ex = 3 * np.sqrt(p["cov2"][:, 0, 0]) + 1
    ey = 3 * np.sqrt(p["cov2"][:, 1, 1]) + 1
    keep = p["vis"] & (p["u"] + ex >= x0) & (p["u"] - ex <= x0 + w) & \
        (p["v"] + ey >= y0) & (p["v"] - ey <= y0 + h)
    idx = np.nonzero(keep)[0]
    cam = dict(sc.cam, cx=sc.cam["cx"] - x0, cy=sc.cam["cy"] - y0, width=w, height=h)
    g = sc.grad_image[y0:y0 + h, x0:x0 + w]
    out, scale = RR.render(sc.means[idx], sc.scales[idx], sc.rots[idx], sc.opac[idx],
                           sc.colors[idx], cam, grad_image=g, geometry=True)
    return idx, out, scale


@pytest.mark.parametrize("win", [(700, 400, 40, 24), (1890, 1064, 30, 16)])
def test_full_size_windows(win):
    """3 M primitives at 1920 x 1080 (about 2200 per tile), the size the
    training-view benchmark runs: the image on a window, and the gradients of
    a loss whose upstream gradient lives on that window only, against the
    oracle on the window (the second window touches the image's corner)."""
    x0, y0, w, h = win
    sc = W.draw_splat_scene(8, 3_000_000, 1920, 1080)
    g = np.zeros_like(sc.grad_image)
    g[y0:y0 + h, x0:x0 + w] = sc.grad_image[y0:y0 + h, x0:x0 + w]
    img, gc, go, gm, gs, gr = _gpu(sc, cap=4096, grad_image=g, geometry=True)
    idx, ref, scale = _window_oracle(sc, x0, y0, w, h)
    assert len(idx) > 500
    compare(img[y0:y0 + h, x0:x0 + w], ref["image"], scale["image"], "image window", TOL)
    compare(gc[idx], ref["colors"], scale["colors"], "grad colors", TOL)
    compare(go[idx], ref["opac"], scale["opac"], "grad opac", TOL)
    for name, v in zip(GEOM, (gm, gs, gr)):
        compare(v[idx], ref[name], scale[name], f"grad {name}", TOL)
    rest = np.ones(sc.n, bool)
    rest[idx] = False
    for v in (gc, go, gm, gs, gr):
        assert np.all(v[rest] == 0)


def test_training_view_chain():
    """One training view end to end: each primitive's NASGabor colour along
    its central ray for this camera (Section 5.2), composited (Section 3.1),
    and the loss gradient carried back through the compositing into the lobe
    parameters, c0 and the means. The oracle chains its own two stages; the
    error scales compose the stages' scales (an image scale that also covers
    the colours' rounding, and lobe-gradient scales taken with the colour
    gradient's scale as the upstream gradient)."""
    from oracle import nasg_ref as R
    sc = W.draw_splat_scene(9, 500, 64, 48, scale=(0.05, 0.5))
    w = W.draw_workload(9, 500, 4, 1, with_sh=False)
    cam = _camera(sc.cam)
    o = cam.centre("cpu").numpy()                     # the float32 centre both sides use
    d = _dev(sc)
    lob = [torch.from_numpy(x).cuda().requires_grad_(True) for x in (w.quat, w.shape, w.rgbw, w.c0)]
    means = d[0].clone().requires_grad_(True)
    op = d[3].clone().requires_grad_(True)
    img = P.render_view(*lob, means, d[1], d[2], op, cam)
    gi = torch.from_numpy(sc.grad_image).cuda()
    (img * gi).sum().backward()
    torch.cuda.synchronize()

    rgb, s_rgb, _ = R.forward(w.quat, w.shape, w.rgbw, w.c0, R.NORM_EXACT, means=sc.means, cams=o)
    ref, scale = RR.render(sc.means, sc.scales, sc.rots, sc.opac, rgb[0], sc.cam,
                           grad_image=sc.grad_image)
    _, s_col = RR.render(sc.means, sc.scales, sc.rots, sc.opac, s_rgb[0], sc.cam)
    compare(img.detach().cpu().numpy(), ref["image"], scale["image"] + s_col["image"], "image", TOL)
    compare(op.grad.cpu().numpy(), ref["opac"], scale["opac"], "grad opac", TOL)
    gl, _ = R.forward_backward(w.quat, w.shape, w.rgbw, w.c0, ref["colors"][None], R.NORM_EXACT,
                               means=sc.means, cams=o)
    _, sl = R.forward_backward(w.quat, w.shape, w.rgbw, w.c0, scale["colors"][None], R.NORM_EXACT,
                               means=sc.means, cams=o)
    for name, t in zip(("quat", "shape", "rgbw", "c0"), lob):
        compare(t.grad.cpu().numpy(), gl[name], sl[name], f"grad {name}", TOL)
    # the means move the view direction (appearance) and the projection
    # (compositing); the colours' own rounding enters the latter through a
    # scale taken with the appearance scale in place of the colours
    gref, gscale = RR.render(sc.means, sc.scales, sc.rots, sc.opac, rgb[0], sc.cam,
                             grad_image=sc.grad_image, geometry=True)
    _, gscale2 = RR.render(sc.means, sc.scales, sc.rots, sc.opac, s_rgb[0], sc.cam,
                           grad_image=sc.grad_image, geometry=True)
    compare(means.grad.cpu().numpy(), gl["means"] + gref["means"],
            sl["means"] + gscale["means"] + gscale2["means"], "grad means", TOL)


def test_depth_ties_and_float_equal_depths():
    """Depths that are exactly equal (ordered by index) and depths closer than
    a float32 ulp (equal once rounded to float32, so the sort's FP64 tie pass
    decides) must composite in the oracle's (depth, index) order. The camera
    is turned by 1e-6 rad about its y axis, so the camera depth of a mean at
    z = 4 varies by under 1e-6 with x; half of the x values repeat exactly."""
    rng = np.random.default_rng(21)
    n = 600
    x = rng.uniform(-0.8, 0.8, n)
    x[: n // 2] = rng.choice(x[n // 2: n // 2 + 8], n // 2)
    z = np.where(rng.random(n) < 0.8, 4.0, 5.0)
    means = np.stack([x, rng.uniform(-0.6, 0.6, n), z], -1).astype(np.float32)
    th = 1e-6
    R = np.array([[np.cos(th), 0.0, np.sin(th)], [0.0, 1.0, 0.0], [-np.sin(th), 0.0, np.cos(th)]])
    cam = dict(R=R, t=np.zeros(3), fx=60.0, fy=60.0, cx=32.0, cy=24.0, width=64, height=48)
    sc = W.SplatScene(means=means,
                      scales=np.exp(rng.uniform(np.log(0.05), np.log(0.3), (n, 3))).astype(np.float32),
                      rots=rng.standard_normal((n, 4)).astype(np.float32),
                      opac=rng.uniform(0.1, 0.8, n).astype(np.float32),
                      colors=rng.standard_normal((n, 3)).astype(np.float32),
                      grad_image=rng.standard_normal((48, 64, 3)).astype(np.float32), cam=cam)
    p = RR.project(sc.means, sc.scales, sc.rots, cam)
    zf = p["z"].astype(np.float32)
    assert len(np.unique(p["z"])) > 2 * len(np.unique(zf))      # many float-equal depths
    assert len(np.unique(p["z"])) < n                             # and exact ties
    _check(sc)


def test_bucket_sort_tiles_with_float_equal_depths():
    """Tiles of 257 to 4096 entries whose depths spread over many float values
    take the bucket sort (no bucket overflows into the network); here a third
    of the primitives repeat another one's z, so under the 1e-6 rad camera
    tilt the lists hold exact ties and depths equal only once rounded to
    float32, which must still composite in the oracle's (depth, index) order."""
    rng = np.random.default_rng(22)
    n = 3000
    z = rng.uniform(3.0, 9.0, n)
    z[: n // 3] = rng.choice(z[n // 3:], n // 3)
    x = rng.uniform(-2.0, 2.0, n) * z / 4.0
    y = rng.uniform(-1.5, 1.5, n) * z / 4.0
    means = np.stack([x, y, z], -1).astype(np.float32)
    th = 1e-6
    R = np.array([[np.cos(th), 0.0, np.sin(th)], [0.0, 1.0, 0.0], [-np.sin(th), 0.0, np.cos(th)]])
    cam = dict(R=R, t=np.zeros(3), fx=60.0, fy=60.0, cx=32.0, cy=24.0, width=64, height=48)
    sc = W.SplatScene(means=means,
                      scales=np.exp(rng.uniform(np.log(0.1), np.log(0.3), (n, 3))).astype(np.float32),
                      rots=rng.standard_normal((n, 4)).astype(np.float32),
                      opac=rng.uniform(0.05, 0.6, n).astype(np.float32),
                      colors=rng.standard_normal((n, 3)).astype(np.float32),
                      grad_image=rng.standard_normal((48, 64, 3)).astype(np.float32), cam=cam)
    p = RR.project(sc.means, sc.scales, sc.rots, cam)
    zf = p["z"][p["vis"]].astype(np.float32)
    assert len(np.unique(zf)) < p["vis"].sum()                     # float-equal depths
    tiles = np.bincount((p["v"][p["vis"]] // 16).astype(int).clip(0, 2) * 4 +
                        (p["u"][p["vis"]] // 16).astype(int).clip(0, 3), minlength=12)
    assert tiles.max() > 256                                       # tiles past the network's first size
    _check(sc, cap=4096)


@pytest.mark.parametrize("n", [1500, 3000])
def test_network_sort_for_crowded_depths(n):
    """Every primitive at exactly the same depth in a 32 x 32 image (four
    tiles, each reached by nearly all of them): the bucket sort cannot split
    the depths and leaves the tiles to the bitonic network, here with
    1025-2048 and 2049-4096 keys (8 and 16 keys per thread); equal depths
    composite in index order, as in the oracle."""
    rng = np.random.default_rng(50 + n)
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), np.full(n, 4.0)],
                     -1).astype(np.float32)
    cam = dict(R=np.eye(3), t=np.zeros(3), fx=40.0, fy=40.0, cx=16.0, cy=16.0, width=32, height=32)
    sc = W.SplatScene(means=means,
                      scales=np.exp(rng.uniform(np.log(0.3), np.log(0.6), (n, 3))).astype(np.float32),
                      rots=rng.standard_normal((n, 4)).astype(np.float32),
                      opac=rng.uniform(0.01, 0.05, n).astype(np.float32),
                      colors=rng.standard_normal((n, 3)).astype(np.float32),
                      grad_image=rng.standard_normal((32, 32, 3)).astype(np.float32), cam=cam)
    p = RR.project(sc.means, sc.scales, sc.rots, cam)
    assert p["vis"].all() and len(np.unique(p["z"])) == 1
    _check(sc, cap=4096)


def test_graph_replays_match_eager():
    """Both compositing calls allocate, copy and synchronise nothing: captured
    into a graph (with their output buffers), replays with eager work and
    poisoned outputs in between reproduce the eager results (the image
    exactly; the gradients up to the order of their FP64 atomic sums)."""
    sc = W.draw_splat_scene(31, 400, 80, 56, scale=(0.05, 0.5))
    d = _dev(sc)
    cam = _camera(sc.cam)
    gi = torch.from_numpy(sc.grad_image).cuda()
    cap = 512
    ws = torch.empty(P.raster_workspace_bytes(sc.n, cam, cap), dtype=torch.uint8, device="cuda")

    def run():
        img, _ = P.raster_fwd(*d, cam, cap, workspace=ws, check_overflow=False)
        gc, go = P.raster_bwd(*d, cam, ws, gi, cap)
        return img, gc, go

    eager = [x.clone() for x in run()]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = run()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(outs[0], eager[0]), rep
        for o, e in zip(outs[1:], eager[1:]):
            assert torch.allclose(o, e, rtol=1e-6, atol=1e-9), rep


def test_widest_image_on_windows():
    """The widest image the boundary accepts (32 768 pixels, 2 048 tiles in a
    row) with 60 000 primitives: windows at the left edge, the middle and the
    right edge against the oracle."""
    width, height = 32768, 24
    sc = W.draw_splat_scene(32, 60_000, width, height, scale=(1e-4, 1e-3))
    img, gc, go = _gpu(sc, cap=1024)
    for x0 in (0, width // 2 - 20, width - 40):
        w, h = 40, height
        g = np.zeros_like(sc.grad_image)
        g[:, x0:x0 + w] = sc.grad_image[:, x0:x0 + w]
        img_w, gc_w, go_w, gm_w, gs_w, gr_w = _gpu(sc, cap=1024, grad_image=g, geometry=True)
        idx, ref, scale = _window_oracle(sc, x0, 0, w, h)
        assert len(idx) > 20
        compare(img[:, x0:x0 + w], ref["image"], scale["image"], f"image window x0={x0}", TOL)
        compare(gc_w[idx], ref["colors"], scale["colors"], f"grad colors x0={x0}", TOL)
        compare(go_w[idx], ref["opac"], scale["opac"], f"grad opac x0={x0}", TOL)
        for name, v in zip(GEOM, (gm_w, gs_w, gr_w)):
            compare(v[idx], ref[name], scale[name], f"grad {name} x0={x0}", TOL)


@pytest.mark.parametrize("width,height,classes", [(2560, 1440, 2), (3840, 2160, 4), (5120, 2880, 8)])
def test_binning_tile_classes_on_windows(width, height, classes):
    """Images of 14 400, 32 400 and 57 600 tiles: binning splits the tiles
    into 2, 4 and 8 classes so that each fits the LDS counters (8192 tiles
    per class). 300 000 primitives; two windows, one at the far corner,
    against the oracle."""
    tiles = ((width + 15) // 16) * ((height + 15) // 16)
    assert (tiles - 1) // classes + 1 <= 8192 < (tiles - 1) // (classes // 2) + 1
    sc = W.draw_splat_scene(34 + classes, 300_000, width, height, scale=(1e-3, 1e-2))
    img, gc, go = _gpu(sc, cap=1024)
    for x0, y0 in ((width // 3, height // 2), (width - 48, height - 32)):
        w, h = 48, 32
        g = np.zeros_like(sc.grad_image)
        g[y0:y0 + h, x0:x0 + w] = sc.grad_image[y0:y0 + h, x0:x0 + w]
        img_w, gc_w, go_w, gm_w, gs_w, gr_w = _gpu(sc, cap=1024, grad_image=g, geometry=True)
        idx, ref, scale = _window_oracle(sc, x0, y0, w, h)
        assert len(idx) > 20
        at = f"{width}x{height} x0={x0} y0={y0}"
        compare(img[y0:y0 + h, x0:x0 + w], ref["image"], scale["image"], f"image window {at}", TOL)
        compare(gc_w[idx], ref["colors"], scale["colors"], f"grad colors {at}", TOL)
        compare(go_w[idx], ref["opac"], scale["opac"], f"grad opac {at}", TOL)
        for name, v in zip(GEOM, (gm_w, gs_w, gr_w)):
            compare(v[idx], ref[name], scale[name], f"grad {name} {at}", TOL)


def test_many_tiles_on_windows():
    """An 8192 x 4352 image (512 x 272 = 139 264 tiles, more than the binning
    pass counts per tile class in LDS, so it takes the per-entry path) with
    400 000 primitives: windows at two corners and inside against the oracle."""
    width, height = 8192, 4352
    sc = W.draw_splat_scene(33, 400_000, width, height, scale=(1e-3, 1e-2))
    img, gc, go = _gpu(sc, cap=1024)
    for x0, y0 in ((0, 0), (3000, 2100), (width - 64, height - 48)):
        w, h = 64, 48
        g = np.zeros_like(sc.grad_image)
        g[y0:y0 + h, x0:x0 + w] = sc.grad_image[y0:y0 + h, x0:x0 + w]
        img_w, gc_w, go_w, gm_w, gs_w, gr_w = _gpu(sc, cap=1024, grad_image=g, geometry=True)
        idx, ref, scale = _window_oracle(sc, x0, y0, w, h)
        assert len(idx) > 20
        at = f"x0={x0} y0={y0}"
        compare(img[y0:y0 + h, x0:x0 + w], ref["image"], scale["image"], f"image window {at}", TOL)
        compare(gc_w[idx], ref["colors"], scale["colors"], f"grad colors {at}", TOL)
        compare(go_w[idx], ref["opac"], scale["opac"], f"grad opac {at}", TOL)
        for name, v in zip(GEOM, (gm_w, gs_w, gr_w)):
            compare(v[idx], ref[name], scale[name], f"grad {name} {at}", TOL)


def test_gradient_descent_lowers_photometric_loss():
    """The gradients train: from a perturbed copy of a scene (lobes, c0,
    opacities, means, scales, rotations), Adam on the squared difference to
    the original scene's image, rendered through the appearance evaluation
    and the compositing, lowers the loss well below its start."""
    sc = W.draw_splat_scene(40, 300, 64, 48, scale=(0.05, 0.3), behind=0.0)
    w = W.draw_workload(40, 300, 4, 1, with_sh=False)
    cam = _camera(sc.cam)
    d = _dev(sc)
    lob = [torch.from_numpy(x).cuda() for x in (w.quat, w.shape, w.rgbw, w.c0)]
    with torch.no_grad():
        target = P.render_view(*lob, d[0], d[1], d[2], d[3], cam)
    gen = torch.Generator(device="cuda").manual_seed(0)
    noisy = lambda t, s: (t + s * torch.randn(t.shape, device="cuda", generator=gen)).contiguous()  # noqa: E731
    params = [noisy(lob[0], 0.2), lob[1].clone(), noisy(lob[2], 0.2), noisy(lob[3], 0.2),
              noisy(d[0], 0.02), d[1].clone(), noisy(d[2], 0.2), (d[3] * 0.7).contiguous()]
    for t in params:
        t.requires_grad_(True)
    opt = torch.optim.Adam([params[i] for i in (0, 2, 3, 4, 6, 7)], lr=5e-3)
    losses = []
    for _ in range(40):
        opt.zero_grad()
        img = P.render_view(*params[:4], *params[4:], cam)
        loss = ((img - target) ** 2).sum()
        loss.backward()
        opt.step()
        with torch.no_grad():
            params[7].clamp_(0.0, 1.0)
        losses.append(float(loss.detach()))
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses[::8]


def test_backward_without_matching_forward_computes_nothing():
    """A backward on a workspace holding no forward of the same sizes (never
    run, or run with another tile capacity) is caught on the device before any
    tile list is read: zero gradients and the stale flag set; the matching
    backward clears the flag."""
    sc = W.draw_splat_scene(50, 200, 48, 40, scale=(0.05, 0.4))
    d = _dev(sc)
    cam = _camera(sc.cam)
    gi = torch.from_numpy(sc.grad_image).cuda()
    ws = torch.zeros(P.raster_workspace_bytes(sc.n, cam, 512), dtype=torch.uint8, device="cuda")
    stale = lambda: int(ws[4:8].view(torch.int32).item())  # noqa: E731
    out = P.raster_bwd(*d, cam, ws, gi, 512, geometry=True)
    torch.cuda.synchronize()
    assert stale() == 1 and all(bool(torch.all(t == 0)) for t in out)
    P.raster_fwd(*d, cam, 256, workspace=ws)
    out = P.raster_bwd(*d, cam, ws, gi, 512)
    torch.cuda.synchronize()
    assert stale() == 1 and all(bool(torch.all(t == 0)) for t in out)
    out = P.raster_bwd(*d, cam, ws, gi, 256)
    torch.cuda.synchronize()
    assert stale() == 0 and bool(torch.any(out[0] != 0))
