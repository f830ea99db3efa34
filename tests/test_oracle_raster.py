"""Pins of the FP64 compositing oracle (Section 3.1 volume-rendering sum over
projected Gaussians). Nothing here runs on the GPU."""
import numpy as np
import pytest

from oracle import raster_ref as RR

CAM = dict(R=np.eye(3), t=np.zeros(3), fx=100.0, fy=120.0, cx=32.0, cy=24.0, width=64, height=48)


def _one(mean, scale, q=(1, 0, 0, 0), sigma=0.5, color=(1.0, 0.5, 0.25)):
    return (np.array([mean], float), np.array([scale], float), np.array([q], float),
            np.array([sigma]), np.array([color]))


def test_axis_aligned_projection():
    """Scales (sx, sy, sz) at depth Z on the optical axis project to
    diag((fx sx/Z)^2, (fy sy/Z)^2)."""
    m, s, r, o, c = _one((0, 0, 5.0), (0.2, 0.3, 0.4))
    p = RR.project(m, s, r, CAM)
    np.testing.assert_allclose(p["cov2"][0], np.diag([(100 * 0.2 / 5) ** 2, (120 * 0.3 / 5) ** 2]),
                               rtol=1e-14, atol=1e-14)
    assert p["u"][0] == pytest.approx(32.0) and p["v"][0] == pytest.approx(24.0)


def test_single_gaussian_closed_form():
    """One isotropic Gaussian on the optical axis (any rotation): every pixel
    inside the 3-sigma circle gets c sigma exp(-r^2 / (2 s^2)) with
    s = f scale / Z the projected standard deviation."""
    m, s, r, o, c = _one((0.0, 0.0, 4.0), (0.1, 0.1, 0.1), q=(0.3, 0.2, -0.5, 0.1), sigma=0.7)
    cam = dict(CAM, fy=100.0, cx=31.3, cy=24.6)
    out, _ = RR.render(m, s, r, o, c, cam)
    sd = 100 * 0.1 / 4
    u, v = 31.3, 24.6
    yy, xx = np.mgrid[0:48, 0:64] + 0.5
    r2 = (xx - u) ** 2 + (yy - v) ** 2
    ref = np.where(r2 / sd ** 2 <= 9, 0.7 * np.exp(-r2 / (2 * sd * sd)), 0.0)
    np.testing.assert_allclose(out["image"], ref[..., None] * c[0], rtol=1e-12, atol=1e-15)


def test_front_primitive_occludes():
    """Two overlapping Gaussians: C = c1 a1 + c2 a2 (1 - a1), nearer first,
    whatever their index order."""
    m = np.array([[0, 0, 6.0], [0, 0, 3.0]])
    s = np.full((2, 3), 0.3)
    r = np.array([[1.0, 0, 0, 0]] * 2)
    o = np.array([0.6, 0.8])
    c = np.array([[1.0, 0, 0], [0, 1.0, 0]])
    out, _ = RR.render(m, s, r, o, c, CAM)
    # pixel at the image centre (32, 24) sampled at (32.5, 24.5)
    p = RR.project(m, s, r, CAM)
    dx, dy = 32.5 - p["u"], 24.5 - p["v"]
    q = p["a"] * dx * dx + 2 * p["b"] * dx * dy + p["c"] * dy * dy
    al = o * np.exp(-0.5 * q)
    ref = c[1] * al[1] + c[0] * al[0] * (1 - al[1])
    np.testing.assert_allclose(out["image"][24, 32], ref, rtol=1e-13)


def test_behind_camera_and_zero_opacity_leave_black():
    m = np.array([[0, 0, -3.0], [0, 0, 4.0]])
    s = np.full((2, 3), 0.3)
    r = np.array([[1.0, 0, 0, 0]] * 2)
    out, _ = RR.render(m, s, r, np.array([0.9, 0.0]), np.ones((2, 3)), CAM)
    assert np.all(out["image"] == 0)


def _scene(seed, n):
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.8, n), rng.uniform(3, 8, n)], -1)
    scales = np.exp(rng.uniform(np.log(0.03), np.log(0.3), (n, 3)))
    rots = rng.standard_normal((n, 4))
    opac = rng.uniform(0.05, 0.9, n)
    colors = rng.standard_normal((n, 3))
    return means, scales, rots, opac, colors


def test_gradients_against_finite_differences():
    means, scales, rots, opac, colors = _scene(3, 12)
    cam = dict(CAM, width=24, height=20, cx=12.0, cy=10.0, fx=30.0, fy=30.0)
    g = np.random.default_rng(4).standard_normal((20, 24, 3))
    out, scale = RR.render(means, scales, rots, opac, colors, cam, grad_image=g)

    def loss(o=opac, c=colors):
        return float((RR.render(means, scales, rots, o, c, cam)[0]["image"] * g).sum())
    h = 1e-6
    for i in range(len(opac)):
        op, om = opac.copy(), opac.copy()
        op[i] += h
        om[i] -= h
        num = (loss(o=op) - loss(o=om)) / (2 * h)
        assert abs(num - out["opac"][i]) <= 1e-7 * (scale["opac"][i] + 1e-12), i
        for k in range(3):
            cp, cm = colors.copy(), colors.copy()
            cp[i, k] += h
            cm[i, k] -= h
            num = (loss(c=cp) - loss(c=cm)) / (2 * h)
            assert abs(num - out["colors"][i, k]) <= 1e-7 * (scale["colors"][i, k] + 1e-12), (i, k)


def test_image_is_linear_in_colours():
    means, scales, rots, opac, colors = _scene(5, 30)
    a = RR.render(means, scales, rots, opac, colors, CAM)[0]["image"]
    b = RR.render(means, scales, rots, opac, 2 * colors, CAM)[0]["image"]
    np.testing.assert_allclose(b, 2 * a, rtol=1e-14, atol=1e-15)


def test_window_render_matches_crop():
    """Rendering a window with the principal point shifted by the window's
    corner, over only the primitives whose 3-sigma box meets the window,
    reproduces that window of the full render (used to check large images on
    windows)."""
    import workloads as W
    sc = W.draw_splat_scene(11, 600, 80, 60, scale=(0.05, 0.5))
    full, fs = RR.render(sc.means, sc.scales, sc.rots, sc.opac, sc.colors, sc.cam,
                         grad_image=sc.grad_image)
    x0, y0, w, h = 50, 37, 30, 23
    g = np.zeros_like(sc.grad_image)
    g[y0:y0 + h, x0:x0 + w] = sc.grad_image[y0:y0 + h, x0:x0 + w]
    masked, _ = RR.render(sc.means, sc.scales, sc.rots, sc.opac, sc.colors, sc.cam, grad_image=g)
    p = RR.project(sc.means, sc.scales, sc.rots, sc.cam)
    ex = 3 * np.sqrt(p["cov2"][:, 0, 0]) + 1
    ey = 3 * np.sqrt(p["cov2"][:, 1, 1]) + 1
    keep = p["vis"] & (p["u"] + ex >= x0) & (p["u"] - ex <= x0 + w) & \
        (p["v"] + ey >= y0) & (p["v"] - ey <= y0 + h)
    idx = np.nonzero(keep)[0]
    assert 0 < len(idx) < 600
    cam = dict(sc.cam, cx=sc.cam["cx"] - x0, cy=sc.cam["cy"] - y0, width=w, height=h)
    win, _ = RR.render(sc.means[idx], sc.scales[idx], sc.rots[idx], sc.opac[idx], sc.colors[idx],
                       cam, grad_image=sc.grad_image[y0:y0 + h, x0:x0 + w])
    np.testing.assert_allclose(win["image"], full["image"][y0:y0 + h, x0:x0 + w], rtol=1e-12,
                               atol=1e-14)
    np.testing.assert_allclose(win["colors"], masked["colors"][idx], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(win["opac"], masked["opac"][idx], rtol=1e-11, atol=1e-13)
    rest = np.ones(600, bool)
    rest[idx] = False
    assert np.all(masked["colors"][rest] == 0) and np.all(masked["opac"][rest] == 0)


def test_rotation_jacobian_against_differences():
    rng = np.random.default_rng(8)
    q = rng.standard_normal((5, 4))
    jac = RR.quat_rotation_jacobian(q)
    h = 1e-6
    for k in range(4):
        qp, qm = q.copy(), q.copy()
        qp[:, k] += h
        qm[:, k] -= h
        num = (RR.quat_rotation(qp) - RR.quat_rotation(qm)) / (2 * h)
        np.testing.assert_allclose(jac[..., k], num, rtol=1e-7, atol=1e-9)


def test_geometry_gradients_against_finite_differences():
    """dL/dmeans, dL/dscales, dL/dquaternions (through rho, with the support,
    near plane and clamp held fixed) against central differences of the
    rendered loss."""
    means, scales, rots, opac, colors = _scene(13, 10)
    cam = dict(CAM, width=24, height=20, cx=12.0, cy=10.0, fx=30.0, fy=34.0,
               R=RR.quat_rotation(np.array([[0.97, 0.1, -0.15, 0.12]]))[0], t=np.array([0.1, -0.2, 0.3]))
    g = np.random.default_rng(14).standard_normal((20, 24, 3))
    out, scale = RR.render(means, scales, rots, opac, colors, cam, grad_image=g, geometry=True)

    def loss(m=means, s=scales, r=rots):
        return float((RR.render(m, s, r, opac, colors, cam)[0]["image"] * g).sum())
    h = 1e-6
    for name, arr, kw in (("means", means, "m"), ("scales", scales, "s"), ("rots", rots, "r")):
        for i in range(arr.shape[0]):
            for k in range(arr.shape[1]):
                ap, am = arr.copy(), arr.copy()
                ap[i, k] += h
                am[i, k] -= h
                num = (loss(**{kw: ap}) - loss(**{kw: am})) / (2 * h)
                tol = 1e-6 * (np.abs(out[name][i]).max() + scale[name][i].max() + 1e-9)
                assert abs(num - out[name][i, k]) <= tol, (name, i, k, num, out[name][i, k])
