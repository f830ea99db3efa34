"""Pins of the FP64 oracle for the paper's own lobe parametrisation
(Supplementary C: frame from three cosines, activation table; Supplementary F:
frame derivatives). Nothing here runs on the GPU."""
import numpy as np
import pytest

import workloads as W
from oracle import nasg_paper as Pp
from oracle import nasg_ref as R


def _raw_lobes(seed, k, n, spread=1.0):
    rng = np.random.default_rng(seed)
    frame = np.zeros((k, n, 4))
    frame[..., :3] = spread * rng.standard_normal((k, n, 3))
    shape = np.stack([rng.uniform(-0.7, 2.5, (k, n)), rng.uniform(-2.0, 1.8, (k, n)),
                      rng.uniform(-2.0, 0.0, (k, n)), rng.uniform(0, 2 * np.pi, (k, n))], -1)
    rgbw = 0.8 * rng.standard_normal((k, 3, n))
    return frame, shape, rgbw


def test_activation_ranges():
    frame, shape, rgbw = _raw_lobes(1, 4, 500, spread=4.0)
    shape[..., 2] = np.linspace(-30, 30, shape[..., 2].size).reshape(shape[..., 2].shape)
    cos, act, w = Pp.activate(frame, shape, rgbw)
    assert np.all(np.abs(cos) <= 1) and np.all(np.abs(w) <= 1)
    assert np.all(act[..., 0] > 0) and np.all(act[..., 1] > 0)
    assert np.all((act[..., 2] >= 0) & (act[..., 2] <= 40))
    np.testing.assert_array_equal(act[..., 3], shape[..., 3])     # phase passes through


def test_frame_orthonormal_right_handed():
    frame, shape, rgbw = _raw_lobes(2, 3, 400, spread=2.0)
    cos, _, _ = Pp.activate(frame, shape, rgbw)
    x, y, z = Pp.frame_from_cosines(cos)
    m = np.stack([x, y, z], -1)
    eye = np.einsum("...ji,...jk->...ik", m, m)
    np.testing.assert_allclose(eye, np.broadcast_to(np.eye(3), eye.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(m), 1.0, atol=1e-13)


def test_frame_is_spherical_direction_and_tangent_rotation():
    """z is the unit vector at polar angle phi and azimuth theta; x is the
    meridian tangent dz/dphi turned by psi about z (Rodrigues), computed here
    from the angles with cos/sin rather than from the sqrt form."""
    frame, shape, rgbw = _raw_lobes(3, 2, 300, spread=2.0)
    cos, _, _ = Pp.activate(frame, shape, rgbw)
    th, ph, ps = np.arccos(cos[..., 0]), np.arccos(cos[..., 1]), np.arccos(cos[..., 2])
    z_ref = np.stack([np.cos(th) * np.sin(ph), np.sin(th) * np.sin(ph), np.cos(ph)], -1)
    e_phi = np.stack([np.cos(th) * np.cos(ph), np.sin(th) * np.cos(ph), -np.sin(ph)], -1)
    x_ref = np.cos(ps)[..., None] * e_phi + np.sin(ps)[..., None] * np.cross(z_ref, e_phi)
    x, _, z = Pp.frame_from_cosines(cos)
    np.testing.assert_allclose(z, z_ref, atol=1e-14)
    np.testing.assert_allclose(x, x_ref, atol=1e-14)


def test_printed_jacobians_against_finite_differences():
    frame, shape, rgbw = _raw_lobes(4, 1, 50, spread=0.8)
    cos, _, _ = Pp.activate(frame, shape, rgbw)
    jx, jz = Pp.frame_cosine_jacobians(cos)
    h = 1e-6
    for i in range(3):
        cp, cm = cos.copy(), cos.copy()
        cp[..., i] += h
        cm[..., i] -= h
        xp, _, zp = Pp.frame_from_cosines(cp)
        xm, _, zm = Pp.frame_from_cosines(cm)
        np.testing.assert_allclose(jx[..., i], (xp - xm) / (2 * h), atol=2e-8)
        np.testing.assert_allclose(jz[..., i], (zp - zm) / (2 * h), atol=2e-8)


@pytest.mark.parametrize("norm", [R.NORM_EXACT, R.NORM_APPROX])
def test_same_lobes_as_the_quaternion_path(norm):
    """The paper's parametrisation feeds the same evaluation: with the
    quaternion of the same frame and the activated values, colours and the
    c0 / mean gradients agree, and the raw gradients are the activated ones
    times the activation derivatives."""
    wl = W.draw_workload(5, 300, 4, 3, param="angles")
    cos, act, w = Pp.activate(wl.quat, wl.shape, wl.rgbw)
    x, y, z = Pp.frame_from_cosines(cos)
    q = Pp.quat_from_frame(x, y, z)
    geo = {"means": wl.means, "cams": wl.cams}
    out_p, _ = Pp.forward_backward(wl.quat, wl.shape, wl.rgbw, wl.c0, wl.grad_rgb, norm, **geo)
    out_q, _ = R.forward_backward(q, act, w, wl.c0, wl.grad_rgb, norm, **geo)
    for key in ("rgb", "c0", "means"):
        np.testing.assert_allclose(out_p[key], out_q[key], rtol=1e-9, atol=1e-11)
    tk = np.tanh(np.asarray(wl.shape, np.float64)[..., 2])
    chain = np.stack([act[..., 0], act[..., 1], 20 * (1 - tk * tk), np.ones_like(tk)], -1)
    np.testing.assert_allclose(out_p["shape"], out_q["shape"] * chain, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(out_p["rgbw"], out_q["rgbw"] * (1 - w * w), rtol=1e-10,
                               atol=1e-14)


def test_sines_near_saturation_keep_their_digits():
    """Far out (|u| = 15) 1 - tanh^2 of the rounded tanh loses ~4 digits; the
    oracle's sines and chain factors are sech(u) evaluated directly, which
    agrees with 4 e^{-2|u|}/(1 + e^{-2|u|})^2 (the same function written out)
    to rounding."""
    u = np.array([-15.0, -9.0, 0.3, 12.0, 15.0])
    t = np.exp(-2 * np.abs(u))
    np.testing.assert_allclose(Pp.sech(u) ** 2, 4 * t / (1 + t) ** 2, rtol=1e-14)


def _loss(frame, shape, rgbw, c0, g, geo, norm):
    rgb = Pp.forward(frame, shape, rgbw, c0, norm, **geo)[0]
    return float((rgb * g).sum())


def _fd(fun, x, rel=1e-5):
    """Richardson-extrapolated central differences, elementwise."""
    out = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        h = rel * max(1.0, abs(x[i]))

        def c(hh):
            xp = x.copy()
            xp[i] += hh
            xm = x.copy()
            xm[i] -= hh
            return (fun(xp) - fun(xm)) / (2 * hh)
        out[i] = (4 * c(h / 2) - c(h)) / 3
    return out


@pytest.mark.parametrize("norm", [R.NORM_EXACT, R.NORM_APPROX])
def test_raw_gradients_against_finite_differences(norm):
    """Every raw-value gradient against Richardson central differences of one
    primitive's loss (one lobe at a time for lobe values); views are placed
    near lobe 0's axis so the lobes are O(1) there."""
    rng = np.random.default_rng(40 + norm)
    K, N, V = 3, 4, 3
    frame, shape, rgbw = _raw_lobes(41 + norm, K, N, spread=0.9)
    c0 = rng.standard_normal((N, 3))
    cos, _, _ = Pp.activate(frame, shape, rgbw)
    z0 = Pp.frame_from_cosines(cos[0])[2]
    cams = 8.0 * rng.standard_normal((V, 3))
    means = cams[0][None] + 4.0 * (z0 + 0.3 * rng.standard_normal((N, 3)))
    g = rng.standard_normal((V, N, 3))
    geo = {"means": means, "cams": cams}
    out, scale = Pp.forward_backward(frame, shape, rgbw, c0, g, norm, **geo)

    for n in range(N):
        gn = g[:, n:n + 1]
        gg = {"means": means[n:n + 1], "cams": cams}
        for l in range(K):
            sl = (slice(l, l + 1), slice(n, n + 1))
            base = {"quat": frame[sl].copy(), "shape": shape[sl].copy(),
                    "rgbw": rgbw[l:l + 1, :, n:n + 1].copy()}
            for name in ("quat", "shape", "rgbw"):
                def f(x, name=name):
                    b = dict(base)
                    b[name] = x
                    return _loss(b["quat"], b["shape"], b["rgbw"], np.zeros((1, 3)), gn, gg, norm)
                num = _fd(f, base[name])
                ana = out[name][sl] if name != "rgbw" else out["rgbw"][l:l + 1, :, n:n + 1]
                sc = scale[name][sl] if name != "rgbw" else scale["rgbw"][l:l + 1, :, n:n + 1]
                err = np.abs(num - ana) / (sc + 1e-300)
                if name == "quat":
                    err = err[..., :3]
                assert err.max() < 1e-6, (name, n, l, err.max())
        # the unused fourth frame slot has no gradient
        assert np.all(out["quat"][:, n, 3] == 0)

        def fm(x):
            return _loss(frame[:, n:n + 1], shape[:, n:n + 1], rgbw[:, :, n:n + 1],
                         np.zeros((1, 3)), gn, {"means": x, "cams": cams}, norm)
        num = _fd(fm, means[n:n + 1].copy())
        err = np.abs(num - out["means"][n:n + 1]) / (scale["means"][n:n + 1] + 1e-300)
        assert err.max() < 1e-6, ("means", n, err.max())


def test_frame_gradient_finite_at_saturated_cosines():
    """Raw frame values far out (tanh within 1e-12 of +-1) keep finite raw
    gradients: the chain factor sech^2 u cancels the printed 1/s."""
    wl = W.draw_workload(6, 64, 2, 2, param="angles")
    wl.quat[..., :3] = np.clip(6.0 * wl.quat[..., :3], -15.0, 15.0)
    out, scale = Pp.forward_backward(wl.quat, wl.shape, wl.rgbw, wl.c0, wl.grad_rgb,
                                     R.NORM_EXACT, means=wl.means, cams=wl.cams)
    assert np.all(np.isfinite(out["quat"])) and np.all(np.isfinite(scale["quat"]))
