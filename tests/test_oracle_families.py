"""Pins of the FP64 oracle for the other lobe families (Supplementary A
distribution table; Supplementary D for the spherical beta; Supplementary E for
NASG). Nothing here runs on the GPU."""
import numpy as np
import pytest
from scipy.stats import vonmises_fisher

import workloads as W
from oracle import families as F
from oracle import nasg_ref as R
from sphere_quad import fibonacci_sphere, lobe_frame_grid

ID_Q = np.array([1.0, 0.0, 0.0, 0.0])


@pytest.fixture(scope="module")
def grid():
    """Lobe-frame grid with a panel edge on the equator (u = 0 at s = 1/sqrt 2),
    where the hemisphere families have a kink."""
    lo_half = np.geomspace(1e-6, 0.5, 50)
    panels = np.unique(np.concatenate([[0.0], lo_half, (1.0 - lo_half)[::-1], [1.0, 2 ** -0.5]]))
    return lobe_frame_grid(panels=panels)


@pytest.mark.parametrize("fam,shape", [
    (F.SG, (0.01, 0, 0, 0)), (F.SG, (3.0, 0, 0, 0)), (F.SG, (900.0, 0, 0, 0)),
    (F.SB, (0.0, 0, 0, 0)), (F.SB, (2.5, 0, 0, 0)), (F.SB, (300.0, 0, 0, 0)),
    (F.SC, (0.0, 0, 0, 0)), (F.SC, (0.3, 0, 0, 0)), (F.SC, (0.95, 0, 0, 0)),
    (F.NASG, (4.0, 2.0, 0, 0)), (F.NASG, (300.0, 50.0, 0, 0)),
])
def test_unit_mass(grid, fam, shape):
    d, w = grid
    G = F.lobe_value(fam, d, ID_Q, np.array(shape, float))
    assert abs((G * w).sum() - 1.0) < 1e-9


def test_unit_mass_random_frame_fibonacci():
    d, w = fibonacci_sphere(1_000_000)
    q = np.array([0.3, -0.7, 0.2, 0.6])
    for fam, shape in [(F.SG, (8.0, 0, 0, 0)), (F.SB, (6.0, 0, 0, 0)), (F.SC, (0.5, 0, 0, 0))]:
        G = F.lobe_value(fam, d, q, np.array(shape, float))
        assert abs((G * w).sum() - 1) < 1e-5, fam


def test_sg_is_von_mises_fisher():
    rng = np.random.default_rng(0)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for lam in (0.5, 7.0, 120.0):
        ref = vonmises_fisher(np.array([0.0, 0.0, 1.0]), lam).pdf(d)
        np.testing.assert_allclose(F.lobe_value(F.SG, d, ID_Q, np.array([lam, 0, 0, 0.])), ref,
                                   rtol=1e-10)


def test_sb_closed_values():
    d = np.array([[0, 0, 1.0], [0, 0.6, 0.8], [1.0, 0, 0], [0, 0.8, -0.6]])
    G = F.lobe_value(F.SB, d, ID_Q, np.array([3.0, 0, 0, 0]))
    np.testing.assert_allclose(G, [4 / (2 * np.pi), 4 / (2 * np.pi) * 0.8 ** 3, 0.0, 0.0], rtol=1e-14)


def test_sc_uniform_at_rho0_and_peak_value():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(F.lobe_value(F.SC, d, ID_Q, np.zeros(4)), 1 / (4 * np.pi), rtol=1e-14)
    rho = 0.4
    peak = F.lobe_value(F.SC, np.array([[0, 0, 1.0]]), ID_Q, np.array([rho, 0, 0, 0]))
    np.testing.assert_allclose(peak, ((1 + rho) / (1 - rho)) ** 2 / (4 * np.pi), rtol=1e-14)


def test_printed_sc_denominator_is_not_a_density(grid):
    """With 1 - rho^2 - 2 rho z.d (as printed) the mass is not 4 pi c = 1."""
    d, w = grid
    rho = 0.3
    u = 1 - rho * rho - 2 * rho * d[:, 2]
    G = ((1 - rho * rho) / u) ** 2 / (4 * np.pi)
    assert abs((G * w).sum() - 1) > 0.1


@pytest.mark.parametrize("mu", [0.0, 0.7, 25.0])
def test_asg_isotropic_closed_form(grid, mu):
    """mu = lam: G = max(z.d, 0) e^{-mu (1 - (z.d)^2)}, whose integral is
    pi (1 - e^{-mu}) / mu (pi at mu = 0)."""
    d, w = grid
    G = F.lobe_value(F.ASG, d, ID_Q, np.array([mu, mu, 0, 0]))
    ref = np.pi if mu == 0 else np.pi * (1 - np.exp(-mu)) / mu
    assert abs((G * w).sum() - ref) < 1e-9 * max(1, ref)


def test_asg_axes():
    """Decay along x with mu and along y with lam; y = z x x."""
    G = F.lobe_value(F.ASG, np.array([[0.6, 0, 0.8], [0, 0.6, 0.8]]), ID_Q, np.array([2.0, 5.0, 0, 0]))
    np.testing.assert_allclose(G, [0.8 * np.exp(-2 * 0.36), 0.8 * np.exp(-5 * 0.36)], rtol=1e-14)


def test_nasg_family_is_nasgabor_without_carrier():
    rng = np.random.default_rng(2)
    d = rng.standard_normal((100, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = np.array([0.1, 0.9, -0.3, 0.2])
    shape = np.array([40.0, 7.0, 0.0, 0.0])
    np.testing.assert_allclose(F.lobe_value(F.NASG, d, q, np.array([40.0, 7.0, 5.0, 1.0])),
                               R.lobe_value(d, q, shape, R.NORM_EXACT), rtol=1e-12)


def _family_workload(fam, seed, n, k, v):
    """Quaternion frames, family parameters in moderate ranges, views near the
    first lobe's axis so every family is O(1) there."""
    rng = np.random.default_rng(seed)
    quat = rng.standard_normal((k, n, 4))
    p = {F.SG: lambda: np.stack([rng.uniform(0.5, 15, (k, n))] + [np.zeros((k, n))] * 3, -1),
         F.SB: lambda: np.stack([rng.uniform(1.0, 12, (k, n))] + [np.zeros((k, n))] * 3, -1),
         F.SC: lambda: np.stack([rng.uniform(0.05, 0.9, (k, n))] + [np.zeros((k, n))] * 3, -1),
         F.ASG: lambda: np.stack([rng.uniform(0.2, 10, (k, n)), rng.uniform(0.2, 10, (k, n))]
                                 + [np.zeros((k, n))] * 2, -1),
         F.NASG: lambda: np.stack([rng.uniform(0.5, 12, (k, n)), rng.uniform(0.0, 6, (k, n))]
                                  + [np.zeros((k, n))] * 2, -1)}[fam]()
    rgbw = rng.standard_normal((k, 3, n))
    z0 = R.frame_from_quat(quat[0])[2]
    cams = 8.0 * rng.standard_normal((v, 3))
    means = cams[0][None] + 4.0 * (z0 + 0.3 * rng.standard_normal((n, 3)))
    g = rng.standard_normal((v, n, 3))
    c0 = rng.standard_normal((n, 3))
    return quat, p, rgbw, c0, g, {"means": means, "cams": cams}


def _fd(fun, x, rel=1e-5):
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


@pytest.mark.parametrize("fam", [F.SG, F.SB, F.SC, F.ASG, F.NASG])
def test_gradients_against_finite_differences(fam):
    quat, shape, rgbw, c0, g, geo = _family_workload(fam, 70 + fam, 4, 3, 3)
    out, scale = F.forward_backward(fam, quat, shape, rgbw, c0, g, **geo)

    def loss(q, s, w, c, gg, means):
        rgb = F.forward(fam, q, s, w, c, means=means, cams=geo["cams"])[0]
        return float((rgb * gg).sum())

    K, N = quat.shape[:2]
    for n in range(N):
        gn = g[:, n:n + 1]
        mn = geo["means"][n:n + 1]
        for l in range(K):
            sl = (slice(l, l + 1), slice(n, n + 1))
            base = {"quat": quat[sl].copy(), "shape": shape[sl].copy(),
                    "rgbw": rgbw[l:l + 1, :, n:n + 1].copy()}
            for name in ("quat", "shape", "rgbw"):
                def f(x, name=name):
                    b = dict(base)
                    b[name] = x
                    return loss(b["quat"], b["shape"], b["rgbw"], np.zeros((1, 3)), gn, mn)
                num = _fd(f, base[name])
                ana = out[name][sl] if name != "rgbw" else out["rgbw"][l:l + 1, :, n:n + 1]
                sc = scale[name][sl] if name != "rgbw" else scale["rgbw"][l:l + 1, :, n:n + 1]
                err = np.abs(num - ana) / (sc + 1e-300)
                assert err.max() < 1e-6, (F.NAMES[fam], name, n, l, err.max())
        num = _fd(lambda x: loss(quat[:, n:n + 1], shape[:, n:n + 1], rgbw[:, :, n:n + 1],
                                 np.zeros((1, 3)), gn, x), mn.copy())
        err = np.abs(num - out["means"][n:n + 1]) / (scale["means"][n:n + 1] + 1e-300)
        assert err.max() < 1e-6, (F.NAMES[fam], "means", n, err.max())


def test_nasg_family_with_the_papers_raw_values():
    """NASG accepts the paper's raw values; the k and zeta slots are unused."""
    wl = W.draw_workload(8, 50, 3, 2, param="angles")
    out, scale = F.forward_backward(F.NASG, wl.quat, wl.shape, wl.rgbw, wl.c0, wl.grad_rgb,
                                    means=wl.means, cams=wl.cams, param="angles")
    assert np.all(out["shape"][..., 2:] == 0)
    assert np.all(np.isfinite(out["quat"])) and np.all(np.isfinite(out["shape"]))
