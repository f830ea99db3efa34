"""Pins of the FP64 NASGabor oracle against things other than itself.

* quadrature of the normalised lobe over the sphere (unit mass) where the
  closed-form integral of Section 5.1 is exact (a = 0 or k = 0), and the
  APPROX (NASG) normaliser at k = 0;
* the von Mises-Fisher density (scipy) for a = 0, k = 0, zeta = 0;
* reductions of the definition on special great circles and points;
* symmetries: rotation equivariance, quaternion sign / scale, reflections;
* mpmath evaluation of e^{-Lam} sinhc(sqrt(Lam^2 - k^2));
* central finite differences of every gradient (Supplementary E/F with the
  sign reading of dC^{-1}/dlam), and the projector invariants.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.stats import vonmises_fisher

from oracle import nasg_ref as R
from sphere_quad import fibonacci_sphere, lobe_frame_grid

ID_Q = np.array([1.0, 0.0, 0.0, 0.0])


@pytest.fixture(scope="module")
def grid():
    return lobe_frame_grid()


# ------------------------------------------------------------------ normalisers

EXACT_CASES = [  # (lam, a, k, zeta) with a = 0 or k = 0
    (5, 0, 0, 0), (5, 0, 8, 0), (5, 3, 0, 0), (1, 1000, 0, 0), (20, 100, 0, 0),
    (1000, 1000, 0, 0), (50, 0, 16, 1.0), (0.3, 0, 3, 2.0), (0.05, 0.5, 0, 0),
    (2, 0, 40, 3.0), (1, 0, 1, 0.5), (12, 0, 12, 0),  # k = Lam: sinhc at 0
]


@pytest.mark.parametrize("shape", EXACT_CASES)
def test_exact_normaliser_unit_mass(grid, shape):
    d, w = grid
    G = R.lobe_value(d, ID_Q, np.array(shape, float), R.NORM_EXACT)
    assert abs((G * w).sum() - 1.0) < 1e-10


@pytest.mark.parametrize("shape", [s for s in EXACT_CASES if s[2] == 0])
def test_approx_normaliser_unit_mass_at_k0(grid, shape):
    d, w = grid
    G = R.lobe_value(d, ID_Q, np.array(shape, float), R.NORM_APPROX)
    assert abs((G * w).sum() - 1.0) < 1e-10


def test_approx_is_exact_at_k0_only():
    lam, a = 3.0, 2.0
    na = R.norm_approx(lam, a)[0]
    assert na == pytest.approx(R.norm_exact(lam, a, 0.0, 0.0)[0], rel=1e-14)
    # with a carrier the approximation ignores it: exact = 2 x approx when the
    # carrier averages to one half (large k, zeta = 0) is not required, only
    # that they differ
    assert abs(R.norm_exact(lam, a, 8.0, 0.0)[0] / na - 1) > 0.1


def test_closed_form_not_exact_with_anisotropy_and_carrier(grid):
    """For a > 0 and k > 0 the printed closed form misses the true integral by
    a few percent (recorded, not asserted to be exact)."""
    d, w = grid
    for shape in [(2, 1, 4, 0), (5, 3, 8, 0)]:
        G = R.lobe_value(d, ID_Q, np.array(shape, float), R.NORM_EXACT)
        mass = (G * w).sum()
        assert 1e-3 < abs(mass - 1) < 5e-2


def test_fibonacci_unit_mass_random_frame():
    d, w = fibonacci_sphere(1_000_000)
    q = np.array([0.3, -0.7, 0.2, 0.6])
    for shape in [(5, 3, 0, 0), (20, 0, 10, 0.7)]:
        G = R.lobe_value(d, q, np.array(shape, float), R.NORM_EXACT)
        assert abs((G * w).sum() - 1) < 1e-6


def test_psi_at_k0_is_one():
    L = np.array([1e-3, 0.5, 1.0, 7.0, 300.0, 1e6])
    P, dPL, dPk, _ = R.psi(L, np.zeros_like(L))
    np.testing.assert_allclose(P, 1.0, rtol=1e-13)
    np.testing.assert_allclose(dPL, 0.0, atol=1e-12)
    np.testing.assert_allclose(dPk, 0.0, atol=1e-12)


@pytest.mark.parametrize("L,k", [(1e6, 16), (710, 3), (5, 5), (5, 5.0001), (3, 10),
                                 (0.5, 0.2), (20, 16), (16.0000001, 16), (2, 40),
                                 (1.3, 0.9), (40, 1e-3)])
def test_exp_sinhc_against_mpmath(L, k):
    mpmath.mp.dps = 50
    Lm, km = mpmath.mpf(L), mpmath.mpf(k)
    r = Lm * Lm - km * km

    def S(rr):
        if rr > 0:
            u = mpmath.sqrt(rr)
            return mpmath.sinh(u) / u
        if rr < 0:
            u = mpmath.sqrt(-rr)
            return mpmath.sin(u) / u
        return mpmath.mpf(1)

    ref = mpmath.e ** (-Lm) * S(r)
    dref = mpmath.e ** (-Lm) * mpmath.diff(S, r)
    F, dF = R.exp_sinhc(np.array([L], float), np.array([k], float))
    assert float(F[0]) == pytest.approx(float(ref), rel=1e-12, abs=1e-300)
    assert float(dF[0]) == pytest.approx(float(dref), rel=1e-9, abs=1e-300)


# ------------------------------------------------------------ special reductions

@pytest.mark.parametrize("lam", [0.5, 3.0, 40.0, 900.0])
def test_vmf_special_case(lam):
    """a = 0, k = 0, zeta = 0: G is the von Mises-Fisher density in both modes."""
    rng = np.random.default_rng(11)
    q = rng.standard_normal(4)
    z = R.frame_from_quat(q[None])[2][0]
    d = z[None] + (3.0 / math.sqrt(lam)) * rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ref = vonmises_fisher(z, lam).pdf(d)
    for norm in (R.NORM_EXACT, R.NORM_APPROX):
        G = R.lobe_value(d, q, np.array([lam, 0, 0, 0.0]), norm)
        np.testing.assert_allclose(G, ref, rtol=1e-11, atol=1e-300)


def test_yz_great_circle_ignores_anisotropy_and_frequency():
    """On the y-z great circle d.x = 0: tau = 0 and the carrier is constant, so
    G = N (1 + cos zeta)/2 exp(lam (d.z - 1))."""
    lam, a, k, zeta = 4.0, 7.0, 9.0, 0.8
    th = np.linspace(0.01, 3.1, 50)
    d = np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], -1)
    N = R.norm_exact(lam, a, k, zeta)[0]
    G = R.lobe_value(d, ID_Q, np.array([lam, a, k, zeta]), R.NORM_EXACT)
    np.testing.assert_allclose(G, N * 0.5 * (1 + math.cos(zeta)) * np.exp(lam * (np.cos(th) - 1)),
                               rtol=1e-13)


def test_xz_great_circle_full_anisotropy():
    """On the x-z great circle tau = a and d.x = sin(theta)."""
    lam, a, k, zeta = 2.0, 3.0, 5.0, 0.3
    th = np.linspace(0.01, 3.1, 50)
    d = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], -1)
    kap = (np.cos(th) + 1) / 2
    N = R.norm_approx(lam, a)[0]
    ref = N * 0.5 * (1 + np.cos(k * np.sin(th) + zeta)) * np.exp(2 * lam * kap ** (1 + a) - 2 * lam) * kap ** a
    G = R.lobe_value(d, ID_Q, np.array([lam, a, k, zeta]), R.NORM_APPROX)
    np.testing.assert_allclose(G, ref, rtol=1e-12)


def test_peak_antipode_and_positivity():
    lam, a, k, zeta = 3.0, 2.0, 6.0, 1.1
    N = R.norm_exact(lam, a, k, zeta)[0]
    G = R.lobe_value(np.array([[0, 0, 1.0], [0, 0, -1.0]]), ID_Q, np.array([lam, a, k, zeta]),
                     R.NORM_EXACT)
    assert G[0] == pytest.approx(N * 0.5 * (1 + math.cos(zeta)), rel=1e-15)
    assert G[1] == 0.0
    rng = np.random.default_rng(3)
    d = rng.standard_normal((5000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    assert (R.lobe_value(d, rng.standard_normal(4), np.array([lam, a, k, zeta]),
                         R.NORM_EXACT) >= 0).all()


# --------------------------------------------------------------------- symmetry

def test_frame_matches_scipy_rotation():
    rng = np.random.default_rng(2)
    q = rng.standard_normal((50, 4)) * rng.uniform(0.1, 5, (50, 1))
    ax, ay, az = R.frame_from_quat(q)
    M = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(ax, M[:, :, 0], atol=1e-14)
    np.testing.assert_allclose(ay, M[:, :, 1], atol=1e-14)
    np.testing.assert_allclose(az, M[:, :, 2], atol=1e-14)
    np.testing.assert_allclose(np.cross(az, ax), ay, atol=1e-14)   # y = z x x


def _hamilton(r, q):
    w1, x1, y1, z1 = r
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rotation_equivariance_and_quaternion_gauge():
    rng = np.random.default_rng(5)
    shape = np.array([6.0, 4.0, 7.0, 0.4])
    q = rng.standard_normal(4)
    z = R.frame_from_quat(q[None])[2][0]
    d = z[None] + 0.5 * rng.standard_normal((300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    G = R.lobe_value(d, q, shape, R.NORM_EXACT)
    r = rng.standard_normal(4)
    Rm = Rotation.from_quat((r / np.linalg.norm(r))[[1, 2, 3, 0]]).as_matrix()
    G2 = R.lobe_value(d @ Rm.T, _hamilton(r, q), shape, R.NORM_EXACT)
    np.testing.assert_allclose(G2, G, rtol=1e-9, atol=1e-12 * G.max())
    np.testing.assert_allclose(R.lobe_value(d, -3.7 * q, shape, R.NORM_EXACT), G,
                               rtol=1e-11, atol=1e-13 * G.max())


def test_reflection_symmetry_without_phase():
    rng = np.random.default_rng(8)
    d = rng.standard_normal((400, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:, 2] = np.abs(d[:, 2])
    shape = np.array([3.0, 5.0, 9.0, 0.0])
    G = R.lobe_value(d, ID_Q, shape, R.NORM_EXACT)
    for flip in ([-1, 1, 1], [1, -1, 1]):
        np.testing.assert_allclose(R.lobe_value(d * np.array(flip), ID_Q, shape, R.NORM_EXACT), G,
                                   rtol=1e-12, atol=1e-300)


# -------------------------------------------------------------------- gradients

def _designed_workload(seed, n, k, v, dirs_mode):
    """Lobes with moderate bandwidth, views near the lobe axes (so G is O(1))."""
    rng = np.random.default_rng(seed)
    quat = rng.standard_normal((k, n, 4))
    shape = np.stack([rng.uniform(0.5, 12, (k, n)), rng.uniform(0.0, 6, (k, n)),
                      rng.uniform(0, 10, (k, n)), rng.uniform(0, 2 * np.pi, (k, n))], -1)
    rgbw = rng.standard_normal((k, 3, n))
    c0 = rng.standard_normal((n, 3))
    z0 = R.frame_from_quat(quat[0])[2]                       # axis of lobe 0
    if dirs_mode:
        geo = {"dirs": 1.7 * (z0 + 0.4 * rng.standard_normal((n, 3)))}
        v = 1
    else:
        cams = 8.0 * rng.standard_normal((v, 3))
        means = cams[0][None] + 4.0 * (z0 + 0.3 * rng.standard_normal((n, 3)))
        geo = {"means": means, "cams": cams}
    g = rng.standard_normal((v, n, 3))
    return quat, shape, rgbw, c0, g, geo


def _loss(quat, shape, rgbw, c0, g, geo, norm):
    rgb = R.forward(quat, shape, rgbw, c0, norm, **geo)[0]
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
@pytest.mark.parametrize("dirs_mode", [True, False])
def test_gradients_against_finite_differences(norm, dirs_mode):
    """Every analytic gradient against Richardson central differences of the
    loss of one primitive (and one lobe for lobe parameters), so that the
    difference quotient is not swamped by the other primitives' terms."""
    quat, shape, rgbw, c0, g, geo = _designed_workload(21 + norm, 5, 3, 3, dirs_mode)
    out, scale = R.forward_backward(quat, shape, rgbw, c0, g, norm, **geo)
    K, N = quat.shape[:2]
    key = "dirs" if dirs_mode else "means"

    def geo_of(n, x=None):
        gg = {}
        for kk, vv in geo.items():
            gg[kk] = vv if kk == "cams" else vv[n:n + 1].copy()
        if x is not None:
            gg[key] = x
        return gg

    for n in range(N):
        gn = g[:, n:n + 1]
        for l in range(K):
            sl = (slice(l, l + 1), slice(n, n + 1))
            for name in ["quat", "shape"]:
                base = {"quat": quat[sl], "shape": shape[sl]}

                def f(x, name=name):
                    b = dict(base)
                    b[name] = x
                    return _loss(b["quat"], b["shape"], rgbw[l:l + 1, :, n:n + 1],
                                 np.zeros((1, 3)), gn, geo_of(n), norm)
                num = _fd(f, base[name])
                err = np.abs(num - out[name][sl]) / (scale[name][sl] + 1e-300)
                assert err.max() < 1e-6, (name, n, l, err.max())
            # the rgb weight enters linearly
            def fw(x):
                return _loss(quat[sl], shape[sl], x, np.zeros((1, 3)), gn, geo_of(n), norm)
            num = _fd(fw, rgbw[l:l + 1, :, n:n + 1])
            err = np.abs(num - out["rgbw"][l:l + 1, :, n:n + 1]) / (
                scale["rgbw"][l:l + 1, :, n:n + 1] + 1e-300)
            assert err.max() < 1e-6, ("rgbw", n, l, err.max())

        def fg(x):
            return _loss(quat[:, n:n + 1], shape[:, n:n + 1], rgbw[:, :, n:n + 1],
                         np.zeros((1, 3)), gn, geo_of(n, x), norm)
        num = _fd(fg, geo[key][n:n + 1])
        err = np.abs(num - out[key][n:n + 1]) / (scale[key][n:n + 1] + 1e-300)
        assert err.max() < 1e-6, (key, n, err.max())

    def fc(x):
        return _loss(quat, shape, rgbw, x, g, geo, norm)
    num = _fd(fc, c0)
    err = np.abs(num - out["c0"]) / (scale["c0"] + 1e-12)
    assert err.max() < 1e-6, ("c0", err.max())


def test_paper_plus_sign_in_dC_dlam_disagrees_with_fd():
    """The printed '+ 2 lam sqrt(1+a) e^{-2 lam}' numerator does not match a
    finite difference of C^{-1}; the '-' reading does."""
    lam, a = 1.0, 0.5
    h = 1e-6
    fd = (R.norm_approx(lam + h, a)[0] - R.norm_approx(lam - h, a)[0]) / (2 * h)
    ours = R.norm_approx(lam, a)[1]
    printed = (math.sqrt(1 + a) * (1 - math.exp(-2 * lam)) + 2 * lam * math.sqrt(1 + a)
               * math.exp(-2 * lam)) / (2 * math.pi * (1 - math.exp(-2 * lam)) ** 2)
    assert ours == pytest.approx(fd, rel=1e-8)
    assert abs(printed / fd - 1) > 0.5


def test_exact_normaliser_derivatives_fd():
    rng = np.random.default_rng(4)
    for _ in range(20):
        p = np.array([rng.uniform(0.2, 30), rng.uniform(0, 20), rng.uniform(0, 20),
                      rng.uniform(0, 2 * np.pi)])
        res = R.norm_exact(*p)
        for j in range(4):
            def f(x, j=j):
                q = p.copy()
                q[j] = x
                return R.norm_exact(*q)[0]
            h = 1e-5 * max(1, abs(p[j]))
            num = (4 * (f(p[j] + h / 2) - f(p[j] - h / 2)) / h - (f(p[j] + h) - f(p[j] - h)) / (2 * h)) / 3
            assert res[1 + j] == pytest.approx(num, rel=1e-6, abs=1e-9 * abs(res[0]))


def test_projector_invariants():
    quat, shape, rgbw, c0, g, geo = _designed_workload(5, 8, 4, 1, False)
    out, _ = R.forward_backward(quat, shape, rgbw, c0, g, R.NORM_EXACT, **geo)
    # q . dL/dq = 0 (scale invariance in |q|)
    dots = (out["quat"] * quat).sum(-1)
    assert np.abs(dots).max() < 1e-10 * np.abs(out["quat"]).max()
    # one view: dL/dmu . d = 0 (d depends on mu only through its direction)
    e = geo["means"] - geo["cams"][0][None]
    d = e / np.linalg.norm(e, axis=1, keepdims=True)
    assert np.abs((out["means"] * d).sum(-1)).max() < 1e-10 * np.abs(out["means"]).max()


def test_linearity_in_weights_and_c0():
    quat, shape, rgbw, c0, g, geo = _designed_workload(6, 4, 2, 2, False)
    r1 = R.forward(quat, shape, rgbw, c0, R.NORM_EXACT, **geo)[0]
    r2 = R.forward(quat, shape, 2 * rgbw, c0, R.NORM_EXACT, **geo)[0]
    r3 = R.forward(quat, shape, rgbw, c0 + 1.0, R.NORM_EXACT, **geo)[0]
    tol = 1e-13 * np.abs(r1).max()
    np.testing.assert_allclose(r2 - c0[None], 2 * (r1 - c0[None]), rtol=1e-12, atol=tol)
    np.testing.assert_allclose(r3, r1 + 1.0, rtol=1e-12, atol=tol)


def test_special_points_gradients_finite():
    """d = +z: value N (1+cos zeta)/2, finite gradients; d = -z: everything 0."""
    quat = np.array([[[1.0, 0, 0, 0], [1.0, 0, 0, 0]]])         # K=1, N=2
    shape = np.array([[[3.0, 2.0, 5.0, 0.7], [3.0, 2.0, 5.0, 0.7]]])
    rgbw = np.ones((1, 3, 2))
    c0 = np.zeros((2, 3))
    dirs = np.array([[0, 0, 2.0], [0, 0, -2.0]])
    g = np.ones((1, 2, 3))
    out, _ = R.forward_backward(quat, shape, rgbw, c0, g, R.NORM_EXACT, dirs=dirs)
    N = R.norm_exact(3.0, 2.0, 5.0, 0.7)[0]
    assert out["rgb"][0, 0, 0] == pytest.approx(N * 0.5 * (1 + math.cos(0.7)), rel=1e-15)
    assert out["rgb"][0, 1, 0] == 0.0
    for v in out.values():
        assert np.isfinite(v).all()
    assert np.all(out["shape"][0, 1] == 0) and np.all(out["quat"][0, 1] == 0)
    assert np.all(out["dirs"][1] == 0)


def test_quat_gradient_two_step_chain():
    """dL/dq through (d axis/d q_hat)^T then the tangent projection equals the
    projected Jacobian of frame_jacobians; its scale bounds the scale of the
    projected Jacobian's absolute terms."""
    rng = np.random.default_rng(5)
    q = rng.standard_normal((6, 7, 4))
    q[0, :, 1:3] *= 1e-3                     # near a rotation about a coordinate axis
    gx, gz = rng.standard_normal((6, 7, 3)), rng.standard_normal((6, 7, 3))
    jx, jz = R.frame_jacobians(q)
    ref = np.einsum("knci,knc->kni", jx, gx) + np.einsum("knci,knc->kni", jz, gz)
    g, sc = R.quat_gradient(q, gx, gz, np.abs(gx), np.abs(gz))
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-14)
    old = np.einsum("knci,knc->kni", np.abs(jx), np.abs(gx)) + np.einsum("knci,knc->kni", np.abs(jz), np.abs(gz))
    assert np.all(sc >= old * (1 - 1e-12))

