"""The FP64 oracle in the edge regions of the NASGabor lobe (Section 5.1
definition and closed-form integral), against mpmath at 50 digits.

Hypothesis draws cases in each region of ``workloads.edges`` (views next to
the lobe axis and its antipode, the series and sine branches of the
normaliser's sinhc, zeta near pi with k near 0, sharp lobes near their peak,
k = 0, carrier zeros). For each case and both normalisers:

* the value G must match the 50-digit value within FP64 rounding, with the
  conditioning of the case made explicit: the carrier's relative sensitivity
  to the rounding of k d.x + zeta near a carrier zero, and the sensitivity of
  the direction to the rounding of the frame next to the axis;
* every gradient (quaternion, lam, a, k, zeta, raw direction) must match
  mpmath's numerical derivative of the 50-digit value within 1e-9 of the
  oracle's rounding scale (times the same conditioning).

The derivatives are independent of the oracle's analytic formulas; the value
pins the oracle's evaluation (the half-chord forms next to the poles, the
half-angle carrier, the delta form of Psi) against the definition itself.
"""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st
from scipy.spatial.transform import Rotation

import mp_lobe as MP
from oracle import nasg_ref as R
from workloads import edges as E

UNIT = st.floats(min_value=0.0, max_value=1.0, exclude_max=True, allow_nan=False)
DRAWS = st.lists(UNIT, min_size=8, max_size=8)
EPS64 = 2.2e-16


def _oracle(c, norm):
    q = c["q"][None, None]
    shape = c["shape"][None, None]
    rgbw = np.array([[[1.0], [0.0], [0.0]]])
    grad = np.array([[[1.0, 0.0, 0.0]]])
    out, scale = R.forward_backward(q, shape, rgbw, np.zeros((1, 3)), grad, norm,
                                    dirs=c["dir"][None])
    g = np.concatenate([out["quat"][0, 0], out["shape"][0, 0], out["dirs"][0]])
    s = np.concatenate([scale["quat"][0, 0], scale["shape"][0, 0], scale["dirs"][0]])
    return out["rgb"][0, 0, 0], g, s


def _conditioning(c):
    """Relative sensitivity of G and its gradients to FP64 rounding of the
    intermediate quantities, beyond O(1): the carrier near a zero (relative
    change of cos^2(t/2) per unit rounding of t = k d.x + zeta) and the
    direction next to the axis or antipode (rounding of the frame against the
    angle from +-z)."""
    ax, _, az = R.frame_from_quat(c["q"].astype(np.float64))
    d = c["dir"].astype(np.float64)
    d = d / np.linalg.norm(d)
    lam, a, k, zeta = c["shape"].astype(np.float64)
    dx = float(d @ ax)
    t = k * dx + zeta
    car = (abs(k * dx) + abs(zeta) + 1.0) * abs(math.tan(t / 2)) if math.cos(t / 2) != 0 else 1e300
    ang = min(np.linalg.norm(d - az), np.linalg.norm(d + az))
    return 1.0 + car + 1.0 / max(ang, 1e-300), ang


def _check(c, norm):
    G, g, s = _oracle(c, norm)
    Gm = MP.value(c["q"], c["shape"], c["dir"], norm)
    cond, ang = _conditioning(c)
    tol_v = 1e-12 + 8 * EPS64 * cond
    assert abs(G - Gm) <= tol_v * abs(Gm) + 1e-300, (c, norm, G, Gm)
    if ang == 0.0:
        # exactly on the axis or the antipode the derivative depends on the
        # direction of approach; the oracle's limit values there are pinned
        # by the special-point tests
        return
    gm = np.asarray(MP.gradient(c["q"], c["shape"], c["dir"], norm))
    tol_g = 1e-9 + 8 * EPS64 * cond
    err = np.abs(g - gm) / (s + 1e-300)
    assert np.all(err <= tol_g), (c, norm, err, g, gm)


def test_axis_frames_table_matches_scipy():
    """The generator's exactly known frames: x and z are the first and third
    columns of the rotation matrix of q/|q| (scipy, scalar-last quaternions)."""
    for q, x, z in E.AXIS_FRAMES:
        m = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        np.testing.assert_allclose(m[:, 0], x, atol=1e-15)
        np.testing.assert_allclose(m[:, 2], z, atol=1e-15)


def test_series_exact_points_are_exact():
    """Lam^2 - k^2 of the exact series-branch points is 0, 1 or -1 in FP64."""
    for lam, a, k in E.SERIES_EXACT:
        lam32, a32, k32 = np.float32(lam), np.float32(a), np.float32(k)
        big = float(lam32) * (1.0 + float(a32))
        assert big * big - float(k32) ** 2 in (0.0, 1.0, -1.0, big * big)


@pytest.mark.parametrize("region", E.REGIONS)
@pytest.mark.parametrize("norm", [R.NORM_EXACT, R.NORM_APPROX])
@settings(max_examples=25, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(u=DRAWS)
def test_oracle_matches_50_digit_lobe(region, norm, u):
    _check(E.edge_case(region, u), norm)


@pytest.mark.parametrize("norm", [R.NORM_EXACT, R.NORM_APPROX])
def test_edge_grid_against_50_digits(norm):
    """Every point of the fixed edge grid that the GPU tests use."""
    w = E.edge_grid()
    for i in range(w.n):
        _check({"q": w.quat[0, i], "shape": w.shape[0, i], "dir": w.dirs[i]}, norm)


def test_edge_region_membership():
    """The generator lands in the regions it names (checked on the stored
    float32 values)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        u = rng.random(8)
        c = E.edge_case("series", u)
        lam, a, k, _ = c["shape"].astype(np.float64)
        big = lam * (1 + a)
        assert abs(big * big - k * k) <= 1.5 + 1e-9 or k == 0.0
        c = E.edge_case("trig", u)
        lam, a, k, _ = c["shape"].astype(np.float64)
        assert k > lam * (1 + a)
        c = E.edge_case("phase", u)
        assert 0.9e-4 <= abs(float(c["shape"][3]) - math.pi) <= 1.1e-2
        for reg, sgn in (("axis", 1.0), ("antipode", -1.0)):
            c = E.edge_case(reg, u)
            _, _, az = R.frame_from_quat(c["q"].astype(np.float64))
            d = c["dir"].astype(np.float64)
            ang = np.linalg.norm(d / np.linalg.norm(d) - sgn * az)
            assert 0.5e-7 <= ang <= 0.11
