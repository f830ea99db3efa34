"""Learning-rate utilities on the CPU: the oracle's camera-spacing statistic
against closed forms, the host-side rate formulas against the oracle, and the
argument checks made before the device kernel is called. The kernel itself is
compared with the oracle in test_gpu_lr.py."""
import math

import numpy as np
import pytest

from oracle import lr_ref as Q
from paper_2606_09794_amd import lr


def test_cube_vertices_spacing():
    """Cameras on the corners of a cube of side s: each one's three nearest
    others are its edge neighbours, at distance s."""
    s = 2.5
    c = np.array([[x, y, z] for x in (0, s) for y in (0, s) for z in (0, s)])
    assert Q.knn_distance(c) == pytest.approx(s, rel=1e-15)


def test_ring_spacing():
    """C cameras evenly on a circle of radius r: the neighbours are two chords
    2 r sin(pi/C) and one chord 2 r sin(2 pi/C)."""
    C, r = 12, 4.0
    a = 2 * np.pi * np.arange(C) / C
    c = np.stack([r * np.cos(a), r * np.sin(a), np.zeros(C)], -1)
    ref = (2 * 2 * r * math.sin(math.pi / C) + 2 * r * math.sin(2 * math.pi / C)) / 3
    assert Q.knn_distance(c) == pytest.approx(ref, rel=1e-13)


def test_line_spacing_ends():
    """C cameras on a line at spacing s, k = 2: an inner camera's two nearest
    are both at s, an end camera's at s and 2 s, so two of the C per-camera
    values are 1.5 s and the rest s."""
    C, s = 9, 0.75
    c = np.stack([s * np.arange(C), np.zeros(C), np.zeros(C)], -1)
    per = Q.knn_per_camera(c, 2)
    assert per[0] == per[-1] == pytest.approx(1.5 * s, rel=1e-15)
    assert per[1:-1] == pytest.approx([s] * (C - 2), rel=1e-15)
    assert Q.knn_distance(c, 2) == pytest.approx(((C - 2) * s + 3 * s) / C, rel=1e-15)
    # k = 1 sees only the spacing
    assert Q.knn_distance(c, 1) == pytest.approx(s, rel=1e-15)


def test_coincident_cameras_count_at_zero():
    """Two cameras at one place are each other's nearest neighbour, at 0."""
    c = [[0, 0, 0], [0, 0, 0], [3, 4, 0]]
    assert Q.knn_per_camera(c, 1) == [0.0, 0.0, 5.0]
    assert Q.knn_per_camera(c, 2) == [2.5, 2.5, 5.0]


def test_rate_scales():
    f, o = lr.rate_scales(0.5, 1.0)
    assert (f, o) == pytest.approx((4.0, 0.5 ** 0.6))
    assert lr.rate_scales(1.3, 1.3) == pytest.approx((1.0, 1.0))
    assert lr.rate_scales(0.7, 2.1) == pytest.approx(Q.rate_scales(0.7, 2.1))
    with pytest.raises(ValueError):
        lr.rate_scales(0.0, 1.0)


def test_cosine_schedule():
    T = 30000
    assert lr.cosine_factor(0, T) == 1.0 and lr.cosine_factor(6999, T) == 1.0
    assert lr.cosine_factor(T // 2, T) == pytest.approx(0.5)
    assert lr.cosine_factor(T, T) == pytest.approx(0.0, abs=1e-15)
    for t in (7000, 12345, 29999):
        assert lr.cosine_factor(t, T) == pytest.approx(Q.cosine_factor(t, T))


@pytest.mark.parametrize("shape,k", [((3, 3), 3), ((4, 2), 1), ((40, 3), 0), ((40, 3), 33),
                                     ((65537, 3), 3)])
def test_camera_knn_rejects_before_the_device(shape, k):
    with pytest.raises(ValueError):
        lr.camera_knn(np.zeros(shape), k)
