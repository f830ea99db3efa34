"""Learning-rate utilities: the oracle against closed forms, the package
against the oracle (host code, no GPU)."""
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
    assert lr.knn_distance(c) == pytest.approx(s, rel=1e-12)


def test_ring_spacing():
    """C cameras evenly on a circle of radius r: the neighbours are two chords
    2 r sin(pi/C) and one chord 2 r sin(2 pi/C)."""
    C, r = 12, 4.0
    a = 2 * np.pi * np.arange(C) / C
    c = np.stack([r * np.cos(a), r * np.sin(a), np.zeros(C)], -1)
    ref = (2 * 2 * r * math.sin(math.pi / C) + 2 * r * math.sin(2 * math.pi / C)) / 3
    assert Q.knn_distance(c) == pytest.approx(ref, rel=1e-13)
    assert lr.knn_distance(c) == pytest.approx(ref, rel=1e-12)


def test_package_matches_oracle_on_random_cameras():
    rng = np.random.default_rng(0)
    c = rng.standard_normal((57, 3)) * 3
    for k in (1, 3, 5):
        assert lr.knn_distance(c, k) == pytest.approx(Q.knn_distance(c, k), rel=1e-12)


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
    with pytest.raises(ValueError):
        lr.knn_distance(np.zeros((3, 3)))
