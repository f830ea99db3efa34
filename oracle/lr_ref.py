"""Reference for the paper's training-rate utilities (test infrastructure
only; see the package header). Plain loops over the definitions.

* Camera-spacing heuristic (Section 4, implementation details): d_knn is the
  average distance between each camera centre and its k nearest other camera
  centres (k = 3), averaged over cameras; the spherical-feature rate is
  eta_f = eta_f,b (d_ref / d_knn)^beta and the opacity rate
  eta_sigma = eta_sigma,b (d_knn / d_ref)^gamma, beta = 2, gamma = 0.6.
  d_ref is the same statistic for a reference scene (the paper's bonsai
  cameras; not available here, so always an argument).
* Cosine schedule (the supplement's learning-rate scheduling): the factor
  eta(t) = (1 + cos(pi t / T_max)) / 2 applied from iteration 7000 on, with t
  the current iteration and T_max the total; before that the factor is 1
  (taken as printed, including the step at t = 7000).
"""
from __future__ import annotations

import math


def knn_one(centres, i, k=3):
    """Mean distance from camera i to its k nearest other cameras."""
    pts = [tuple(float(c) for c in p) for p in centres]
    ds = sorted(math.dist(pts[i], q) for j, q in enumerate(pts) if j != i)
    return sum(ds[:k]) / k


def knn_per_camera(centres, k=3):
    """knn_one for every camera, in camera order."""
    if len(centres) <= k:
        raise ValueError("need more than k cameras")
    return [knn_one(centres, i, k) for i in range(len(centres))]


def knn_distance(centres, k=3):
    """Average over cameras of the mean distance to the k nearest others."""
    per = knn_per_camera(centres, k)
    return math.fsum(per) / len(per)


def rate_scales(d_knn, d_ref, beta=2.0, gamma=0.6):
    """(eta_f / eta_f,b, eta_sigma / eta_sigma,b)."""
    return (d_ref / d_knn) ** beta, (d_knn / d_ref) ** gamma


def cosine_factor(t, t_max, start=7000):
    """Multiplier of the scheduled learning rates at iteration t."""
    if t < start:
        return 1.0
    return 0.5 * (1.0 + math.cos(math.pi * t / t_max))
