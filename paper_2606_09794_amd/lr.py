"""Learning-rate utilities of the paper's training set-up (host side).

* ``knn_distance``: the average distance between camera centres and their k
  nearest neighbours (k = 3), used to scale the appearance learning rates
  with view sparsity (Section 4, implementation details).
* ``rate_scales``: eta_f = eta_f,b (d_ref / d_knn)^2 for the spherical
  features, eta_sigma = eta_sigma,b (d_knn / d_ref)^0.6 for the opacities.
  d_ref is the statistic of a reference scene (the paper uses its bonsai
  cameras) and must be supplied.
* ``cosine_factor``: (1 + cos(pi t / T_max)) / 2, applied from iteration 7000
  on (1 before), taken as printed.
"""
from __future__ import annotations

import math

import torch


def knn_distance(centres, k: int = 3) -> float:
    """Mean over cameras of the mean distance to the k nearest other cameras.
    ``centres`` is [C][3] (tensor or array-like), C > k."""
    c = torch.as_tensor(centres, dtype=torch.float64)
    if c.dim() != 2 or c.shape[1] != 3:
        raise ValueError("camera centres must be [C][3]")
    if c.shape[0] <= k:
        raise ValueError("need more than k cameras")
    d = torch.cdist(c, c)
    d.fill_diagonal_(float("inf"))
    near = torch.topk(d, k, dim=1, largest=False).values
    return float(near.mean())


def rate_scales(d_knn: float, d_ref: float, beta: float = 2.0, gamma: float = 0.6):
    """(eta_f / eta_f,b, eta_sigma / eta_sigma,b) for a scene with camera
    spacing d_knn against the reference spacing d_ref."""
    if d_knn <= 0 or d_ref <= 0:
        raise ValueError("camera spacings must be positive")
    return (d_ref / d_knn) ** beta, (d_knn / d_ref) ** gamma


def cosine_factor(t: int, t_max: int, start: int = 7000) -> float:
    """Multiplier of the scheduled learning rates at iteration t."""
    if t_max <= 0:
        raise ValueError("t_max must be positive")
    if t < start:
        return 1.0
    return 0.5 * (1.0 + math.cos(math.pi * t / t_max))
