"""Learning-rate utilities of the paper's training set-up.

* ``camera_knn`` / ``knn_distance``: the average distance between camera
  centres and their k nearest neighbours (k = 3), used to scale the
  appearance learning rates with view sparsity (Section 4, implementation
  details). Computed by the library's ``nasg_camera_knn`` kernel in FP64.
* ``rate_scales``: eta_f = eta_f,b (d_ref / d_knn)^2 for the spherical
  features, eta_sigma = eta_sigma,b (d_knn / d_ref)^0.6 for the opacities.
  d_ref is the statistic of a reference scene (the paper uses its bonsai
  cameras) and must be supplied.
* ``cosine_factor``: (1 + cos(pi t / T_max)) / 2, applied from iteration 7000
  on (1 before), taken as printed.

The last two are scalar formulas evaluated once per scene or iteration on the
host.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L


def camera_knn(centres, k: int = 3):
    """(per-camera mean distance to the k nearest other cameras [C] float64 on
    the device, their average over the cameras as a float). ``centres`` is
    [C][3] (tensor or array-like, copied to the current device as float64),
    k < C <= 65536, 1 <= k <= 32."""
    c = torch.as_tensor(centres, dtype=torch.float64)
    if c.dim() != 2 or c.shape[1] != 3:
        raise ValueError("camera centres must be [C][3]")
    n = int(c.shape[0])
    if not 1 <= k <= L.KNN_MAX_K:
        raise ValueError(f"k must be in [1, {L.KNN_MAX_K}]")
    if n <= k:
        raise ValueError("need more than k cameras")
    if n > L.KNN_MAX_CAMERAS:
        raise ValueError(f"at most {L.KNN_MAX_CAMERAS} cameras")
    lib = L.lib()
    c = c.to("cuda").contiguous()
    per = torch.empty(n, dtype=torch.float64, device=c.device)
    mean = torch.empty(1, dtype=torch.float64, device=c.device)
    st = C.c_void_p(torch.cuda.current_stream(c.device).cuda_stream)
    L.check(lib.nasg_camera_knn(C.c_void_p(c.data_ptr()), n, int(k), C.c_void_p(per.data_ptr()),
                                C.c_void_p(mean.data_ptr()), st), "nasg_camera_knn")
    return per, float(mean.item())


def knn_distance(centres, k: int = 3) -> float:
    """Mean over cameras of the mean distance to the k nearest other cameras."""
    return camera_knn(centres, k)[1]


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
