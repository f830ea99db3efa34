"""Seeded synthetic splatting scenes for the compositing path.

A scene is a pinhole camera and N 3D Gaussians, in the layouts of the
compositing entry points: ``means`` [N][3], ``scales`` [N][3] (per-axis
standard deviations), ``rots`` [N][4] (quaternion w, x, y, z, any norm),
``opac`` [N], ``colors`` [N][3], plus an upstream ``grad_image`` [H][W][3].
All arrays are float32; the camera is kept in float64 (rotation R_cw
row-major, translation t, fx, fy, cx, cy, width, height).

Distributions stand in for a trained scene of the paper's Mip-NeRF360 class
seen from one training camera: the camera orientation is Haar-uniform (QR of
a Gaussian matrix, sign-fixed), the focal length is fx = fy = 0.9 width (a
roughly 58 degree horizontal field of view), the principal point is the image
centre; primitive centres are drawn in camera space with depth uniform in
``depth`` and screen position uniform over the image plus a 10 % margin,
then moved to world space; a fraction ``behind`` lies behind the near plane;
scales are log-uniform in ``scale``, opacities uniform in ``opac`` and
colours N(0.5, 0.5^2) per channel.

Nothing here composites anything: the module only draws and transforms the
inputs, so the oracle and the HIP path read identical stored values.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class SplatScene:
    means: np.ndarray
    scales: np.ndarray
    rots: np.ndarray
    opac: np.ndarray
    colors: np.ndarray
    grad_image: np.ndarray
    cam: dict

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


def _rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def draw_splat_scene(seed: int, n: int, width: int, height: int, *,
                     depth=(2.0, 10.0), scale=(0.003, 0.03), opac=(0.05, 0.9),
                     behind: float = 0.05) -> SplatScene:
    rng = np.random.default_rng(seed)
    R = _rotation(rng)
    t = rng.uniform(-1.0, 1.0, 3)
    f = 0.9 * width
    cam = dict(R=R, t=t, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0, width=width, height=height)
    z = rng.uniform(depth[0], depth[1], n)
    nb = int(round(behind * n))
    z[:nb] = rng.uniform(-3.0, 0.15, nb)
    sx = rng.uniform(-0.1 * width, 1.1 * width, n)
    sy = rng.uniform(-0.1 * height, 1.1 * height, n)
    xc = np.stack([(sx - cam["cx"]) / f * np.abs(z), (sy - cam["cy"]) / f * np.abs(z), z], -1)
    perm = rng.permutation(n)
    xc = xc[perm]
    means = ((xc - t) @ R).astype(np.float32)          # x = R^T (x_c - t)
    scales = np.exp(rng.uniform(math.log(scale[0]), math.log(scale[1]), (n, 3))).astype(np.float32)
    rots = rng.standard_normal((n, 4)).astype(np.float32)
    op = rng.uniform(opac[0], opac[1], n).astype(np.float32)
    colors = (0.5 + 0.5 * rng.standard_normal((n, 3))).astype(np.float32)
    grad_image = rng.standard_normal((height, width, 3)).astype(np.float32)
    return SplatScene(means, scales, rots, op, colors, grad_image, cam)
