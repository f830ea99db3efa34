"""Designed inputs in the edge regions of the NASGabor lobe (seeded).

The regions are where the Section 5.1 definition and its closed-form
integral are numerically delicate:

* ``axis``         view directions 1e-7 .. 1e-1 rad from the lobe axis z
* ``antipode``     view directions 1e-7 .. 1e-1 rad from -z
* ``series``       |Lam^2 - k^2| <= 1.5, Lam = lam (1 + a): the power-series
                   branch of the normaliser's sinhc and its boundaries,
                   including k = Lam and |Lam^2 - k^2| = 1 exactly
* ``trig``         k > Lam with small Lam (the sine branch of sinhc)
* ``phase``        zeta within 1e-4 .. 1e-2 of pi with k in [0, 1e-1] or
                   k = 0 (1 + cos(zeta) Psi, the normaliser's factor, near 0)
* ``sharp``        Lam in 1e2 .. 1e6 viewed within a few peak widths
* ``k0``           k = 0 exactly
* ``carrier_zero`` k d.x + zeta = pi up to the rounding of the stored zeta

``switch_grid`` places lobes on both sides of lam = 1/2 and of
Lam = lam (1 + a) = 3/2, where an evaluator may change its arithmetic.

A case is built from a vector ``u`` of uniform draws in [0, 1) (numpy's
seeded generator here, Hypothesis in the oracle's property tests), so both
consumers share the region definitions. Frames come from a table of
quaternions whose frames are signed coordinate axes (rotations of the cube),
so that a view direction can sit 1e-7 rad from +-z with float32-exact
components; ``aimed_workload`` instead aims lobes at cameras with frames from
scipy's rotation class. Nothing here evaluates the appearance model: this
module only places and rounds inputs.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

from .gen import Workload, bf16_bits_to_f32, f32_to_bf16_bits

REGIONS = ("axis", "antipode", "series", "trig", "phase", "sharp", "k0", "carrier_zero")

# (quaternion (w, x, y, z), x axis, z axis): the first and third columns of
# the rotation matrix of q/|q| (checked against scipy in the tests). Every
# entry is exact in float32 and bfloat16.
AXIS_FRAMES = (
    ((1, 0, 0, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 1, 0, 0), (1, 0, 0), (0, 0, -1)),
    ((1, 1, 0, 0), (1, 0, 0), (0, -1, 0)),
    ((1, 0, 1, 0), (0, 0, -1), (1, 0, 0)),
    ((1, 0, 0, 1), (0, 1, 0), (0, 0, 1)),
    ((1, 1, 1, 1), (0, 1, 0), (1, 0, 0)),
    ((1, -1, -1, -1), (0, 0, 1), (0, 1, 0)),
    ((0, 0, 1, 1), (-1, 0, 0), (0, 1, 0)),
    ((1, -1, 0, 0), (1, 0, 0), (0, 1, 0)),
    ((0, 0, 0, 1), (-1, 0, 0), (0, 0, 1)),
    ((1, 0, -1, 0), (0, 0, 1), (-1, 0, 0)),
    ((1, 1, -1, 1), (0, 0, 1), (0, -1, 0)),
)

# series-branch points with Lam^2 - k^2 exactly 0, +1 or -1 (binary fractions,
# exact in float32 and bfloat16): (lam, a, k)
SERIES_EXACT = (
    (1.0, 0.0, 1.0), (2.0, 1.0, 4.0), (0.5, 3.0, 2.0), (1.25, 0.0, 0.75), (0.75, 0.0, 1.25),
    (1.0, 0.0, 0.0), (0.625, 1.0, 0.75), (0.375, 1.0, 1.25), (4.0, 3.0, 16.0),
)


def _logu(u: float, lo: float, hi: float) -> float:
    return float(10.0 ** (lo + (hi - lo) * u))


def _perp_dir(frame, s: float, eps: float, phi: float) -> np.ndarray:
    """s z rotated by eps towards the frame-plane direction at azimuth phi
    (built from the two coordinate axes orthogonal to z)."""
    z = np.asarray(frame[2], np.float64)
    i = int(np.argmax(np.abs(z)))
    e1 = np.zeros(3)
    e2 = np.zeros(3)
    e1[(i + 1) % 3] = 1.0
    e2[(i + 2) % 3] = 1.0
    return s * math.cos(eps) * z + math.sin(eps) * (math.cos(phi) * e1 + math.sin(phi) * e2)


def edge_case(region: str, u: Sequence[float]) -> Dict[str, np.ndarray]:
    """One designed lobe and view: float32 q [4], shape (lam, a, k, zeta) [4]
    and a raw view direction [3]. ``u`` holds at least 8 draws in [0, 1)."""
    u = [float(x) for x in u]
    if len(u) < 8:
        raise ValueError("edge_case needs 8 uniform draws")
    frame = AXIS_FRAMES[int(u[7] * len(AXIS_FRAMES)) % len(AXIS_FRAMES)]
    phi = 2.0 * math.pi * u[6]
    rnd_dir = np.array([math.cos(phi) * math.sqrt(1 - (2 * u[5] - 1) ** 2),
                        math.sin(phi) * math.sqrt(1 - (2 * u[5] - 1) ** 2), 2 * u[5] - 1])
    lam = _logu(u[0], -1.0, 3.0)
    a = _logu(u[1], -2.0, 3.0)
    k = 16.0 * u[2]
    zeta = 2.0 * math.pi * u[3]
    d = rnd_dir
    if region in ("axis", "antipode"):
        eps = _logu(u[4], -7.0, -1.0)
        if region == "antipode":
            # a lobe broad enough to reach behind itself
            lam = _logu(u[0], -1.0, 1.0)
            a = _logu(u[1], -2.0, 1.0)
        d = _perp_dir(frame, 1.0 if region == "axis" else -1.0, eps, phi)
    elif region == "series":
        if u[4] < 0.3:
            lam, a, k = SERIES_EXACT[int(u[0] * len(SERIES_EXACT)) % len(SERIES_EXACT)]
        else:
            lam = (4 + int(u[0] * 61)) / 16.0                  # 0.25 .. 4
            a = (0.0, 0.5, 1.0, 3.0)[int(u[1] * 4) % 4]
            big = lam * (1.0 + a)
            r = 3.0 * u[2] - 1.5
            k = math.floor(math.sqrt(max(big * big - r, 0.0)) * 64.0 + 0.5) / 64.0
    elif region == "trig":
        lam = _logu(u[0], -1.5, 0.5)
        a = _logu(u[1], -2.0, 0.5)
        k = lam * (1.0 + a) + 1.5 + 14.0 * u[2]
    elif region == "phase":
        off = _logu(u[4], -4.0, -2.0) * (1.0 if u[3] < 0.5 else -1.0)
        zeta = math.pi + off
        k = 0.0 if u[2] < 0.3 else _logu(u[2], -5.0, -1.0)
        lam = _logu(u[0], 0.0, 3.0)
        a = _logu(u[1], 0.0, 3.0)
        width = 1.0 / math.sqrt(lam * (1.0 + a))
        d = _perp_dir(frame, 1.0, 3.0 * width * u[5], phi)
    elif region == "sharp":
        big = 10.0 ** (2.0 + 4.0 * u[0])                     # 1e2 .. 1e6
        a = _logu(u[1], 0.0, min(3.0, math.log10(big) - 0.5))
        lam = big / (1.0 + a)
        h = 6.0 * u[4] / big                                # 1 - d.z within a few widths
        d = _perp_dir(frame, 1.0, 2.0 * math.asin(math.sqrt(h / 2.0)), phi)
    elif region == "k0":
        k = 0.0
        if u[4] < 0.5:
            width = 1.0 / math.sqrt(lam * (1.0 + a))
            d = _perp_dir(frame, 1.0, min(2.0 * width * u[5], 3.0), phi)
    elif region == "carrier_zero":
        lam = _logu(u[0], 0.0, 2.0)
        a = _logu(u[1], 0.0, 2.0)
        k = 1.0 + 15.0 * u[2]
        width = 1.0 / math.sqrt(lam * (1.0 + a))
        d = _perp_dir(frame, 1.0, min(1.5 * width * (0.2 + u[5]), 1.5), phi)
        dx = float(np.dot(np.asarray(d, np.float32).astype(np.float64),
                          np.asarray(frame[1], np.float64)))
        zeta = (math.pi - k * dx) % (2.0 * math.pi)
    else:
        raise ValueError(f"unknown edge region {region!r}")
    return {"q": np.asarray(frame[0], np.float32),
            "shape": np.asarray([lam, a, k, zeta], np.float32),
            "dir": np.asarray(d, np.float32)}


def _finish(w: Workload, dtype: str) -> Workload:
    if dtype == "bf16":
        w.orig = {"quat": w.quat, "shape": w.shape, "rgbw": w.rgbw}
        w.quat_bits = f32_to_bf16_bits(w.quat)
        w.shape_bits = f32_to_bf16_bits(w.shape)
        w.rgbw_bits = f32_to_bf16_bits(w.rgbw)
        w.quat = bf16_bits_to_f32(w.quat_bits)
        w.shape = bf16_bits_to_f32(w.shape_bits)
        w.rgbw = bf16_bits_to_f32(w.rgbw_bits)
        w.dtype = "bf16"
    elif dtype != "f32":
        raise ValueError(f"unknown storage dtype {dtype!r}")
    return w


def edge_workload(seed: int, per_region: int, regions: Sequence[str] = REGIONS,
                  dtype: str = "f32") -> Workload:
    """``per_region`` designed primitives for each region: one lobe each
    (K = 1), one raw view direction (V = 1), c0 = 0 (so the colour's error
    scale is the lobe's own), weights and upstream gradient N(0, 1)."""
    rng = np.random.default_rng(seed)
    cases = [edge_case(r, rng.random(8)) for r in regions for _ in range(per_region)]
    n = len(cases)
    quat = np.stack([c["q"] for c in cases])[None].astype(np.float32)
    shape = np.stack([c["shape"] for c in cases])[None].astype(np.float32)
    dirs = np.stack([c["dir"] for c in cases]).astype(np.float32)
    rgbw = rng.standard_normal((1, 3, n), dtype=np.float32)
    grad = rng.standard_normal((1, n, 3), dtype=np.float32)
    w = Workload(n=n, k=1, v=1, quat=np.ascontiguousarray(quat), shape=np.ascontiguousarray(shape),
                 rgbw=rgbw, c0=np.zeros((n, 3), np.float32), dirs=dirs, grad_rgb=grad)
    return _finish(w, dtype)


def edge_grid(dtype: str = "f32") -> Workload:
    """A fixed grid of the named edge points (one lobe, one raw view each):

    * k = Lam exactly and Lam^2 - k^2 = +-0.5, +-1, +-1.5 (binary-fraction
      lam, a, k where exact), and k > Lam with Lam in {0.05, 0.3, 1};
    * zeta = pi +- 1e-2 and pi +- 1e-4, each with k in {0, 1e-4, 1e-2},
      viewed at 0, 1 and 2 peak widths;
    * views 1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1 rad from +z and from -z,
      each for a sharp (lam = 100, a = 300) and a broad (lam = 1, a = 0.5)
      lobe, at azimuths 0 (d.x largest) and pi/2 (d.x = 0);
    * Lam in {1e2, 1e4, 1e6} viewed at 0.1, 1 and 3 peak widths;
    * k = 0 exactly at the peak and off it.
    """
    rows = []          # (q, (lam, a, k, zeta), dir)
    f0 = AXIS_FRAMES[0]
    f3 = AXIS_FRAMES[5]
    for lam, a, k in SERIES_EXACT:
        rows.append((f0, (lam, a, k, 0.7), _perp_dir(f0, 1.0, 0.3, 0.4)))
    for big in (2.0, 8.0, 12.0):
        for r in (-1.5, -1.0, -0.5, 0.5, 1.0, 1.5):
            rows.append((f3, (big / 2.0, 1.0, math.sqrt(big * big - r), 2.1),
                         _perp_dir(f3, 1.0, 0.2, 1.0)))
    for big in (0.05, 0.3, 1.0):
        for k in (big + 1.01, 4.0, 16.0):
            rows.append((f0, (big / 1.5, 0.5, k, 1.3), _perp_dir(f0, 1.0, 0.5, 0.2)))
    for off in (1e-2, -1e-2, 1e-4, -1e-4):
        for k in (0.0, 1e-4, 1e-2):
            for wd in (0.0, 1.0, 2.0):
                lam, a = 20.0, 4.0
                rows.append((f3, (lam, a, k, math.pi + off),
                             _perp_dir(f3, 1.0, wd / math.sqrt(lam * (1 + a)), 0.9)))
    for eps in (1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1):
        for s in (1.0, -1.0):
            for lam, a in ((100.0, 300.0), (1.0, 0.5)):
                for phi in (0.0, 0.5 * math.pi):
                    for fr in (f0, AXIS_FRAMES[6]):
                        rows.append((fr, (lam, a, 5.0, 0.8), _perp_dir(fr, s, eps, phi)))
    for big in (1e2, 1e4, 1e6):
        for wd in (0.1, 1.0, 3.0):
            a = 99.0
            rows.append((f0, (big / (1 + a), a, 9.0, 2.5),
                         _perp_dir(f0, 1.0, wd / math.sqrt(big), 0.3)))
    for wd in (0.0, 0.5, 2.0):
        rows.append((f0, (30.0, 10.0, 0.0, 1.9), _perp_dir(f0, 1.0, wd / math.sqrt(330.0), 2.0)))
    n = len(rows)
    rng = np.random.default_rng(77)
    quat = np.asarray([r[0][0] for r in rows], np.float32)[None]
    shape = np.asarray([r[1] for r in rows], np.float32)[None]
    dirs = np.asarray([r[2] for r in rows], np.float32)
    rgbw = rng.standard_normal((1, 3, n), dtype=np.float32)
    grad = rng.standard_normal((1, n, 3), dtype=np.float32)
    w = Workload(n=n, k=1, v=1, quat=np.ascontiguousarray(quat), shape=np.ascontiguousarray(shape),
                 rgbw=rgbw, c0=np.zeros((n, 3), np.float32), dirs=dirs, grad_rgb=grad)
    return _finish(w, dtype)


def aimed_workload(seed: int, n: int, k: int, v: int, dtype: str = "f32") -> Workload:
    """Camera-mode workload whose lobes are aimed at the cameras: means
    uniform in [-5, 5]^3 and V cameras on the sphere of radius 10 (as the
    standard workloads); lobe l of primitive i has its axis 10^U(-5, -1.5) rad
    from the direction from camera (i + l) mod V to the primitive, a random
    twist about it, and a sharp envelope (Lam = lam (1 + a) log-uniform in
    [1e2, 1e6]); k ~ U[0, 16], zeta ~ U[0, 2 pi). Every lobe therefore meets
    one view near its peak and the others far from it."""
    from scipy.spatial.transform import Rotation

    rng = np.random.default_rng(seed)
    means = rng.uniform(-5.0, 5.0, (n, 3)).astype(np.float32)
    g = rng.standard_normal((v, 3))
    cams = (10.0 * g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    li = (np.arange(n)[None, :] + np.arange(k)[:, None]) % v           # [K][N] camera index
    e = means.astype(np.float64)[None] - cams.astype(np.float64)[li]   # [K][N][3]
    t = e / np.linalg.norm(e, axis=-1, keepdims=True)
    # tilt by eps about a random axis orthogonal to t, then twist about the result
    r = rng.standard_normal((k, n, 3))
    r -= (r * t).sum(-1, keepdims=True) * t
    r /= np.linalg.norm(r, axis=-1, keepdims=True)
    eps = 10.0 ** rng.uniform(-5.0, -1.5, (k, n))
    z = np.cos(eps)[..., None] * t + np.sin(eps)[..., None] * r
    xr = rng.standard_normal((k, n, 3))
    xr -= (xr * z).sum(-1, keepdims=True) * z
    xr /= np.linalg.norm(xr, axis=-1, keepdims=True)
    y = np.cross(z, xr)
    mats = np.stack([xr, y, z], axis=-1).reshape(-1, 3, 3)
    q_xyzw = Rotation.from_matrix(mats).as_quat()
    quat = np.concatenate([q_xyzw[:, 3:], q_xyzw[:, :3]], axis=1).reshape(k, n, 4).astype(np.float32)
    big = 10.0 ** rng.uniform(2.0, 6.0, (k, n))
    a = 10.0 ** rng.uniform(0.0, 1.0, (k, n)) * np.minimum(100.0, big / 10.0) / 10.0
    lam = big / (1.0 + a)
    kk = rng.uniform(0.0, 16.0, (k, n))
    zeta = rng.uniform(0.0, 2.0 * math.pi, (k, n))
    shape = np.stack([lam, a, kk, zeta], -1).astype(np.float32)
    rgbw = (0.5 * rng.standard_normal((k, 3, n))).astype(np.float32)
    c0 = (0.5 * rng.standard_normal((n, 3))).astype(np.float32)
    grad = rng.standard_normal((v, n, 3)).astype(np.float32)
    w = Workload(n=n, k=k, v=v, quat=np.ascontiguousarray(quat), shape=np.ascontiguousarray(shape),
                 rgbw=np.ascontiguousarray(rgbw), c0=c0, means=means, cams=cams, grad_rgb=grad)
    return _finish(w, dtype)


def switch_grid(dtype: str = "f32") -> Workload:
    """Lobes around lam = 1/2 and Lam = lam (1 + a) = 3/2: lam in {0.49, 0.5,
    0.51, 1}, Lam in {1.49, 1.5, 1.51, 3}, k in {0, 0.3, Lam, Lam + 2, 6} (the
    hyperbolic, series and sine branches of the normaliser's sinhc), zeta in
    {0, pi/2, pi - 1e-3}, each viewed at the peak and one peak width off (one
    lobe and one raw view per primitive)."""
    rows = []
    fr = AXIS_FRAMES[5]
    for lam in (0.49, 0.5, 0.51, 1.0):
        for big in (1.49, 1.5, 1.51, 3.0):
            a = big / lam - 1.0
            for k in (0.0, 0.3, big, big + 2.0, 6.0):
                for zeta in (0.0, 0.5 * math.pi, math.pi - 1e-3):
                    for wd in (0.0, 1.0):
                        rows.append((fr, (lam, a, k, zeta),
                                     _perp_dir(fr, 1.0, wd / math.sqrt(big), 0.7)))
    n = len(rows)
    rng = np.random.default_rng(91)
    quat = np.asarray([r[0][0] for r in rows], np.float32)[None]
    shape = np.asarray([r[1] for r in rows], np.float32)[None]
    dirs = np.asarray([r[2] for r in rows], np.float32)
    rgbw = rng.standard_normal((1, 3, n), dtype=np.float32)
    grad = rng.standard_normal((1, n, 3), dtype=np.float32)
    w = Workload(n=n, k=1, v=1, quat=np.ascontiguousarray(quat), shape=np.ascontiguousarray(shape),
                 rgbw=rgbw, c0=np.zeros((n, 3), np.float32), dirs=dirs, grad_rgb=grad)
    return _finish(w, dtype)
