"""Seeded synthetic inputs in the storage layout of the appearance path.

Layouts (primitive index fastest within each lobe, lobe-major):

* ``quat``  [K][N][4]  lobe-frame quaternion (w, x, y, z), any nonzero norm
* ``shape`` [K][N][4]  (lambda, a, k, zeta): bandwidth, anisotropy, carrier
                       frequency and carrier phase
* ``rgbw``  [K][3][N]  per-lobe RGB weight, channel-planar
* ``c0``    [N][3]     diffuse colour
* ``means`` [N][3]     primitive centres, with ``cams`` [V][3] camera centres
* ``dirs``  [N][3]     alternatively one raw (unnormalised) view direction per
                       primitive; then V = 1
* ``grad_rgb`` [V][N][3] upstream gradient of the per-view colour
* ``sh``    [16][3][N] degree-3 spherical-harmonics coefficients

Distributions follow the parameter ranges of the paper's kernel
parametrisation (Supplementary Material C): frames Haar-uniform (a normal
4-vector is a uniform unit quaternion after normalisation), bandwidth and
anisotropy log-uniform in [1, 1e3], carrier frequency uniform in [0, 16],
carrier phase uniform in [0, 2 pi), weights and diffuse colour N(0, 0.5^2).
Scene geometry: means uniform in [-5, 5]^3, camera centres uniform on the
sphere of radius 10, which stands in for the paper's Mip-NeRF360-class scenes
(roughly 3 M primitives per scene).

With ``param="angles"`` the lobe slots hold the paper's own stored values
instead, all before activation (Supplementary C): ``quat`` holds
(u_theta, u_phi, u_psi, 0) with frame cosines tanh(u) drawn from N(0, 1);
``shape`` holds (u_lambda, u_a, u_k, zeta) with u_lambda, u_a uniform in
[0, ln 1e3] (so lambda = e^u and a = e^u are log-uniform in [1, 1e3] as
above), u_k from N(0, 1) (k = 20 (tanh u + 1) spreads over the paper's
[0, 40]) and zeta = 0 (the paper's carrier); ``rgbw`` holds the weights'
u from N(0, 0.5^2) (w = tanh u).

With ``family`` other than "nasgabor" the shape slot holds that lobe
family's values (the distribution table of Supplementary A): "nasg"
(lambda, a, 0, 0) and "sg" (lambda, 0, 0, 0) with lambda, a log-uniform in
[1, 1e3]; "sb" (beta, 0, 0, 0) with beta log-uniform in [1, 1e3]; "sc"
(rho, 0, 0, 0) with rho uniform in [0, 0.95]; "asg" (mu, lambda, 0, 0) both
log-uniform in [1, 1e3]. Frames, weights and geometry are drawn as above.

Nothing here evaluates the appearance model: the module draws, rounds to the
storage dtype and gathers, so the oracle and the HIP path consume identical
stored bits.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even).

    Returns the 16-bit patterns as uint16. Inputs are finite by construction.
    """
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    bias = np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))
    return ((b + bias) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns to float32."""
    return (np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


@dataclasses.dataclass
class Workload:
    """One scene's worth of inputs in storage layout (see module docstring)."""

    n: int
    k: int
    v: int
    quat: np.ndarray            # float32 values of the stored lobe params
    shape: np.ndarray
    rgbw: np.ndarray
    c0: np.ndarray
    means: Optional[np.ndarray] = None
    cams: Optional[np.ndarray] = None
    dirs: Optional[np.ndarray] = None
    grad_rgb: Optional[np.ndarray] = None
    sh: Optional[np.ndarray] = None
    dtype: str = "f32"          # storage dtype of quat / shape / rgbw
    quat_bits: Optional[np.ndarray] = None   # uint16 patterns when dtype == "bf16"
    shape_bits: Optional[np.ndarray] = None
    rgbw_bits: Optional[np.ndarray] = None
    orig: Optional[dict] = None  # float32 values before bf16 rounding
    param: str = "quat"         # "quat" or "angles" (the paper's raw values)
    family: str = "nasgabor"    # lobe family of the shape slot

    @property
    def evals(self) -> int:
        return self.n * self.v


@dataclasses.dataclass
class Scene:
    workload: Workload
    index: int


def _draw_lobes(rng: np.random.Generator, k: int, n: int):
    quat = rng.standard_normal((k, n, 4), dtype=np.float32)
    lam = np.exp(rng.uniform(0.0, math.log(1e3), (k, n))).astype(np.float32)
    a = np.exp(rng.uniform(0.0, math.log(1e3), (k, n))).astype(np.float32)
    kk = rng.uniform(0.0, 16.0, (k, n)).astype(np.float32)
    zeta = rng.uniform(0.0, TWO_PI, (k, n)).astype(np.float32)
    shape = np.stack([lam, a, kk, zeta], axis=-1)
    rgbw = (0.5 * rng.standard_normal((k, 3, n), dtype=np.float32)).astype(np.float32)
    c0 = (0.5 * rng.standard_normal((n, 3), dtype=np.float32)).astype(np.float32)
    return quat, np.ascontiguousarray(shape), rgbw, c0


FAMILIES = ("nasgabor", "nasg", "sg", "sb", "sc", "asg")


def _draw_family_lobes(rng: np.random.Generator, k: int, n: int, family: str):
    quat = rng.standard_normal((k, n, 4), dtype=np.float32)
    logu = lambda: np.exp(rng.uniform(0.0, math.log(1e3), (k, n))).astype(np.float32)  # noqa: E731
    z = np.zeros((k, n), np.float32)
    if family in ("nasg", "asg"):
        p0 = logu()
        p1 = logu()
    elif family in ("sg", "sb"):
        p0, p1 = logu(), z
    elif family == "sc":
        p0, p1 = rng.uniform(0.0, 0.95, (k, n)).astype(np.float32), z
    else:
        raise ValueError(f"unknown lobe family {family!r}")
    shape = np.stack([p0, p1, z, z], axis=-1)
    rgbw = (0.5 * rng.standard_normal((k, 3, n), dtype=np.float32)).astype(np.float32)
    c0 = (0.5 * rng.standard_normal((n, 3), dtype=np.float32)).astype(np.float32)
    return quat, np.ascontiguousarray(shape), rgbw, c0


def _draw_paper_lobes(rng: np.random.Generator, k: int, n: int):
    frame = np.zeros((k, n, 4), np.float32)
    frame[..., :3] = rng.standard_normal((k, n, 3), dtype=np.float32)
    ul = rng.uniform(0.0, math.log(1e3), (k, n)).astype(np.float32)
    ua = rng.uniform(0.0, math.log(1e3), (k, n)).astype(np.float32)
    uk = rng.standard_normal((k, n), dtype=np.float32)
    shape = np.stack([ul, ua, uk, np.zeros_like(uk)], axis=-1)
    rgbw = (0.5 * rng.standard_normal((k, 3, n), dtype=np.float32)).astype(np.float32)
    c0 = (0.5 * rng.standard_normal((n, 3), dtype=np.float32)).astype(np.float32)
    return frame, np.ascontiguousarray(shape), rgbw, c0


def _draw_cams(rng: np.random.Generator, v: int) -> np.ndarray:
    g = rng.standard_normal((v, 3))
    return (10.0 * g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)


CAMERA_LAYOUTS = ("sphere", "orbit", "forward")


def draw_camera_centres(seed: int, n: int, layout: str = "sphere") -> np.ndarray:
    """[n][3] float64 camera centres in the layouts of the paper's captures:
    "sphere", directions uniform on a shell of radius 10 (the appearance
    workloads' cameras); "orbit", a walk-around at radius 4-6 with heights in
    [0.5, 2.5] and jittered angular steps; "forward", a forward-facing
    capture, a jittered 2D grid of spacing 0.2 in the plane z = -3."""
    rng = np.random.default_rng(seed)
    if layout == "sphere":
        g = rng.standard_normal((n, 3))
        return 10.0 * g / np.linalg.norm(g, axis=1, keepdims=True)
    if layout == "orbit":
        a = 2 * np.pi * (np.arange(n) + 0.3 * rng.random(n)) / n
        r = rng.uniform(4.0, 6.0, n)
        return np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(0.5, 2.5, n)], -1)
    if layout == "forward":
        side = int(np.ceil(np.sqrt(n)))
        ij = np.stack(np.divmod(np.arange(n), side), -1).astype(np.float64)
        xy = 0.2 * (ij + 0.25 * rng.standard_normal((n, 2)))
        return np.concatenate([xy, np.full((n, 1), -3.0)], -1)
    raise ValueError(f"layout must be one of {CAMERA_LAYOUTS}")


def draw_workload(seed: int, n: int, k: int, v: int, *, dirs_mode: bool = False,
                  with_grad: bool = True, with_sh: bool = True, dtype: str = "f32",
                  rng: Optional[np.random.Generator] = None, param: str = "quat",
                  family: str = "nasgabor") -> Workload:
    """Draw one workload. Order of draws: lobes, diffuse colour, geometry,
    upstream gradient, SH coefficients."""
    rng = np.random.default_rng(seed) if rng is None else rng
    if family != "nasgabor" and param == "quat":
        quat, shape, rgbw, c0 = _draw_family_lobes(rng, k, n, family)
    elif param == "quat":
        quat, shape, rgbw, c0 = _draw_lobes(rng, k, n)
    elif param == "angles":
        quat, shape, rgbw, c0 = _draw_paper_lobes(rng, k, n)
    else:
        raise ValueError(f"unknown lobe parametrisation {param!r}")
    means = cams = dirs = None
    if dirs_mode:
        if v != 1:
            raise ValueError("per-primitive directions imply a single view")
        dirs = rng.standard_normal((n, 3), dtype=np.float32)
    else:
        means = rng.uniform(-5.0, 5.0, (n, 3)).astype(np.float32)
        cams = _draw_cams(rng, v)
    grad_rgb = rng.standard_normal((v, n, 3), dtype=np.float32) if with_grad else None
    sh = (0.3 * rng.standard_normal((16, 3, n), dtype=np.float32)).astype(np.float32) if with_sh else None
    w = Workload(n=n, k=k, v=v, quat=quat, shape=shape, rgbw=rgbw, c0=c0, means=means,
                 cams=cams, dirs=dirs, grad_rgb=grad_rgb, sh=sh, param=param, family=family)
    if dtype == "bf16":
        w.orig = {"quat": quat, "shape": shape, "rgbw": rgbw}
        w.quat_bits = f32_to_bf16_bits(quat)
        w.shape_bits = f32_to_bf16_bits(shape)
        w.rgbw_bits = f32_to_bf16_bits(rgbw)
        w.quat = bf16_bits_to_f32(w.quat_bits)
        w.shape = bf16_bits_to_f32(w.shape_bits)
        w.rgbw = bf16_bits_to_f32(w.rgbw_bits)
        w.dtype = "bf16"
    elif dtype != "f32":
        raise ValueError(f"unknown storage dtype {dtype!r}")
    return w


# ---- the five reference workloads -------------------------------------------------

def config0(n: int = 4096, seed: int = 0) -> Workload:
    """Plain forward, FP32: K = 4, one raw view direction per primitive."""
    return draw_workload(seed, n, 4, 1, dirs_mode=True)


def config1(n: int = 1 << 20, seed: int = 1) -> Workload:
    """Forward+backward, FP32: K = 8, one camera, per-primitive upstream gradient."""
    return draw_workload(seed, n, 8, 1)


def config2(n: int = 3_000_000, seed: int = 2, v: int = 16) -> Workload:
    """Batched views, FP32: K = 8, V = 16 cameras in one launch."""
    return draw_workload(seed, n, 8, v)


def config3(n: int = 6_000_000, seed: int = 3, dtype: str = "bf16") -> Workload:
    """Precision form: K = 16, V = 8, lobe parameters stored in bf16."""
    return draw_workload(seed, n, 16, 8, dtype=dtype, with_sh=False)


def config4(seed: int = 4, n_scenes: int = 32, scale: float = 1.0,
            with_sh: bool = False) -> List[Scene]:
    """Uneven batch: scenes with N log-uniform in [5e4, 2e6] (times ``scale``),
    K drawn from {4, 8, 16} and V from {1, 4, 16}."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(5e4), math.log(2e6), n_scenes))
    ks = rng.choice([4, 8, 16], n_scenes)
    vs = rng.choice([1, 4, 16], n_scenes)
    scenes = []
    for s in range(n_scenes):
        n = max(1, int(round(float(ns[s]) * scale)))
        wl = draw_workload(0, n, int(ks[s]), int(vs[s]), with_sh=with_sh, rng=rng)
        scenes.append(Scene(workload=wl, index=s))
    return scenes


def take_primitives(w: Workload, idx: np.ndarray) -> Workload:
    """Gather a subset of primitives (all lobes, all views). Pure indexing."""
    idx = np.asarray(idx, dtype=np.int64)
    sub = Workload(
        n=int(idx.size), k=w.k, v=w.v,
        quat=np.ascontiguousarray(w.quat[:, idx]),
        shape=np.ascontiguousarray(w.shape[:, idx]),
        rgbw=np.ascontiguousarray(w.rgbw[:, :, idx]),
        c0=np.ascontiguousarray(w.c0[idx]),
        means=None if w.means is None else np.ascontiguousarray(w.means[idx]),
        cams=w.cams,
        dirs=None if w.dirs is None else np.ascontiguousarray(w.dirs[idx]),
        grad_rgb=None if w.grad_rgb is None else np.ascontiguousarray(w.grad_rgb[:, idx]),
        sh=None if w.sh is None else np.ascontiguousarray(w.sh[:, :, idx]),
        dtype=w.dtype, param=w.param, family=w.family,
    )
    if w.dtype == "bf16":
        sub.quat_bits = np.ascontiguousarray(w.quat_bits[:, idx])
        sub.shape_bits = np.ascontiguousarray(w.shape_bits[:, idx])
        sub.rgbw_bits = np.ascontiguousarray(w.rgbw_bits[:, :, idx])
        if w.orig is not None:
            sub.orig = {"quat": np.ascontiguousarray(w.orig["quat"][:, idx]),
                        "shape": np.ascontiguousarray(w.orig["shape"][:, idx]),
                        "rgbw": np.ascontiguousarray(w.orig["rgbw"][:, :, idx])}
    return sub
