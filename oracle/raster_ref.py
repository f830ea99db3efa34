"""FP64 reference for compositing the primitives' colours into an image
(test infrastructure only; see the package header).

Section 3.1: a pixel's colour is C = sum_i T_i alpha_i c_i over the primitives
on its ray in depth order, alpha_i = sigma_i rho_i, T_i = prod_{j<i} (1 -
alpha_j). The primitives are 3D Gaussians, Sigma = R S S^T R^T with R from a
quaternion and S = diag(scale); rho_i on the ray is taken, as in splatting,
from the Gaussian projected onto the image plane (the local affine
approximation of the perspective map at the mean). Readings (the paper leaves
the rasterizer to its splatting library):

* camera: x_c = R_cw x + t, pixel u = fx X/Z + cx, v = fy Y/Z + cy; pixel
  (px, py) is sampled at its centre (px + 1/2, py + 1/2);
* projected covariance Sigma_2 = J R_cw Sigma R_cw^T J^T with
  J = [[fx/Z, 0, -fx X/Z^2], [0, fy/Z, -fy Y/Z^2]]; rho = exp(-q/2),
  q = delta^T Sigma_2^{-1} delta, delta = pixel centre - (u, v);
* support: a primitive reaches a pixel only where q <= 9 (its 3-sigma
  ellipse), and only if Z > 0.2 (near plane);
* depth order by camera-space Z of the mean, ties by primitive index;
* alpha = min(sigma rho, 0.99); black background; no early termination.

Gradients of L = sum(grad_image * image) with respect to the per-primitive
colours (dC/dc_i = alpha_i T_i) and opacities (dC/dalpha_i =
T_i c_i - S_i / (1 - alpha_i), S_i = sum_{j>i} c_j alpha_j T_j; dalpha/dsigma =
rho when unclamped, 0 when clamped).
"""
from __future__ import annotations

import numpy as np

NEAR = 0.2
CLAMP = 0.99
SUPPORT_Q = 9.0


def quat_rotation(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def project(means, scales, rots, cam):
    """Per primitive: pixel mean (u, v), the inverse projected covariance
    (a, b, c) with q = a dx^2 + 2 b dx dy + c dy^2, camera depth Z, and a
    visibility flag (Z > near)."""
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    m = np.asarray(means, np.float64)
    xc = m @ R.T + t
    X, Y, Z = xc[:, 0], xc[:, 1], xc[:, 2]
    vis = Z > NEAR
    Zs = np.where(vis, Z, 1.0)
    u = fx * X / Zs + cx
    v = fy * Y / Zs + cy
    Rw = quat_rotation(rots)
    s = np.asarray(scales, np.float64)
    M = Rw * s[:, None, :]                                   # R S
    cov = M @ np.swapaxes(M, -1, -2)                         # R S S^T R^T
    covc = R[None] @ cov @ R.T[None]
    J = np.zeros((m.shape[0], 2, 3))
    J[:, 0, 0] = fx / Zs
    J[:, 0, 2] = -fx * X / (Zs * Zs)
    J[:, 1, 1] = fy / Zs
    J[:, 1, 2] = -fy * Y / (Zs * Zs)
    c2 = J @ covc @ np.swapaxes(J, -1, -2)
    det = c2[:, 0, 0] * c2[:, 1, 1] - c2[:, 0, 1] ** 2
    a = c2[:, 1, 1] / det
    b = -c2[:, 0, 1] / det
    c = c2[:, 0, 0] / det
    return dict(u=u, v=v, a=a, b=b, c=c, z=Z, vis=vis, cov2=c2)


def render(means, scales, rots, opac, colors, cam, grad_image=None):
    """Image [H][W][3] (and, with grad_image, the gradients w.r.t. colours
    [N][3] and opacities [N]) with rounding scales."""
    W, H = int(cam["width"]), int(cam["height"])
    p = project(means, scales, rots, cam)
    order = np.lexsort((np.arange(len(p["z"])), p["z"]))      # by depth, then index
    order = order[p["vis"][order]]
    col = np.asarray(colors, np.float64)[order]
    sig = np.asarray(opac, np.float64)[order]
    px = (np.arange(W) + 0.5)[None, :].repeat(H, 0).ravel()
    py = (np.arange(H) + 0.5)[:, None].repeat(W, 1).ravel()
    dx = px[:, None] - p["u"][order][None, :]
    dy = py[:, None] - p["v"][order][None, :]
    q = p["a"][order] * dx * dx + 2 * p["b"][order] * dx * dy + p["c"][order] * dy * dy
    inside = q <= SUPPORT_Q
    rho = np.where(inside, np.exp(-0.5 * q), 0.0)
    raw = sig[None, :] * rho
    alpha = np.minimum(raw, CLAMP)
    T = np.cumprod(np.concatenate([np.ones((alpha.shape[0], 1)), 1 - alpha[:, :-1]], 1), 1)
    wgt = alpha * T                                          # [P][M]
    contrib = wgt[..., None] * col[None]                     # [P][M][3]
    img = contrib.sum(1)
    out = {"image": img.reshape(H, W, 3)}
    scale = {"image": np.abs(contrib).sum(1).reshape(H, W, 3)}
    if grad_image is None:
        return out, scale
    g = np.asarray(grad_image, np.float64).reshape(-1, 3)
    n = len(p["z"])
    gcol = np.zeros((n, 3))
    scol = np.zeros((n, 3))
    gcol[order] = np.einsum("pm,pc->mc", wgt, g)
    scol[order] = np.einsum("pm,pc->mc", wgt, np.abs(g))
    # dC/dalpha_i = T_i c_i - S_i / (1 - alpha_i), S_i = colour behind i
    behind = np.cumsum(contrib[:, ::-1], 1)[:, ::-1] - contrib
    dca = T[..., None] * col[None] - behind / (1 - alpha)[..., None]
    sca = T[..., None] * np.abs(col)[None] + (np.cumsum(np.abs(contrib[:, ::-1]), 1)[:, ::-1]
                                              - np.abs(contrib)) / (1 - alpha)[..., None]
    dsig = np.where(raw < CLAMP, rho, 0.0)
    gop = np.zeros(n)
    sop = np.zeros(n)
    gop[order] = np.einsum("pmc,pc,pm->m", dca, g, dsig)
    sop[order] = np.einsum("pmc,pc,pm->m", sca, np.abs(g), dsig)
    out.update(colors=gcol, opac=gop)
    scale.update(colors=scol, opac=sop)
    return out, scale
