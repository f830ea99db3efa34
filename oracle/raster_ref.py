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
rho when unclamped, 0 when clamped), and with respect to the geometry (means,
scales, quaternions) through rho: dalpha/dq = -sigma rho / 2 below the clamp,
q = a dx^2 + 2 b dx dy + c dy^2 with (a, b; b, c) = Sigma_2^{-1} and
(dx, dy) = pixel centre - (u, v); the support cut q <= 9, the near plane
and the clamp are taken as fixed (their jumps have no derivative). The chain
from the per-primitive sums dL/du, dL/dv, dL/da, dL/db, dL/dc to the 3D
parameters follows the definitions: d(Sigma^{-1}) = -Sigma^{-1} dSigma
Sigma^{-1}, Sigma_2 = M M^T with M = J R_cw R(q/|q|) S, and J, u, v functions
of the camera-space mean.
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


def quat_rotation_jacobian(q):
    """dR/dq for R = quat_rotation(q): [N][3][3][4], including the
    normalisation q -> q/|q| (by the chain through the unit quaternion)."""
    q = np.asarray(q, np.float64)
    nq = np.linalg.norm(q, axis=-1, keepdims=True)
    u = q / nq
    w, x, y, z = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
    zero = np.zeros_like(w)
    # partial derivatives of the unit-quaternion rotation matrix, per component
    dw = np.stack([np.stack([zero, -2 * z, 2 * y], -1), np.stack([2 * z, zero, -2 * x], -1),
                   np.stack([-2 * y, 2 * x, zero], -1)], -2)
    dx = np.stack([np.stack([zero, 2 * y, 2 * z], -1), np.stack([2 * y, -4 * x, -2 * w], -1),
                   np.stack([2 * z, 2 * w, -4 * x], -1)], -2)
    dy = np.stack([np.stack([-4 * y, 2 * x, 2 * w], -1), np.stack([2 * x, zero, 2 * z], -1),
                   np.stack([-2 * w, 2 * z, -4 * y], -1)], -2)
    dz = np.stack([np.stack([-4 * z, -2 * w, 2 * x], -1), np.stack([2 * w, -4 * z, 2 * y], -1),
                   np.stack([2 * x, 2 * y, zero], -1)], -2)
    du = np.stack([dw, dx, dy, dz], -1)                          # dR/du  [N][3][3][4]
    proj = (np.eye(4)[None] - u[:, :, None] * u[:, None, :]) / nq[:, :, None]   # du/dq
    return du @ proj[:, None]


def geometry_chain(means, scales, rots, cam, g2):
    """Gradients w.r.t. means [N][3], scales [N][3] and quaternions [N][4]
    from the per-primitive sums g2 [N][5] = (dL/du, dL/dv, dL/da, dL/db,
    dL/dc) (b the conic's off-diagonal entry). Linear in g2."""
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    fx, fy = float(cam["fx"]), float(cam["fy"])
    m = np.asarray(means, np.float64)
    xc = m @ R.T + t
    X, Y, Z = xc[:, 0], xc[:, 1], xc[:, 2]
    Zs = np.where(Z > NEAR, Z, 1.0)
    Rw = quat_rotation(rots)
    s = np.asarray(scales, np.float64)
    A = R[None] @ Rw * s[:, None, :]                              # R_cw R_w S  [N][3][3]
    J = np.zeros((m.shape[0], 2, 3))
    J[:, 0, 0] = fx / Zs
    J[:, 0, 2] = -fx * X / (Zs * Zs)
    J[:, 1, 1] = fy / Zs
    J[:, 1, 2] = -fy * Y / (Zs * Zs)
    M = J @ A                                                     # [N][2][3]
    S2 = M @ np.swapaxes(M, -1, -2)
    K = np.linalg.inv(S2)
    g2 = np.asarray(g2, np.float64)
    gK = np.zeros((m.shape[0], 2, 2))
    gK[:, 0, 0] = g2[:, 2]
    gK[:, 1, 1] = g2[:, 4]
    gK[:, 0, 1] = gK[:, 1, 0] = 0.5 * g2[:, 3]
    gS2 = -K @ gK @ K                                             # d(S^-1) = -S^-1 dS S^-1
    gM = 2.0 * gS2 @ M                                            # S2 = M M^T, gS2 symmetric
    gJ = gM @ np.swapaxes(A, -1, -2)                              # [N][2][3]
    gA = np.swapaxes(J, -1, -2) @ gM                              # [N][3][3]
    gRS = np.swapaxes(R, -1, -2)[None] @ gA                       # d/d(R_w S)
    g_scales = np.einsum("nij,nij->nj", gRS, Rw)
    gRw = gRS * s[:, None, :]
    g_rots = np.einsum("nij,nijk->nk", gRw, quat_rotation_jacobian(rots))
    # camera-space mean: through (u, v) and J
    gX = g2[:, 0] * fx / Zs - gJ[:, 0, 2] * fx / (Zs * Zs)
    gY = g2[:, 1] * fy / Zs - gJ[:, 1, 2] * fy / (Zs * Zs)
    gZ = (-g2[:, 0] * fx * X / (Zs * Zs) - g2[:, 1] * fy * Y / (Zs * Zs)
          - gJ[:, 0, 0] * fx / (Zs * Zs) + gJ[:, 0, 2] * 2 * fx * X / Zs ** 3
          - gJ[:, 1, 1] * fy / (Zs * Zs) + gJ[:, 1, 2] * 2 * fy * Y / Zs ** 3)
    g_means = np.stack([gX, gY, gZ], -1) @ R
    vis = (Z > NEAR)[:, None]
    return (np.where(vis, g_means, 0.0), np.where(vis, g_scales, 0.0),
            np.where(vis, g_rots, 0.0))


def render(means, scales, rots, opac, colors, cam, grad_image=None, geometry=False):
    """Image [H][W][3] (and, with grad_image, the gradients w.r.t. colours
    [N][3] and opacities [N]; with geometry=True also means, scales and
    rots) with rounding scales."""
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
    if not geometry:
        return out, scale
    # dL/dq per pixel and primitive (zero outside the support and at the clamp)
    sg = sig[None, :]
    dq = np.where(raw < CLAMP, -0.5 * sg * rho, 0.0) * np.einsum("pmc,pc->pm", dca, g)
    sdq = np.where(raw < CLAMP, 0.5 * sg * rho, 0.0) * np.einsum("pmc,pc->pm", sca, np.abs(g))
    a_, b_, c_ = p["a"][order], p["b"][order], p["c"][order]
    terms = [(-2.0 * (a_ * dx + b_ * dy), 2.0 * (np.abs(a_ * dx) + np.abs(b_ * dy))),
             (-2.0 * (b_ * dx + c_ * dy), 2.0 * (np.abs(b_ * dx) + np.abs(c_ * dy))),
             (dx * dx, dx * dx), (2.0 * dx * dy, 2.0 * np.abs(dx * dy)), (dy * dy, dy * dy)]
    g2 = np.zeros((n, 5))
    s2 = np.zeros((n, 5))
    for j, (d_, sd_) in enumerate(terms):
        g2[order, j] = (dq * d_).sum(0)
        s2[order, j] = (sdq * sd_).sum(0)
    gm, gs, gr = geometry_chain(means, scales, rots, cam, g2)
    # the chain is linear in g2: push the unit vectors through it for the
    # Jacobian, and bound the propagated rounding by |Jacobian| x scale
    jac = [geometry_chain(means, scales, rots, cam, np.eye(5)[None, j].repeat(n, 0))
           for j in range(5)]
    out.update(means=gm, scales=gs, rots=gr, g2=g2)
    scale.update(means=sum(np.abs(jac[j][0]) * s2[:, j:j + 1] for j in range(5)),
                 scales=sum(np.abs(jac[j][1]) * s2[:, j:j + 1] for j in range(5)),
                 rots=sum(np.abs(jac[j][2]) * s2[:, j:j + 1] for j in range(5)), g2=s2)
    return out, scale
