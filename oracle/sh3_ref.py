"""FP64 real spherical harmonics up to degree 3 (test infrastructure only).

The comparison appearance model of Section 3.2: f(d) = sum_{l<=3} sum_m
c_lm Y_l^m(d), one coefficient per basis function and colour channel
(16 x 3 = 48 per primitive). The paper does not fix the real-basis
convention; this oracle uses the real orthonormal basis built from the
complex harmonics with the Condon-Shortley phase:
    Y_lm = sqrt(2) Re Y_l^m (m > 0),  Y_l^0 (m = 0),  sqrt(2) Im Y_l^|m| (m < 0),
stored at index l^2 + l + m. Values are written as polynomials in the unit
direction (x, y, z), each with its closed-form normalisation constant
sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the Legendre/azimuthal factors.
No offset and no clamp is applied to the output.
"""
from __future__ import annotations

import math

import numpy as np

from .nasg_ref import view_directions

_PI = math.pi


def _k(l, m):
    return math.sqrt((2 * l + 1) / (4 * _PI) * math.factorial(l - abs(m)) / math.factorial(l + abs(m)))


# Y_lm = K_lm * (sqrt 2 for m != 0) * P_l^|m| part * azimuthal polynomial.
# With the Condon-Shortley phase P_l^m carries (-1)^m.
def basis(d):
    """Y[..., 16] at unit directions d[..., 3]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    s2 = math.sqrt(2.0)
    Y = [None] * 16
    # l = 0
    Y[0] = _k(0, 0) * np.ones_like(x)
    # l = 1: P_1^0 = z, P_1^1 = -sin(theta)
    Y[1] = s2 * _k(1, 1) * (-1.0) * y
    Y[2] = _k(1, 0) * z
    Y[3] = s2 * _k(1, 1) * (-1.0) * x
    # l = 2: P_2^0 = (3z^2-1)/2, P_2^1 = -3 z sin, P_2^2 = 3 sin^2
    Y[4] = s2 * _k(2, 2) * 3.0 * (2 * x * y)
    Y[5] = s2 * _k(2, 1) * (-3.0) * z * y
    Y[6] = _k(2, 0) * 0.5 * (3 * z * z - 1)
    Y[7] = s2 * _k(2, 1) * (-3.0) * z * x
    Y[8] = s2 * _k(2, 2) * 3.0 * (x * x - y * y)
    # l = 3: P_3^0 = (5z^3-3z)/2, P_3^1 = -3/2 (5z^2-1) sin,
    #        P_3^2 = 15 z sin^2, P_3^3 = -15 sin^3
    Y[9] = s2 * _k(3, 3) * (-15.0) * (3 * x * x * y - y ** 3)
    Y[10] = s2 * _k(3, 2) * 15.0 * z * (2 * x * y)
    Y[11] = s2 * _k(3, 1) * (-1.5) * (5 * z * z - 1) * y
    Y[12] = _k(3, 0) * 0.5 * (5 * z ** 3 - 3 * z)
    Y[13] = s2 * _k(3, 1) * (-1.5) * (5 * z * z - 1) * x
    Y[14] = s2 * _k(3, 2) * 15.0 * z * (x * x - y * y)
    Y[15] = s2 * _k(3, 3) * (-15.0) * (x ** 3 - 3 * x * y * y)
    return np.stack(Y, -1)


def basis_grad(d):
    """dY/dd[..., 16, 3] of the polynomials in ``basis`` (unprojected)."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    o = np.zeros_like(x)
    one = np.ones_like(x)
    s2 = math.sqrt(2.0)
    g = [None] * 16
    g[0] = (o, o, o)
    c = -s2 * _k(1, 1)
    g[1] = (o, c * one, o)
    g[2] = (o, o, _k(1, 0) * one)
    g[3] = (c * one, o, o)
    c = s2 * _k(2, 2) * 3.0
    g[4] = (2 * c * y, 2 * c * x, o)
    c = -3.0 * s2 * _k(2, 1)
    g[5] = (o, c * z, c * y)
    g[6] = (o, o, _k(2, 0) * 3 * z)
    g[7] = (c * z, o, c * x)
    c = s2 * _k(2, 2) * 3.0
    g[8] = (2 * c * x, -2 * c * y, o)
    c = -15.0 * s2 * _k(3, 3)
    g[9] = (c * 6 * x * y, c * (3 * x * x - 3 * y * y), o)
    c = 15.0 * s2 * _k(3, 2)
    g[10] = (c * 2 * y * z, c * 2 * x * z, c * 2 * x * y)
    c = -1.5 * s2 * _k(3, 1)
    g[11] = (o, c * (5 * z * z - 1), c * 10 * z * y)
    g[12] = (o, o, _k(3, 0) * 0.5 * (15 * z * z - 3))
    g[13] = (c * (5 * z * z - 1), o, c * 10 * z * x)
    c = 15.0 * s2 * _k(3, 2)
    g[14] = (c * 2 * x * z, -c * 2 * y * z, c * (x * x - y * y))
    c = -15.0 * s2 * _k(3, 3)
    g[15] = (c * (3 * x * x - 3 * y * y), -c * 6 * x * y, o)
    return np.stack([np.stack(t, -1) for t in g], -2)


def forward(sh, means=None, cams=None, dirs=None):
    """rgb [V][N][3] = sum_j sh[j][c][n] Y_j(d_vn), with its abs scale."""
    sh = np.asarray(sh, np.float64)                   # [16][3][N]
    d, _ = view_directions(means, cams, dirs)
    Y = basis(d)                                      # [V][N][16]
    terms = np.einsum("vnj,jcn->vncj", Y, sh)
    return terms.sum(-1), np.abs(terms).sum(-1)


def forward_backward(sh, grad_rgb, means=None, cams=None, dirs=None):
    """rgb plus gradients of L = sum(grad_rgb * rgb) w.r.t. sh and the means
    (or raw directions), each with its rounding scale."""
    sh = np.asarray(sh, np.float64)
    g = np.asarray(grad_rgb, np.float64)              # [V][N][3]
    d, r = view_directions(means, cams, dirs)
    Y = basis(d)
    dY = basis_grad(d)                                # [V][N][16][3]
    terms = np.einsum("vnj,jcn->vncj", Y, sh)
    out = {"rgb": terms.sum(-1)}
    scale = {"rgb": np.abs(terms).sum(-1)}
    out["sh"] = np.einsum("vnc,vnj->jcn", g, Y)
    scale["sh"] = np.einsum("vnc,vnj->jcn", np.abs(g), np.abs(Y))
    beta = np.einsum("vnc,jcn->vnj", g, sh)           # dL/dY_j
    beta_a = np.einsum("vnc,jcn->vnj", np.abs(g), np.abs(sh))
    gd = np.einsum("vnj,vnji->vni", beta, dY)
    sd = np.einsum("vnj,vnji->vni", beta_a, np.abs(dY))
    proj = np.eye(3)[None, None] - d[..., :, None] * d[..., None, :]
    ge = np.einsum("vnij,vnj->vni", proj, gd) / r[..., None]
    se = np.einsum("vnij,vnj->vni", np.abs(proj), sd) / r[..., None]
    key = "dirs" if dirs is not None else "means"
    out[key] = ge.sum(0)
    scale[key] = se.sum(0)
    return out, scale
