"""FP64 real spherical harmonics up to degree 3 (test infrastructure only).

The comparison appearance model of Section 3.2: f(d) = sum_{l<=3} sum_m
c_lm Y_l^m(d), one coefficient per basis function and colour channel
(16 x 3 = 48 per primitive). The paper does not fix the real-basis
convention; this oracle uses the real orthonormal basis built from the
complex harmonics with the Condon-Shortley phase:
    Y_lm = sqrt(2) Re Y_l^m (m > 0),  Y_l^0 (m = 0),  sqrt(2) Im Y_l^|m| (m < 0),
stored at index l^2 + l + m. No offset and no clamp is applied.

Each Y_lm is written as a polynomial in the unit direction (x, y, z): the
normalisation sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for m != 0)
multiplies the associated Legendre factor P_l^|m| (with its (-1)^m) and the
real or imaginary part of (x + i y)^|m|. Values, gradients and the rounding
scales (sums of absolute monomials, the natural size of a floating-point
evaluation of the polynomial) are all computed from the one monomial table.
"""
from __future__ import annotations

import math

import numpy as np

from .nasg_ref import view_directions

_PI = math.pi
_S2 = math.sqrt(2.0)


def _k(l, m):
    return math.sqrt((2 * l + 1) / (4 * _PI) * math.factorial(l - abs(m)) / math.factorial(l + abs(m)))


# (prefactor, [(coefficient, (px, py, pz)), ...]) per basis index
_TABLE = [
    (_k(0, 0), [(1.0, (0, 0, 0))]),
    # l = 1: P_1^0 = z, P_1^1 = -sin(theta); Im/Re of (x + i y) = y / x
    (-_S2 * _k(1, 1), [(1.0, (0, 1, 0))]),
    (_k(1, 0), [(1.0, (0, 0, 1))]),
    (-_S2 * _k(1, 1), [(1.0, (1, 0, 0))]),
    # l = 2: P_2^0 = (3z^2-1)/2, P_2^1 = -3 z sin, P_2^2 = 3 sin^2
    (3.0 * _S2 * _k(2, 2), [(2.0, (1, 1, 0))]),
    (-3.0 * _S2 * _k(2, 1), [(1.0, (0, 1, 1))]),
    (0.5 * _k(2, 0), [(3.0, (0, 0, 2)), (-1.0, (0, 0, 0))]),
    (-3.0 * _S2 * _k(2, 1), [(1.0, (1, 0, 1))]),
    (3.0 * _S2 * _k(2, 2), [(1.0, (2, 0, 0)), (-1.0, (0, 2, 0))]),
    # l = 3: P_3^0 = (5z^3-3z)/2, P_3^1 = -3/2 (5z^2-1) sin, P_3^2 = 15 z sin^2,
    #        P_3^3 = -15 sin^3; (x+iy)^2 = x^2-y^2 + 2ixy, (x+iy)^3 = x^3-3xy^2 + i(3x^2y-y^3)
    (-15.0 * _S2 * _k(3, 3), [(3.0, (2, 1, 0)), (-1.0, (0, 3, 0))]),
    (15.0 * _S2 * _k(3, 2), [(2.0, (1, 1, 1))]),
    (-1.5 * _S2 * _k(3, 1), [(5.0, (0, 1, 2)), (-1.0, (0, 1, 0))]),
    (0.5 * _k(3, 0), [(5.0, (0, 0, 3)), (-3.0, (0, 0, 1))]),
    (-1.5 * _S2 * _k(3, 1), [(5.0, (1, 0, 2)), (-1.0, (1, 0, 0))]),
    (15.0 * _S2 * _k(3, 2), [(1.0, (2, 0, 1)), (-1.0, (0, 2, 1))]),
    (-15.0 * _S2 * _k(3, 3), [(1.0, (3, 0, 0)), (-3.0, (1, 2, 0))]),
]


def _mono(d, p):
    return d[..., 0] ** p[0] * d[..., 1] ** p[1] * d[..., 2] ** p[2]


def _dmono(d, p, axis):
    """Partial derivative of x^px y^py z^pz along `axis`."""
    if p[axis] == 0:
        return np.zeros(d.shape[:-1])
    q = list(p)
    q[axis] -= 1
    return p[axis] * _mono(d, q)


def basis(d):
    """Y[..., 16] at unit directions d[..., 3]."""
    d = np.asarray(d, np.float64)
    return np.stack([pre * sum(c * _mono(d, p) for c, p in terms) for pre, terms in _TABLE], -1)


def basis_abs(d):
    """Sum of |monomials| of each Y_j: the rounding scale of evaluating it."""
    d = np.asarray(d, np.float64)
    return np.stack([abs(pre) * sum(abs(c) * np.abs(_mono(d, p)) for c, p in terms)
                     for pre, terms in _TABLE], -1)


def basis_grad(d, absolute=False):
    """dY/dd[..., 16, 3] of the polynomials (unprojected); with absolute=True,
    the sums of |monomials| of each partial derivative."""
    d = np.asarray(d, np.float64)
    f = np.abs if absolute else (lambda x: x)
    out = []
    for pre, terms in _TABLE:
        comp = []
        for ax in range(3):
            comp.append(f(pre) * sum(f(c * _dmono(d, p, ax)) for c, p in terms))
        out.append(np.stack(comp, -1))
    return np.stack(out, -2)


def forward(sh, means=None, cams=None, dirs=None):
    """rgb [V][N][3] = sum_j sh[j][c][n] Y_j(d_vn), with its rounding scale."""
    sh = np.asarray(sh, np.float64)                   # [16][3][N]
    d, _ = view_directions(means, cams, dirs)
    Y = basis(d)                                      # [V][N][16]
    rgb = np.einsum("vnj,jcn->vnc", Y, sh)
    scale = np.einsum("vnj,jcn->vnc", basis_abs(d), np.abs(sh))
    return rgb, scale


def forward_backward(sh, grad_rgb, means=None, cams=None, dirs=None):
    """rgb plus gradients of L = sum(grad_rgb * rgb) w.r.t. sh and the means
    (or raw directions), each with its rounding scale."""
    sh = np.asarray(sh, np.float64)
    g = np.asarray(grad_rgb, np.float64)              # [V][N][3]
    d, r = view_directions(means, cams, dirs)
    Y = basis(d)
    Ya = basis_abs(d)
    dY = basis_grad(d)                                # [V][N][16][3]
    dYa = basis_grad(d, absolute=True)
    out = {"rgb": np.einsum("vnj,jcn->vnc", Y, sh)}
    scale = {"rgb": np.einsum("vnj,jcn->vnc", Ya, np.abs(sh))}
    out["sh"] = np.einsum("vnc,vnj->jcn", g, Y)
    scale["sh"] = np.einsum("vnc,vnj->jcn", np.abs(g), Ya)
    beta = np.einsum("vnc,jcn->vnj", g, sh)           # dL/dY_j
    beta_a = np.einsum("vnc,jcn->vnj", np.abs(g), np.abs(sh))
    gd = np.einsum("vnj,vnji->vni", beta, dY)
    sd = np.einsum("vnj,vnji->vni", beta_a, dYa)
    proj = np.eye(3)[None, None] - d[..., :, None] * d[..., None, :]
    ge = np.einsum("vnij,vnj->vni", proj, gd) / r[..., None]
    se = np.einsum("vnij,vnj->vni", np.abs(proj), sd) / r[..., None]
    key = "dirs" if dirs is not None else "means"
    out[key] = ge.sum(0)
    scale[key] = se.sum(0)
    return out, scale
