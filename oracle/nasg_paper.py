"""FP64 reference for the paper's own lobe parametrisation (test
infrastructure only; see the package header).

Supplementary C gives each lobe nine stored values, all pre-activation
("raw") numbers u that an optimiser updates directly:

* frame: three cosines c = tanh(u) (activation table), with the sines
  s = +sqrt(1 - c^2) (so theta, phi, psi lie in [0, pi]). For c = tanh(u)
  that sine is sech(u) and is evaluated as 1/cosh(u): the same value, but
  1 - c^2 of a rounded c near +-1 would lose the digits the sine needs. The
  mean direction and the tangent axis are
      z = (c_theta s_phi, s_theta s_phi, c_phi),
      x = (c_theta c_phi c_psi - s_theta s_psi,
           s_theta c_phi c_psi + c_theta s_psi,
           -s_phi c_psi),
  and y = z cross x completes R = [x y z]. (The supplement names the in-plane
  angle tau in the construction and psi in the derivatives; it is one angle,
  called psi here because tau is the anisotropy exponent of the lobe.)
* bandwidths lam = exp(u), a = exp(u); frequency k = 20 (tanh(u) + 1);
* colour weights w = tanh(u).

A fourth value in the shape slot is the carrier phase zeta, passed through
without activation (zeta = 0 is the paper's carrier); the fourth frame slot
is unused.

Gradients: the evaluation core of ``nasg_ref`` gives dL/dx, dL/dz and the
gradients with respect to the activated lam, a, k, zeta and w. The frame
derivatives follow Supplementary F: dG/dc = dG/dx . dx/dc + dG/dz . dz/dc
with the printed Jacobians of x and z in c_theta, c_phi, c_psi (they use
ds/dc = -c/s); each activated gradient is then multiplied by the derivative
of its activation (sech^2 u = 1 - tanh^2 u for tanh, evaluated as
1/cosh^2(u); the value itself for exp; 20 sech^2 u for k). The rounding scale
of each raw gradient is the activated one times the absolute chain factor.
"""
from __future__ import annotations

import numpy as np

from . import nasg_ref as R


def activate(frame_raw, shape_raw, rgbw_raw):
    """Activated lobe values (activation table of Supplementary C).

    frame_raw [K][N][4] -> cosines [K][N][3]; shape_raw [K][N][4] ->
    (lam, a, k, zeta) [K][N][4]; rgbw_raw [K][3][N] -> weights [K][3][N]."""
    f = np.asarray(frame_raw, np.float64)
    sr = np.asarray(shape_raw, np.float64)
    cos = np.tanh(f[..., :3])
    shape = np.stack([np.exp(sr[..., 0]), np.exp(sr[..., 1]),
                      20.0 * (np.tanh(sr[..., 2]) + 1.0), sr[..., 3]], -1)
    w = np.tanh(np.asarray(rgbw_raw, np.float64))
    return cos, shape, w


def sech(u):
    """sech u = sqrt(1 - tanh^2 u) (the square root of d tanh(u)/du), as
    1/cosh(u)."""
    with np.errstate(over="ignore"):
        return 1.0 / np.cosh(np.asarray(u, np.float64))


def _sines(cos, sin):
    return np.sqrt(1 - cos * cos) if sin is None else sin


def frame_from_cosines(cos, sin=None):
    """Columns x, y, z of R for cosines (c_theta, c_phi, c_psi) [..., 3]
    (sines sqrt(1 - c^2), or ``sin`` when given)."""
    ct, cp, cs = cos[..., 0], cos[..., 1], cos[..., 2]
    sn = _sines(cos, sin)
    st, sp, ss = sn[..., 0], sn[..., 1], sn[..., 2]
    z = np.stack([ct * sp, st * sp, cp], -1)
    x = np.stack([ct * cp * cs - st * ss, st * cp * cs + ct * ss, -sp * cs], -1)
    y = np.cross(z, x)
    return x, y, z


def frame_cosine_jacobians(cos, sin=None):
    """dx/dc and dz/dc for c = (c_theta, c_phi, c_psi), each [..., 3 (axis
    component), 3 (which cosine)], as printed in Supplementary F."""
    ct, cp, cs = cos[..., 0], cos[..., 1], cos[..., 2]
    sn = _sines(cos, sin)
    st, sp, ss = sn[..., 0], sn[..., 1], sn[..., 2]
    zero = np.zeros_like(ct)
    one = np.ones_like(ct)
    with np.errstate(all="ignore"):
        dx_dct = np.stack([cp * cs + ct / st * ss, -ct / st * cp * cs + ss, zero], -1)
        dz_dct = np.stack([sp, -ct / st * sp, zero], -1)
        dx_dcp = np.stack([ct * cs, st * cs, cp / sp * cs], -1)
        dz_dcp = np.stack([-ct * cp / sp, -st * cp / sp, one], -1)
        dx_dcs = np.stack([ct * cp + st * cs / ss, st * cp - ct * cs / ss, -sp], -1)
        dz_dcs = np.stack([zero, zero, zero], -1)
    jx = np.stack([dx_dct, dx_dcp, dx_dcs], -1)
    jz = np.stack([dz_dct, dz_dcp, dz_dcs], -1)
    return jx, jz


def forward(frame_raw, shape_raw, rgbw_raw, c0, norm, means=None, cams=None, dirs=None):
    """rgb [V][N][3] and its rounding scale."""
    cos, shape, w = activate(frame_raw, shape_raw, rgbw_raw)
    x, _, z = frame_from_cosines(cos, sech(np.asarray(frame_raw, np.float64)[..., :3]))
    d, _ = R.view_directions(means, cams, dirs)
    Cn = R.normaliser(shape, norm)[0]
    t = R.lobe_terms(d, x, z, shape, Cn)
    wk = np.transpose(w, (0, 2, 1))
    contrib = t["G"][..., None] * wk[:, None, :, :]
    c0 = np.asarray(c0, np.float64)
    return c0[None] + contrib.sum(0), np.abs(c0)[None] + np.abs(contrib).sum(0)


def forward_backward(frame_raw, shape_raw, rgbw_raw, c0, grad_rgb, norm, means=None,
                     cams=None, dirs=None):
    """Colours and the gradients of L = sum(grad_rgb * rgb) w.r.t. the raw
    frame, shape and weight values, c0 and the means (or dirs), each with its
    rounding scale. Keys as ``nasg_ref.forward_backward``; "quat" holds the
    raw frame gradient (fourth component 0)."""
    cos, shape, w = activate(frame_raw, shape_raw, rgbw_raw)
    sin = sech(np.asarray(frame_raw, np.float64)[..., :3])
    x, _, z = frame_from_cosines(cos, sin)
    out, scale, axes = R.frame_forward_backward(x, z, shape, w, c0, grad_rgb, norm,
                                                means, cams, dirs)
    gx, gz, sx, sz = axes
    jx, jz = frame_cosine_jacobians(cos, sin)
    g_cos = np.einsum("knci,knc->kni", jx, gx) + np.einsum("knci,knc->kni", jz, gz)
    s_cos = (np.einsum("knci,knc->kni", np.abs(jx), sx)
             + np.einsum("knci,knc->kni", np.abs(jz), sz))
    dcos = sin * sin                                       # d tanh(u)/du = sech^2 u
    zero = np.zeros(g_cos.shape[:-1] + (1,))
    out["quat"] = np.concatenate([g_cos * dcos, zero], -1)
    scale["quat"] = np.concatenate([s_cos * dcos, zero], -1)

    sr = np.asarray(shape_raw, np.float64)
    sk = sech(sr[..., 2])
    chain = np.stack([shape[..., 0], shape[..., 1], 20.0 * sk * sk, np.ones_like(sk)], -1)
    out["shape"] = out["shape"] * chain
    scale["shape"] = scale["shape"] * np.abs(chain)

    dw = sech(rgbw_raw) ** 2
    out["rgbw"] = out["rgbw"] * dw
    scale["rgbw"] = scale["rgbw"] * dw
    return out, scale


def quat_from_frame(x, y, z):
    """A unit quaternion (w, x, y, z) whose rotation has columns x, y, z
    (the standard trace-based conversion; used to compare with the
    quaternion parametrisation)."""
    m = np.stack([x, y, z], -1)                              # [..., 3, 3], columns
    tr = m[..., 0, 0] + m[..., 1, 1] + m[..., 2, 2]
    q = np.empty(m.shape[:-2] + (4,))
    c0 = tr > 0
    c1 = (~c0) & (m[..., 0, 0] >= m[..., 1, 1]) & (m[..., 0, 0] >= m[..., 2, 2])
    c2 = (~c0) & (~c1) & (m[..., 1, 1] >= m[..., 2, 2])
    c3 = ~(c0 | c1 | c2)
    with np.errstate(all="ignore"):
        s = np.sqrt(tr + 1.0) * 2
        q0 = np.stack([0.25 * s, (m[..., 2, 1] - m[..., 1, 2]) / s,
                       (m[..., 0, 2] - m[..., 2, 0]) / s, (m[..., 1, 0] - m[..., 0, 1]) / s], -1)
        s = np.sqrt(1.0 + m[..., 0, 0] - m[..., 1, 1] - m[..., 2, 2]) * 2
        q1 = np.stack([(m[..., 2, 1] - m[..., 1, 2]) / s, 0.25 * s,
                       (m[..., 0, 1] + m[..., 1, 0]) / s, (m[..., 0, 2] + m[..., 2, 0]) / s], -1)
        s = np.sqrt(1.0 + m[..., 1, 1] - m[..., 0, 0] - m[..., 2, 2]) * 2
        q2 = np.stack([(m[..., 0, 2] - m[..., 2, 0]) / s, (m[..., 0, 1] + m[..., 1, 0]) / s,
                       0.25 * s, (m[..., 1, 2] + m[..., 2, 1]) / s], -1)
        s = np.sqrt(1.0 + m[..., 2, 2] - m[..., 0, 0] - m[..., 1, 1]) * 2
        q3 = np.stack([(m[..., 1, 0] - m[..., 0, 1]) / s, (m[..., 0, 2] + m[..., 2, 0]) / s,
                       (m[..., 1, 2] + m[..., 2, 1]) / s, 0.25 * s], -1)
    for c, qq in ((c0, q0), (c1, q1), (c2, q2), (c3, q3)):
        q[c] = qq[c]
    return q
