"""FP64 reference for the other lobe families of the paper's study (test
infrastructure only; see the package header).

The distribution table of Supplementary A lists the spherical functions the
paper compares; these are evaluated here on the same skeleton as the NASGabor
lobe (rgb = c0 + sum_l w_l G_l(d), frame from the quaternion or the paper's
raw values), with the stored shape slot holding each family's parameters:

* NASG (Supplementary E; the NASGabor lobe without carrier):
      G = C^{-1} e^{2 lam (kappa^(1+tau) - 1)} kappa^tau,
      C^{-1} = lam sqrt(1+a) / (2 pi (1 - e^{-2 lam})),     shape = (lam, a, -, -)
  Evaluated by the NASGabor oracle with k = zeta = 0 and the NASG normaliser.
* Spherical Gaussian (SG):
      G = c exp{lam (z.d - 1)},  c = lam / (2 pi (1 - e^{-2 lam})),   shape = (lam, -, -, -)
* Spherical beta (SB; Supplementary D normalises it over the hemisphere):
      G = (beta + 1)/(2 pi) (z.d)^beta for z.d >= 0, else 0,     shape = (beta, -, -, -)
* Spherical Cauchy (SC):
      G = 1/(4 pi) ((1 - rho^2) / (1 + rho^2 - 2 rho z.d))^2,     shape = (rho, -, -, -)
  The table prints the denominator as 1 - rho^2 - 2 rho z.d, which vanishes
  on the sphere for rho > 0 and is not a density; the cited distribution has
  1 + rho^2 - 2 rho z.d, and with it 1/(4 pi) is exactly the printed constant
  (unit mass, pinned by quadrature).
* Anisotropic spherical Gaussian (ASG):
      G = max(z.d, 0) exp{-mu (x.d)^2 - lam (y.d)^2},  y = z x x,  shape = (mu, lam, -, -)
  The table gives no normalisation constant; none is applied (c = 1).

Gradients: dG/d(parameter) (normaliser included), and the frame partials in
the form dG/dx = s_x d, dG/dy = s_y d, dG/dz = s_z d; through y = z x x a
dependence on y adds g_y x z to dL/dx and x x g_y to dL/dz. The direction
gradient is dG/dd = s_x x + s_y y + s_z z. Each output carries the rounding
scale used by the parity tests (sum of absolute elementary contributions).
"""
from __future__ import annotations

import numpy as np

from . import nasg_paper as Pp
from . import nasg_ref as R

NASGABOR, NASG, SG, SB, SC, ASG = 0, 1, 2, 3, 4, 5
NAMES = {NASGABOR: "nasgabor", NASG: "nasg", SG: "sg", SB: "sb", SC: "sc", ASG: "asg"}


def normaliser(family, shape):
    """(c, dln c/dp0, dln c/dp1) per lobe for SG, SB, SC and ASG."""
    s = np.asarray(shape, np.float64)
    p0 = s[..., 0]
    one = np.ones_like(p0)
    zero = np.zeros_like(p0)
    if family == SG:
        c, dl, _ = R.norm_approx(p0, zero)       # lam / (2 pi (1 - e^{-2 lam})) and its partial
        return c, dl / c, zero
    if family == SB:
        return (p0 + 1) / (2 * np.pi), 1.0 / (p0 + 1), zero
    if family == SC:
        return one / (4 * np.pi), zero, zero
    if family == ASG:
        return one, zero, zero
    raise ValueError("no separate normaliser for this family")


def lobe_terms(family, d, ax, ay, az, shape):
    """G and its partials per (lobe, view, primitive) for SG, SB, SC, ASG.

    Returns dict with G, the scalars sx, sy, sz (dG/daxis = s d), dG/dp0,
    dG/dp1 (normaliser included) and, for the scales, lists of the elementary
    terms of each."""
    s = np.asarray(shape, np.float64)
    p0 = s[..., 0][:, None, :]
    p1 = s[..., 1][:, None, :]
    dx = np.einsum("vnc,knc->kvn", d, ax)
    dy = np.einsum("vnc,knc->kvn", d, ay)
    dz = np.einsum("vnc,knc->kvn", d, az)
    c, dlc0, dlc1 = (t[:, None, :] for t in normaliser(family, shape))
    zero = np.zeros_like(dz)
    with np.errstate(all="ignore"):
        if family == SG:
            e = np.exp(p0 * (dz - 1))
            G = c * e
            sx, sy, sz = [zero], [zero], [p0 * G]
            dp0 = [(dz - 1) * G, dlc0 * G]
            dp1 = [zero]
        elif family == SB:
            pos = dz > 0
            t = np.where(pos, dz, 1.0)
            G = np.where(pos, c * t ** p0, 0.0)
            sx, sy = [zero], [zero]
            sz = [np.where(pos, p0 * G / t, 0.0)]
            dp0 = [np.where(pos, np.log(t) * G, 0.0), dlc0 * G]
            dp1 = [zero]
        elif family == SC:
            rho = p0
            u = 1 + rho * rho - 2 * rho * dz
            q = (1 - rho * rho) / u
            G = c * q * q
            sx, sy = [zero], [zero]
            sz = [4 * rho * G / u]
            # dG/drho = G [ -4 rho / (1 - rho^2) - 4 (rho - z.d) / u ]
            dp0 = [-4 * rho / (1 - rho * rho) * G, -4 * (rho - dz) / u * G]
            dp1 = [zero]
        elif family == ASG:
            mu, lam = p0, p1
            pos = dz > 0
            e = np.exp(-mu * dx * dx - lam * dy * dy)
            G = np.where(pos, c * dz * e, 0.0)
            sz = [np.where(pos, c * e, 0.0)]
            sx = [-2 * mu * dx * G]
            sy = [-2 * lam * dy * G]
            dp0 = [-dx * dx * G]
            dp1 = [-dy * dy * G]
        else:
            raise ValueError("unknown family")
    return dict(G=G, sx=sx, sy=sy, sz=sz, dp0=dp0, dp1=dp1)


def _frame(quat):
    """Quaternion-frame axes x, y, z [K][N][3] and a function mapping
    (dL/dx, dL/dz, their scales) to the quaternion gradient and scale."""
    q = np.asarray(quat, np.float64)
    x, y, z = R.frame_from_quat(q)

    def back(gx, gz, sx, sz):
        return R.quat_gradient(q, gx, gz, sx, sz)
    return x, y, z, back


def forward_backward(family, quat, shape, rgbw, c0, grad_rgb, means=None, cams=None, dirs=None,
                     param="quat"):
    """Colours and the gradients of L = sum(grad_rgb * rgb) for a family
    other than NASGabor, each with its rounding scale. Keys as
    ``nasg_ref.forward_backward``; unused shape slots get zero gradients."""
    if family == NASG:
        s = np.array(shape, np.float64)
        s[..., 2:] = 0.0
        if param == "angles":
            s[..., 2] = -np.inf                       # k = 20 (tanh u + 1) = 0
            out, scale = Pp.forward_backward(quat, s, rgbw, c0, grad_rgb, R.NORM_APPROX,
                                             means, cams, dirs)
        else:
            out, scale = R.forward_backward(quat, s, rgbw, c0, grad_rgb, R.NORM_APPROX,
                                            means, cams, dirs)
        out["shape"][..., 2:] = 0.0
        scale["shape"][..., 2:] = 0.0
        return out, scale
    if param != "quat":
        raise ValueError("the paper's raw values are defined for NASGabor and NASG only")
    x, y, z, back = _frame(quat)
    d, r = R.view_directions(means, cams, dirs)
    t = lobe_terms(family, d, x, y, z, shape)
    w = np.transpose(np.asarray(rgbw, np.float64), (0, 2, 1))   # [K][N][3]
    g = np.asarray(grad_rgb, np.float64)
    c0 = np.asarray(c0, np.float64)
    G = t["G"]
    contrib = G[..., None] * w[:, None, :, :]
    out = {"rgb": c0[None] + contrib.sum(0)}
    scale = {"rgb": np.abs(c0)[None] + np.abs(contrib).sum(0)}
    gw = g[None] * w[:, None, :, :]
    gG = gw.sum(-1)
    gGa = np.abs(gw).sum(-1)

    def red(terms):
        tot = sum(terms)
        ab = sum(np.abs(x_) for x_ in terms)
        return (gG * tot).sum(1), (gGa * ab).sum(1), tot, ab

    g0, s0, _, _ = red(t["dp0"])
    g1, s1, _, _ = red(t["dp1"])
    _, _, sx, sxa = red(t["sx"])
    _, _, sy, sya = red(t["sy"])
    _, _, sz, sza = red(t["sz"])
    zk = np.zeros_like(g0)
    out["shape"] = np.stack([g0, g1, zk, zk], -1)
    scale["shape"] = np.stack([s0, s1, zk, zk], -1)

    gx = np.einsum("kvn,vnc->knc", gG * sx, d)
    gy = np.einsum("kvn,vnc->knc", gG * sy, d)
    gz = np.einsum("kvn,vnc->knc", gG * sz, d)
    ax_ = np.einsum("kvn,vnc->knc", gGa * sxa, np.abs(d))
    ay_ = np.einsum("kvn,vnc->knc", gGa * sya, np.abs(d))
    az_ = np.einsum("kvn,vnc->knc", gGa * sza, np.abs(d))
    # y = z x x: dL/dx += g_y x z, dL/dz += x x g_y
    gx_t = gx + np.cross(gy, z)
    gz_t = gz + np.cross(x, gy)
    # scale of a x b: component m gets |a_j| |b_k| + |a_k| |b_j|
    abs_cross = lambda a, b: np.abs(np.cross(np.abs(a)[..., None, :] * np.eye(3),  # noqa: E731
                                             b[..., None, :])).sum(-2)
    ax_t = ax_ + abs_cross(ay_, z)
    az_t = az_ + abs_cross(ay_, x)
    out["quat"], scale["quat"] = back(gx_t, gz_t, ax_t, az_t)

    out["rgbw"] = np.einsum("vnc,kvn->kcn", g, G)
    scale["rgbw"] = np.einsum("vnc,kvn->kcn", np.abs(g), np.abs(G))
    out["c0"] = g.sum(0)
    scale["c0"] = np.abs(g).sum(0)

    gd = (np.einsum("kvn,knc->vnc", gG * sx, x) + np.einsum("kvn,knc->vnc", gG * sy, y)
          + np.einsum("kvn,knc->vnc", gG * sz, z))
    sd = (np.einsum("kvn,knc->vnc", gGa * sxa, np.abs(x)) + np.einsum("kvn,knc->vnc", gGa * sya, np.abs(y))
          + np.einsum("kvn,knc->vnc", gGa * sza, np.abs(z)))
    proj = np.eye(3)[None, None] - d[..., :, None] * d[..., None, :]
    ge = np.einsum("vnij,vnj->vni", proj, gd) / r[..., None]
    # the projection's two terms (identity and d d^T) count as separate
    # elementary contributions: (|g| + |d| (|d| . |g|)) / |e|
    se = (sd + np.abs(d) * (np.abs(d) * sd).sum(-1, keepdims=True)) / r[..., None]
    key = "dirs" if dirs is not None else "means"
    out[key] = ge.sum(0)
    scale[key] = se.sum(0)
    return out, scale


def forward(family, quat, shape, rgbw, c0, means=None, cams=None, dirs=None, param="quat"):
    """rgb [V][N][3] and its rounding scale."""
    v = 1 if dirs is not None else np.asarray(cams).shape[0]
    n = np.asarray(c0).shape[0]
    out, scale = forward_backward(family, quat, shape, rgbw, c0, np.zeros((v, n, 3)), means, cams,
                                  dirs, param)
    return out["rgb"], scale["rgb"]


def lobe_value(family, d, q, shape):
    """G of one lobe (quaternion frame) at unit directions d [M][3]."""
    d = np.asarray(d, np.float64).reshape(-1, 3)
    x, y, z = R.frame_from_quat(np.asarray(q, np.float64)[None, None])
    s = np.asarray(shape, np.float64)[None, None]
    if family == NASG:
        s = s.copy()
        s[..., 2:] = 0.0
        return R.lobe_value(d, q, s[0, 0], R.NORM_APPROX)
    t = lobe_terms(family, d[:, None, :], x, y, z, s)
    return t["G"][0, :, 0]
