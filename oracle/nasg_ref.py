"""FP64 NASGabor reference (test infrastructure only; see the package header).

Everything is evaluated in float64 from the stored float32 / bfloat16 values,
vectorised over primitives, lobes and views, written term by term from the
paper:

* Appearance model (Section 4.2, appearance-model equation):
      rgb(d) = c0 + sum_l w_l G_l(d)
* NASGabor lobe (Section 5.1, definition):
      G = 1/2 (1 + cos(k d.x + zeta)) exp{2 lam kappa^(1+tau) - 2 lam} kappa^tau,
      kappa = (d.z + 1) / 2,  tau = a (d.x)^2 / (1 - (d.z)^2)
  times a normaliser (below). The phase zeta is an extension used by the
  synthetic workloads; zeta = 0 is the paper's carrier.
* Normalisers:
    EXACT  = 1 / I with the closed-form integral of Section 5.1,
             I = pi (1 - e^{-2 lam}) / (lam sqrt(1+a)) * (1 + cos(zeta) Psi),
             Psi = 2 Lam e^{-Lam} sinhc(sqrt(Lam^2 - k^2)) / (1 - e^{-2 Lam}),
             Lam = lam (1 + a).  With zeta = 0 this is the printed formula;
             the phase only scales the carrier's odd part, whose envelope
             integral vanishes, so it multiplies Psi by cos(zeta).
    APPROX = C^{-1} = lam sqrt(1+a) / (2 pi (1 - e^{-2 lam})), the NASG
             normaliser that ignores the carrier (Section 5.1, last paragraph;
             Supplementary E/F definitions of C^{-1}).
* Gradients follow the product-rule decomposition of Supplementary F
  (p, E, C^{-1} and carrier contributions) with these readings:
    - d ln(E)/da uses ln(kappa) (Supp. E prints ln(tau) once; Supp. F has
      ln(kappa)).
    - dC^{-1}/dlam = sqrt(1+a) [(1 - e^{-2 lam}) - 2 lam e^{-2 lam}]
                     / (2 pi (1 - e^{-2 lam})^2): the printed "+" before
      2 lam is a sign error (finite differences confirm "-").
    - epsilon in "1 + epsilon - e^{-2 lam}" is taken as 0.
    - EXACT mode adds the derivatives of 1/I (derived here from the closed
      form; not printed in the paper) for lam, a, k and zeta.
    - dG/dd (for the mean gradient) is not printed: because dG/dx and dG/dz
      are both scalar multiples of d, dG/dx = s_x d and dG/dz = s_z d, and
      dG/dd = s_x x + s_z z.
* Special points (Section 5.1 lists G(z) = 1, G(-z) = 0 for the unnormalised
  kernel): at d = z the continuous limit N (1 + cos zeta) / 2 is used (kappa
  = 1 makes p = E = 1 whatever tau is); at d = -z, G = 0 and every gradient
  is 0. Where 1 - (d.z)^2 = 0 the tau terms are dropped.
"""
from __future__ import annotations

import numpy as np

NORM_EXACT = 0
NORM_APPROX = 1

PI = np.pi


# --------------------------------------------------------------------------- frame

def frame_from_quat(q):
    """Columns x, y, z of the rotation matrix of q / |q|, q = (w, x, y, z).

    The paper's lobe frame is R = [x y z] with y = z cross x (Supplementary C);
    the workloads parametrise it by a quaternion instead of three cosines.
    """
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    ww, xx, yy, zz = w * w, x * x, y * y, z * z
    n2 = (ww + xx + yy + zz)[..., None]
    # R(q/|q|) = M(q)/|q|^2 with M homogeneous of degree 2 in q (one rounding
    # of |q|^2 instead of one per normalised component)
    ax = np.stack([ww + xx - yy - zz, 2 * (x * y + w * z), 2 * (x * z - w * y)], -1) / n2
    ay = np.stack([2 * (x * y - w * z), ww - xx + yy - zz, 2 * (y * z + w * x)], -1) / n2
    az = np.stack([2 * (x * z + w * y), 2 * (y * z - w * x), ww - xx - yy + zz], -1) / n2
    return ax, ay, az


def axis_jacobians(qn):
    """d(x axis)/d q_hat and d(z axis)/d q_hat, each [..., 3, 4], at a unit
    quaternion q_hat (rows: axis components; columns: w, x, y, z)."""
    w, x, y, z = qn[..., 0], qn[..., 1], qn[..., 2], qn[..., 3]
    zero = np.zeros_like(w)
    jx = np.stack([
        np.stack([zero, zero, -4 * y, -4 * z], -1),
        np.stack([2 * z, 2 * y, 2 * x, 2 * w], -1),
        np.stack([-2 * y, 2 * z, -2 * w, 2 * x], -1),
    ], -2)
    jz = np.stack([
        np.stack([2 * y, 2 * z, 2 * w, 2 * x], -1),
        np.stack([-2 * x, -2 * w, 2 * z, 2 * y], -1),
        np.stack([zero, -4 * x, -4 * y, zero], -1),
    ], -2)
    return jx, jz


def frame_jacobians(q):
    """d(x axis)/dq and d(z axis)/dq, each [..., 3, 4], for the frame of q/|q|.

    Chain: axis(q_hat) with q_hat = q/|q|, d q_hat/dq = (I - q_hat q_hat^T)/|q|.
    """
    q = np.asarray(q, dtype=np.float64)
    nrm = np.linalg.norm(q, axis=-1, keepdims=True)
    qn = q / nrm
    jx, jz = axis_jacobians(qn)
    eye = np.broadcast_to(np.eye(4), q.shape[:-1] + (4, 4))
    proj = (eye - qn[..., :, None] * qn[..., None, :]) / nrm[..., None]
    return jx @ proj, jz @ proj


def quat_gradient(q, gx, gz, sx, sz):
    """dL/dq [..., 4] from dL/dx, dL/dz [..., 3] and its rounding scale, by the
    chain of ``frame_jacobians`` taken in two steps: v = (d axis/d q_hat)^T
    dL/daxis, then dL/dq = (v - q_hat (q_hat . v)) / |q|. The scale keeps the
    two terms of that projection as separate elementary contributions,
    (|v| + |q_hat| (|q_hat| . |v|)) / |q| with |v| from the absolute terms:
    a component of dL/dq can be the small difference of two large ones (a lobe
    that depends on z only, with q near a rotation about a coordinate axis)."""
    q = np.asarray(q, dtype=np.float64)
    nrm = np.linalg.norm(q, axis=-1, keepdims=True)
    qn = q / nrm
    ux, uz = axis_jacobians(qn)
    v = np.einsum("...ci,...c->...i", ux, gx) + np.einsum("...ci,...c->...i", uz, gz)
    va = (np.einsum("...ci,...c->...i", np.abs(ux), sx)
          + np.einsum("...ci,...c->...i", np.abs(uz), sz))
    g = (v - qn * (qn * v).sum(-1, keepdims=True)) / nrm
    sc = (va + np.abs(qn) * (np.abs(qn) * va).sum(-1, keepdims=True)) / nrm
    return g, sc


# --------------------------------------------------------------------- normalisers

def norm_approx(lam, a):
    """C^{-1} = lam sqrt(1+a) / (2 pi (1 - e^{-2 lam})) and its partials.

    Returns (C, dC/dlam, dC/da). Supplementary E/F; the dC/dlam numerator uses
    "-" (sign reading above).
    """
    lam = np.asarray(lam, np.float64)
    a = np.asarray(a, np.float64)
    one_m = -np.expm1(-2 * lam)                 # 1 - e^{-2 lam}
    sq = np.sqrt(1 + a)
    c = lam * sq / (2 * PI * one_m)
    dc_dlam = sq * (one_m - 2 * lam * np.exp(-2 * lam)) / (2 * PI * one_m ** 2)
    dc_da = lam / (2 * sq) / (2 * PI * one_m)
    return c, dc_dlam, dc_da


def _sinhc_series(r, nterms=30):
    """S(r) = sum r^n/(2n+1)! and S'(r) = sum n r^(n-1)/(2n+1)!  (|r| small)."""
    s = np.zeros_like(r)
    ds = np.zeros_like(r)
    fact = 1.0  # (2n+1)!
    rn = np.ones_like(r)      # r^n
    rnm1 = np.zeros_like(r)   # r^(n-1)
    for n in range(nterms):
        if n > 0:
            fact *= (2 * n) * (2 * n + 1)
            rnm1 = rn
            rn = rn * r
        s = s + rn / fact
        if n > 0:
            ds = ds + n * rnm1 / fact
    return s, ds


def exp_sinhc(lam_big, k):
    """F = e^{-Lam} sinhc(sqrt(Lam^2 - k^2)) and e^{-Lam} S'(r), r = Lam^2 - k^2.

    sinhc(u) = sinh(u)/u, which for r < 0 is sin(t)/t with t = sqrt(-r).
    Evaluated without overflow: e^{-Lam} sinh(s) = (e^{s-Lam} - e^{-s-Lam})/2
    with s - Lam = -k^2 / (Lam + s); the power series near r = 0.
    """
    L = np.asarray(lam_big, np.float64)
    k = np.asarray(k, np.float64)
    L, k = np.broadcast_arrays(L, k)
    r = L * L - k * k
    F = np.empty_like(r)
    dF = np.empty_like(r)           # e^{-Lam} S'(r)
    small = np.abs(r) <= 1.0
    pos = (r > 1.0)
    neg = (r < -1.0)
    if np.any(small):
        s_, ds_ = _sinhc_series(r[small])
        e = np.exp(-L[small])
        F[small] = e * s_
        dF[small] = e * ds_
    if np.any(pos):
        s = np.sqrt(r[pos])
        lp, kp = L[pos], k[pos]
        ep = np.exp(-kp * kp / (lp + s))     # e^{s - Lam}
        em = np.exp(-s - lp)                 # e^{-s - Lam}
        sinh_ = 0.5 * (ep - em)
        cosh_ = 0.5 * (ep + em)
        F[pos] = sinh_ / s
        dF[pos] = (s * cosh_ - sinh_) / (2 * s ** 3)
    if np.any(neg):
        t = np.sqrt(-r[neg])
        e = np.exp(-L[neg])
        F[neg] = e * np.sin(t) / t
        dF[neg] = e * (np.sin(t) - t * np.cos(t)) / (2 * t ** 3)
    return F, dF


def psi(lam_big, k):
    """Psi(Lam, k) of Section 5.1 with its partials and 1 - Psi:
    (Psi, dPsi/dLam, dPsi/dk, 1 - Psi).

    Where Lam^2 - k^2 > 1, s = sqrt(Lam^2 - k^2) and delta = Lam - s =
    k^2 / (Lam + s), and Psi = (Lam/s) e^{-delta} (1 - e^{-2s}) / (1 - e^{-2Lam})
    is the same expression regrouped; its log-derivatives
        d ln Psi/dLam = (1/Lam - Lam/s^2) + delta/s
                        + 2 [(Lam/s) g(s) - g(Lam)],   g(x) = 1/(e^{2x} - 1),
        d ln Psi/dk   = (k/s) (1/s - 1 - 2 g(s)),
    are written with 1/Lam - Lam/s^2 = -k^2/(Lam s^2), Lam/s - 1 = delta/s and
    g(s) - g(Lam) = expm1(2 delta) e^{-2Lam} / ((1 - e^{-2s})(1 - e^{-2Lam})),
    so that every term vanishes with k instead of cancelling (Psi = 1 at
    k = 0), and ln Psi = -log1p(-delta/Lam) - delta
    + log1p(e^{-2s} expm1(-2 delta) / (1 - e^{-2Lam})) gives 1 - Psi with
    relative accuracy. Elsewhere the partials come from differentiating
    e^{-Lam} sinhc directly."""
    L, k = np.broadcast_arrays(np.asarray(lam_big, np.float64), np.asarray(k, np.float64))
    shp = L.shape
    L, k = L.reshape(-1), k.reshape(-1)
    F, dFs = exp_sinhc(L, k)
    D = -np.expm1(-2 * L)                    # 1 - e^{-2 Lam}
    dF_dL = -F + dFs * 2 * L
    dF_dk = dFs * (-2 * k)
    P = 2 * L * F / D
    dP_dL = 2 * F / D + 2 * L * dF_dL / D - 2 * L * F * (2 * np.exp(-2 * L)) / D ** 2
    dP_dk = 2 * L * dF_dk / D
    omP = 1 - P
    hyp = L * L - k * k > 1.0
    if np.any(hyp):
        Lh, kh, Dh = L[hyp], k[hyp], D[hyp]
        s = np.sqrt(Lh * Lh - kh * kh)
        delta = kh * kh / (Lh + s)
        Ds = -np.expm1(-2 * s)               # 1 - e^{-2s}
        gs = np.exp(-2 * s) / Ds
        dlnL = (-kh * kh / (Lh * s * s) + delta / s * (1 + 2 * gs)
                + 2 * np.expm1(2 * delta) * np.exp(-2 * Lh) / (Ds * Dh))
        dlnk = kh / s * (1 / s - 1 - 2 * gs)
        lnP = (-np.log1p(-delta / Lh) - delta
               + np.log1p(np.exp(-2 * s) * np.expm1(-2 * delta) / Dh))
        Ph = P[hyp]
        dP_dL[hyp] = Ph * dlnL
        dP_dk[hyp] = Ph * dlnk
        omP[hyp] = -np.expm1(lnP)
    return P.reshape(shp), dP_dL.reshape(shp), dP_dk.reshape(shp), omP.reshape(shp)


def integral_exact(lam, a, k, zeta):
    """Closed-form integral I of the unnormalised NASGabor (Section 5.1),
    with the phase reading (Psi multiplied by cos zeta)."""
    lam = np.asarray(lam, np.float64)
    a = np.asarray(a, np.float64)
    P = psi(lam * (1 + a), k)[0]
    return PI * (-np.expm1(-2 * lam)) / (lam * np.sqrt(1 + a)) * (1 + np.cos(zeta) * P)


def norm_exact(lam, a, k, zeta):
    """N = 1/I and its partials (N, dN/dlam, dN/da, dN/dk, dN/dzeta)."""
    lam = np.asarray(lam, np.float64)
    a = np.asarray(a, np.float64)
    k = np.asarray(k, np.float64)
    zeta = np.asarray(zeta, np.float64)
    Lam = lam * (1 + a)
    P, dP_dL, dP_dk, omP = psi(Lam, k)
    Dl = -np.expm1(-2 * lam)
    sq = np.sqrt(1 + a)
    A = PI * Dl / (lam * sq)
    dA_dlam = PI / sq * (2 * np.exp(-2 * lam) * lam - Dl) / lam ** 2
    dA_da = -A / (2 * (1 + a))
    cz, sz = np.cos(zeta), np.sin(zeta)
    # B = 1 + cos(zeta) Psi; where cos(zeta) < 0 it is formed as
    # 2 cos^2(zeta/2) + |cos zeta| (1 - Psi), two terms of one sign (B -> 0
    # as zeta -> pi with k -> 0, where 1 + cos(zeta) Psi would cancel)
    B = np.where(cz < 0, 2 * np.cos(zeta / 2) ** 2 - cz * omP, 1 + cz * P)
    dB_dlam = cz * dP_dL * (1 + a)
    dB_da = cz * dP_dL * lam
    dB_dk = cz * dP_dk
    dB_dz = -sz * P
    I = A * B
    N = 1 / I
    dN = lambda dI: -dI / (I * I)  # noqa: E731
    return (N, dN(dA_dlam * B + A * dB_dlam), dN(dA_da * B + A * dB_da),
            dN(A * dB_dk), dN(A * dB_dz))


def normaliser(shape, norm):
    """Normaliser and its partials for shape[..., 4] = (lam, a, k, zeta).

    Returns (N, dN/dlam, dN/da, dN/dk, dN/dzeta); the APPROX normaliser does
    not depend on k or zeta.
    """
    s = np.asarray(shape, np.float64)
    lam, a, k, zeta = s[..., 0], s[..., 1], s[..., 2], s[..., 3]
    if norm == NORM_EXACT:
        return norm_exact(lam, a, k, zeta)
    if norm == NORM_APPROX:
        c, dl, da = norm_approx(lam, a)
        z = np.zeros_like(c)
        return c, dl, da, z, z
    raise ValueError("unknown normaliser")


# --------------------------------------------------------------------- directions

def view_directions(means=None, cams=None, dirs=None):
    """Unit view directions [V][N][3] and the distances |mu - o| [V][N].

    Central-ray convention (Section 5.2): one direction per primitive and
    frame, d = (mu - o)/|mu - o| from camera centre o to the primitive mean,
    the direction of the ray r(t) = o + t d (Section 3.1). With raw per-
    primitive directions, d = dirs/|dirs| and V = 1.
    """
    if dirs is not None:
        e = np.asarray(dirs, np.float64)[None]
    else:
        e = np.asarray(means, np.float64)[None, :, :] - np.asarray(cams, np.float64)[:, None, :]
    r = np.linalg.norm(e, axis=-1)
    return e / r[..., None], r


# ------------------------------------------------------------------------- lobes

def lobe_terms(d, ax, az, shape, Cn):
    """Per (lobe, view, primitive) quantities of the definition.

    d [V][N][3]; ax, az [K][N][3]; shape [K][N][4]; Cn [K][N].
    Returns a dict of [K][V][N] arrays (vectors get a trailing 3).
    """
    s = np.asarray(shape, np.float64)
    lam = s[..., 0][:, None, :]
    a = s[..., 1][:, None, :]
    k = s[..., 2][:, None, :]
    zeta = s[..., 3][:, None, :]
    Cn = Cn[:, None, :]
    dx = np.einsum("vnc,knc->kvn", d, ax)
    dz = np.einsum("vnc,knc->kvn", d, az)
    # 1 - d.z and 1 + d.z as half squared chords |d -+ z|^2 / 2 (the same
    # numbers for unit vectors). Each stays relatively accurate where it is
    # small, next to the lobe axis and next to its antipode, where 1 -+ d.z
    # would subtract two nearly equal numbers; kappa = (1 + d.z)/2,
    # 1 - (d.z)^2 = (1 - d.z)(1 + d.z) and ln kappa are all formed from them.
    hp = 0.5 * ((d[None] - az[:, None]) ** 2).sum(-1)
    hm = 0.5 * ((d[None] + az[:, None]) ** 2).sum(-1)
    with np.errstate(all="ignore"):
        kappa = hm / 2
        den = hp * hm                               # 1 - (d.z)^2
        at_pole = den == 0                          # d = +z or d = -z
        anti = hm == 0                              # d = -z
        tau = np.where(at_pole, 0.0, a * dx * dx / den)
        # ln kappa = ln(1 - hp/2): log1p where kappa is near 1
        lnk = np.where(anti, 0.0, np.where(hp < 1.0, np.log1p(-hp / 2),
                                           np.log(np.where(anti, 1.0, kappa))))
        E = np.where(anti, 0.0, np.exp(tau * lnk))  # kappa^tau
        # E kappa - 1 = e^{(1 + tau) ln kappa} - 1
        em1 = np.where(anti, -1.0, np.expm1((1 + tau) * lnk))
        p = np.exp(2 * lam * em1)
        arg = k * dx + zeta
        # (1 + cos t)/2 = cos^2(t/2) and (sin t)/2 = sin(t/2) cos(t/2): the
        # half-angle forms stay relatively accurate at the carrier's zeros,
        # where 1 + cos t would cancel
        c_half, s_half = np.cos(arg / 2), np.sin(arg / 2)
        carrier = c_half * c_half
        half_sin = s_half * c_half                   # (sin arg) / 2
        G = np.where(anti, 0.0, p * E * Cn * carrier)
    return dict(dx=dx, dz=dz, kappa=kappa, den=den, tau=tau, lnk=lnk, E=E, p=p, em1=em1,
                arg=arg, carrier=carrier, half_sin=half_sin, G=G, lam=lam, a=a, k=k, zeta=zeta, Cn=Cn,
                at_pole=at_pole, anti=anti)


def forward(quat, shape, rgbw, c0, norm, means=None, cams=None, dirs=None):
    """rgb [V][N][3] and its rounding scale |c0| + sum_l |w_l G_l|."""
    ax, _, az = frame_from_quat(quat)
    d, _ = view_directions(means, cams, dirs)
    Cn = normaliser(shape, norm)[0]
    t = lobe_terms(d, ax, az, shape, Cn)
    w = np.transpose(np.asarray(rgbw, np.float64), (0, 2, 1))   # [K][N][3]
    contrib = t["G"][..., None] * w[:, None, :, :]               # [K][V][N][3]
    c0 = np.asarray(c0, np.float64)
    rgb = c0[None] + contrib.sum(axis=0)
    scale = np.abs(c0)[None] + np.abs(contrib).sum(axis=0)
    return rgb, scale, t


def forward_backward(quat, shape, rgbw, c0, grad_rgb, norm, means=None, cams=None,
                     dirs=None):
    """Forward colours plus gradients of L = sum(grad_rgb * rgb) w.r.t. every
    stored input, each with its rounding scale (sum of absolute elementary
    contributions). Returns (out, scale), dicts keyed by tensor name:
    rgb, quat, shape, rgbw, c0 and means (or dirs)."""
    quat = np.asarray(quat, np.float64)
    ax, _, az = frame_from_quat(quat)
    out, scale, axes = frame_forward_backward(ax, az, shape, rgbw, c0, grad_rgb, norm,
                                              means, cams, dirs)
    gx_vec, gz_vec, sx_vec, sz_vec = axes
    out["quat"], scale["quat"] = quat_gradient(quat, gx_vec, gz_vec, sx_vec, sz_vec)
    return out, scale


def frame_forward_backward(ax, az, shape, rgbw, c0, grad_rgb, norm, means=None, cams=None,
                           dirs=None):
    """The evaluation for given lobe axes ax, az [K][N][3] (float64) and
    lobe values shape = (lam, a, k, zeta), weights rgbw: colours and the
    gradients w.r.t. shape, rgbw, c0 and the means (or dirs), each with its
    rounding scale, plus the gradients w.r.t. the axes themselves,
    (dL/dx, dL/dz, their scales), for the caller's frame parametrisation."""
    d, r = view_directions(means, cams, dirs)
    Cn, dC_dlam, dC_da, dC_dk, dC_dz = normaliser(shape, norm)
    t = lobe_terms(d, ax, az, shape, Cn)
    w = np.transpose(np.asarray(rgbw, np.float64), (0, 2, 1))   # [K][N][3]
    g = np.asarray(grad_rgb, np.float64)                       # [V][N][3]
    c0 = np.asarray(c0, np.float64)
    G = t["G"]
    contrib = G[..., None] * w[:, None, :, :]
    out = {"rgb": c0[None] + contrib.sum(0)}
    scale = {"rgb": np.abs(c0)[None] + np.abs(contrib).sum(0)}

    # dL/dG per (lobe, view, primitive) and its absolute scale
    gw = g[None] * w[:, None, :, :]                            # [K][V][N][3]
    gG = gw.sum(-1)
    gGa = np.abs(gw).sum(-1)

    live = ~t["anti"]
    pole = t["at_pole"]
    lam, a, k, zeta = t["lam"], t["a"], t["k"], t["zeta"]
    p, E, kappa, lnk, tau = t["p"], t["E"], t["kappa"], t["lnk"], t["tau"]
    dx, dz, den, carrier, arg = t["dx"], t["dz"], t["den"], t["carrier"], t["arg"]
    Cnb = t["Cn"]
    half_sin = t["half_sin"]                         # (sin arg) / 2
    dlam_b = dC_dlam[:, None, :]
    da_b = dC_da[:, None, :]
    dk_b = dC_dk[:, None, :]
    dz_b = dC_dz[:, None, :]

    with np.errstate(all="ignore"):
        safe_den = np.where(pole, 1.0, den)
        # --- a (Supplementary F, derivative with respect to a)
        dtau_da = np.where(pole, 0.0, dx * dx / safe_den)
        dp_da = p * (2 * lam * E * kappa) * lnk * dtau_da
        dE_da = E * lnk * dtau_da
        ga_terms = [dp_da * E * Cnb * carrier, p * dE_da * Cnb * carrier,
                    p * E * da_b * carrier]
        # --- lambda (sign-corrected dC/dlam for APPROX; dN/dlam for EXACT)
        dp_dlam = 2 * p * t["em1"]
        gl_terms = [E * Cnb * dp_dlam * carrier, E * p * dlam_b * carrier]
        # --- k and zeta (carrier, plus the EXACT normaliser's dependence)
        dcar_dk = -dx * half_sin
        dcar_dz = -half_sin
        gk_terms = [p * E * Cnb * dcar_dk, p * E * dk_b * carrier]
        gz_terms = [p * E * Cnb * dcar_dz, p * E * dz_b * carrier]
        # --- x: every term is a multiple of d; collect the scalar factors
        dtau_dx_s = np.where(pole, 0.0, 2 * a * dx / safe_den)
        dE_dx_s = E * lnk * dtau_dx_s
        dp_dx_s = 2 * lam * p * kappa * dE_dx_s
        gx_terms = [dp_dx_s * E * Cnb * carrier, p * dE_dx_s * Cnb * carrier,
                    p * E * Cnb * (-k * half_sin)]
        # --- z
        dkap_dz_s = 0.5
        dtau_dz_s = np.where(pole, 0.0, a * dx * dx * 2 * dz / safe_den ** 2)
        tau_over_kappa = np.where(pole, 0.0, tau / np.where(live, kappa, 1.0))
        dE_dz_s = E * (tau_over_kappa * dkap_dz_s + lnk * dtau_dz_s)
        dp_dz_s = p * 2 * lam * (kappa * dE_dz_s + E * dkap_dz_s)
        gzv_terms = [dp_dz_s * E * Cnb * carrier, p * dE_dz_s * Cnb * carrier]

    def red(terms):
        """Sum over views of dL/dG * dG/dparam and the matching abs scale."""
        tot = sum(terms)
        ab = sum(np.abs(x) for x in terms)
        tot = np.where(live, tot, 0.0)
        ab = np.where(live, ab, 0.0)
        return (gG * tot).sum(1), (gGa * ab).sum(1), tot, ab

    g_a, s_a, _, _ = red(ga_terms)
    g_l, s_l, _, _ = red(gl_terms)
    g_k, s_k, _, _ = red(gk_terms)
    g_z, s_z, _, _ = red(gz_terms)
    _, _, sx, sxa = red(gx_terms)          # scalar s_x with dG/dx = s_x d
    _, _, szv, szva = red(gzv_terms)       # scalar s_z with dG/dz = s_z d

    # vector gradients w.r.t. the frame axes: sum_v gG s d
    gx_vec = np.einsum("kvn,vnc->knc", gG * sx, d)
    gz_vec = np.einsum("kvn,vnc->knc", gG * szv, d)
    sx_vec = np.einsum("kvn,vnc->knc", gGa * sxa, np.abs(d))
    sz_vec = np.einsum("kvn,vnc->knc", gGa * szva, np.abs(d))

    out["shape"] = np.stack([g_l, g_a, g_k, g_z], -1)
    scale["shape"] = np.stack([s_l, s_a, s_k, s_z], -1)

    gwts = np.einsum("vnc,kvn->kcn", g, G)
    out["rgbw"] = gwts
    scale["rgbw"] = np.einsum("vnc,kvn->kcn", np.abs(g), np.abs(G))
    out["c0"] = g.sum(0)
    scale["c0"] = np.abs(g).sum(0)

    # view-direction gradient dL/dd = sum_l gG (s_x x + s_z z), then through
    # d = e/|e|: dL/de = (I - d d^T) dL/dd / |e|
    gd = (np.einsum("kvn,knc->vnc", gG * sx, ax) + np.einsum("kvn,knc->vnc", gG * szv, az))
    sd = (np.einsum("kvn,knc->vnc", gGa * sxa, np.abs(ax))
          + np.einsum("kvn,knc->vnc", gGa * szva, np.abs(az)))
    proj = np.eye(3)[None, None] - d[..., :, None] * d[..., None, :]
    ge = np.einsum("vnij,vnj->vni", proj, gd) / r[..., None]
    # the projection's two terms (identity and d d^T) count as separate
    # elementary contributions: (|g| + |d| (|d| . |g|)) / |e|
    se = (sd + np.abs(d) * (np.abs(d) * sd).sum(-1, keepdims=True)) / r[..., None]
    key = "dirs" if dirs is not None else "means"
    out[key] = ge.sum(0)
    scale[key] = se.sum(0)
    return out, scale, (gx_vec, gz_vec, sx_vec, sz_vec)


def lobe_value(d, q, shape, norm):
    """G for one lobe at unit directions d [..., 3] (used by the pin tests).

    q [4], shape [4]. Uses the same definition as ``lobe_terms``."""
    d = np.asarray(d, np.float64).reshape(-1, 3)
    ax, _, az = frame_from_quat(np.asarray(q, np.float64)[None, None])
    s = np.asarray(shape, np.float64)[None, None]
    Cn = normaliser(s, norm)[0]
    # the M directions of one primitive are treated as M views
    dv = d[:, None, :]
    t = lobe_terms(dv, ax, az, s, Cn)
    return t["G"][0, :, 0]
