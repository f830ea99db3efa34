"""The NASGabor lobe of Section 5.1 evaluated with mpmath at 50 digits, for
one lobe and one raw view direction (test helper).

The value is the definition taken literally (kappa = (1 + d.z)/2,
tau = a (d.x)^2 / (1 - (d.z)^2), E = kappa^tau, p = e^{2 lam (kappa E - 1)},
carrier (1 + cos(k d.x + zeta))/2) times the normaliser (1 / closed-form
integral, or the NASG normaliser); at 50 digits no rounding of the FP64
oracle's size survives, so comparing the oracle with it measures the
oracle's own rounding in the edge regions. Its gradients are mpmath's
numerical derivatives of the same function with respect to every raw input
(quaternion, lam, a, k, zeta, the unnormalised direction): independent of
the oracle's analytic formulas.
"""
from __future__ import annotations

import mpmath as mp

DPS = 50


def _normaliser(lam, a, k, zeta, norm):
    one_m = -mp.expm1(-2 * lam)
    if norm == 1:
        return lam * mp.sqrt(1 + a) / (2 * mp.pi * one_m)
    big = lam * (1 + a)
    r = big * big - k * k
    if r > 0:
        s = mp.sqrt(r)
        sinhc = mp.sinh(s) / s
    elif r < 0:
        s = mp.sqrt(-r)
        sinhc = mp.sin(s) / s
    else:
        sinhc = mp.mpf(1)
    psi = 2 * big * mp.exp(-big) * sinhc / (-mp.expm1(-2 * big))
    integral = mp.pi * one_m / (lam * mp.sqrt(1 + a)) * (1 + mp.cos(zeta) * psi)
    return 1 / integral


def lobe(x, norm):
    """G for x = (qw, qx, qy, qz, lam, a, k, zeta, d0, d1, d2) (mpf values)."""
    qw, qx, qy, qz, lam, a, k, zeta, d0, d1, d2 = x
    n2 = qw * qw + qx * qx + qy * qy + qz * qz
    X = ((qw * qw + qx * qx - qy * qy - qz * qz) / n2, 2 * (qx * qy + qw * qz) / n2,
         2 * (qx * qz - qw * qy) / n2)
    Z = (2 * (qx * qz + qw * qy) / n2, 2 * (qy * qz - qw * qx) / n2,
         (qw * qw - qx * qx - qy * qy + qz * qz) / n2)
    nd = mp.sqrt(d0 * d0 + d1 * d1 + d2 * d2)
    d = (d0 / nd, d1 / nd, d2 / nd)
    dx = d[0] * X[0] + d[1] * X[1] + d[2] * X[2]
    dz = d[0] * Z[0] + d[1] * Z[1] + d[2] * Z[2]
    kappa = (1 + dz) / 2
    if kappa <= 0:
        return mp.mpf(0)
    den = 1 - dz * dz
    tau = a * dx * dx / den if den != 0 else mp.mpf(0)
    E = mp.power(kappa, tau)
    p = mp.exp(2 * lam * (kappa * E - 1))
    carrier = (1 + mp.cos(k * dx + zeta)) / 2
    return _normaliser(lam, a, k, zeta, norm) * p * E * carrier


def inputs(q, shape, d):
    return [mp.mpf(float(v)) for v in list(q) + list(shape) + list(d)]


def value(q, shape, d, norm):
    with mp.workdps(DPS):
        return float(lobe(inputs(q, shape, d), norm))


def gradient(q, shape, d, norm):
    """dG/d(qw, qx, qy, qz, lam, a, k, zeta, d0, d1, d2) as floats."""
    with mp.workdps(DPS):
        x0 = inputs(q, shape, d)
        out = []
        for i in range(len(x0)):
            def f(t, i=i):
                x = list(x0)
                x[i] = t
                return lobe(x, norm)
            out.append(float(mp.diff(f, x0[i])))
        return out
