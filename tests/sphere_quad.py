"""Quadrature rules on the unit sphere, used to pin the oracle's normalisers.

Not product code: plain numerical integration that shares nothing with the
oracle beyond calling its lobe function as the integrand.
"""
import numpy as np


def lobe_frame_grid(n_phi=1024, nodes=32, panels=None):
    """Directions and weights for integrating a lobe centred on +z.

    u = cos(theta) = 1 - 2 s^2 (s in [0, 1], du = 4 s ds) concentrates nodes at
    the peak; s uses composite Gauss-Legendre on geometric panels, phi uses the
    periodic trapezoid rule. Returns d[M][3] and weights[M] with sum = 4 pi.
    """
    if panels is None:
        # geometric towards the peak (s = 0) and towards the antipode (s = 1),
        # where kappa^tau has an algebraic endpoint singularity
        lo_half = np.geomspace(1e-6, 0.5, 50)
        panels = np.concatenate([[0.0], lo_half, (1.0 - lo_half)[::-1][1:], [1.0]])
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    s_all, ws_all = [], []
    for lo, hi in zip(panels[:-1], panels[1:]):
        s_all.append(0.5 * (hi - lo) * xg + 0.5 * (hi + lo))
        ws_all.append(0.5 * (hi - lo) * wg)
    s = np.concatenate(s_all)
    ws = np.concatenate(ws_all) * 4.0 * s          # du = 4 s ds
    u = 1.0 - 2.0 * s * s
    phi = (np.arange(n_phi) + 0.5) * (2 * np.pi / n_phi)
    wphi = np.full(n_phi, 2 * np.pi / n_phi)
    sin_t = np.sqrt(np.clip(1.0 - u * u, 0.0, None))
    d = np.stack([np.outer(sin_t, np.cos(phi)), np.outer(sin_t, np.sin(phi)),
                  np.outer(u, np.ones_like(phi))], -1).reshape(-1, 3)
    w = np.outer(ws, wphi).ravel()
    return d, w


def fibonacci_sphere(m):
    """m quasi-uniform points with equal weights 4 pi / m."""
    i = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / m
    golden = np.pi * (3.0 - np.sqrt(5.0))
    phi = i * golden
    r = np.sqrt(1.0 - z * z)
    d = np.stack([r * np.cos(phi), r * np.sin(phi), z], -1)
    return d, np.full(m, 4.0 * np.pi / m)


def gauss_product_grid(n_u=32, n_phi=64):
    """Plain Gauss-Legendre in cos(theta) x trapezoid in phi (exact for low-degree
    polynomials on the sphere)."""
    xg, wg = np.polynomial.legendre.leggauss(n_u)
    phi = (np.arange(n_phi) + 0.5) * (2 * np.pi / n_phi)
    st = np.sqrt(1 - xg * xg)
    d = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(xg, np.ones_like(phi))], -1).reshape(-1, 3)
    w = np.outer(wg, np.full(n_phi, 2 * np.pi / n_phi)).ravel()
    return d, w
