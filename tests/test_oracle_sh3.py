"""Pins of the FP64 degree-3 SH oracle (Section 3.2 expansion).

The basis is pinned to scipy's complex harmonics (sph_harm_y, with the
Condon-Shortley phase) through the real combination stated in the oracle,
to closed-form values on the +z axis (tests/golden/sh_axis_values.txt), to the
addition theorem, parity and orthonormality by quadrature; the gradients to
central finite differences.
"""
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import sh3_ref as S
from sphere_quad import gauss_product_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sh_axis_values.txt")


def _unit(n, seed):
    d = np.random.default_rng(seed).standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_basis_matches_scipy_real_combination():
    d = _unit(500, 0)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = S.basis(d)
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = np.sqrt(2) * c.real
            elif m < 0:
                ref = np.sqrt(2) * c.imag
            else:
                ref = c.real
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13)


def test_axis_values_golden():
    vals = np.loadtxt(GOLDEN)
    Y = S.basis(np.array([[0, 0, 1.0]]))[0]
    for l in range(4):
        assert Y[l * l + l] == pytest.approx(vals[l], rel=1e-15)
        for m in range(-l, l + 1):
            if m != 0:
                assert Y[l * l + l + m] == 0.0


def test_addition_theorem_and_parity():
    d = _unit(300, 1)
    Y = S.basis(d)
    Ym = S.basis(-d)
    for l in range(4):
        blk = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose((Y[:, blk] ** 2).sum(1), (2 * l + 1) / (4 * np.pi), rtol=1e-13)
        np.testing.assert_allclose(Ym[:, blk], (-1) ** l * Y[:, blk], atol=1e-14)


def test_orthonormal_by_quadrature():
    d, w = gauss_product_grid(16, 32)
    Y = S.basis(d)
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-13)


@pytest.mark.parametrize("dirs_mode", [True, False])
def test_gradients_against_finite_differences(dirs_mode):
    rng = np.random.default_rng(3)
    n, v = 4, 1 if dirs_mode else 3
    sh = 0.3 * rng.standard_normal((16, 3, n))
    g = rng.standard_normal((v, n, 3))
    if dirs_mode:
        geo = {"dirs": rng.standard_normal((n, 3)) * 2}
        key = "dirs"
    else:
        geo = {"means": rng.uniform(-5, 5, (n, 3)), "cams": 10 * _unit(v, 4)}
        key = "means"
    out, scale = S.forward_backward(sh, g, **geo)

    def loss(sh_, geo_):
        return float((S.forward(sh_, **geo_)[0] * g).sum())

    def fd(f, x, rel=1e-5):
        o = np.zeros_like(x)
        it = np.nditer(x, flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            h = rel * max(1.0, abs(x[i]))

            def c(hh):
                xp, xm = x.copy(), x.copy()
                xp[i] += hh
                xm[i] -= hh
                return (f(xp) - f(xm)) / (2 * hh)
            o[i] = (4 * c(h / 2) - c(h)) / 3
        return o

    num = fd(lambda x: loss(x, geo), sh)
    assert (np.abs(num - out["sh"]) / (scale["sh"] + 1e-12)).max() < 1e-7

    def fg(x):
        gg = dict(geo)
        gg[key] = x
        return loss(sh, gg)
    num = fd(fg, geo[key])
    assert (np.abs(num - out[key]) / (scale[key] + 1e-12)).max() < 1e-7
    np.testing.assert_allclose(out["rgb"], S.forward(sh, **geo)[0], rtol=0, atol=0)
