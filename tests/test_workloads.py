"""Seeded workload generators: layouts, determinism, bf16 rounding."""
import numpy as np
import torch

import workloads as W


def test_config0_layout_and_determinism():
    a = W.config0()
    b = W.config0()
    assert a.quat.shape == (4, 4096, 4) and a.shape.shape == (4, 4096, 4)
    assert a.rgbw.shape == (4, 3, 4096) and a.c0.shape == (4096, 3)
    assert a.dirs.shape == (4096, 3) and a.means is None and a.v == 1
    assert a.sh.shape == (16, 3, 4096)
    for f in ("quat", "shape", "rgbw", "c0", "dirs", "grad_rgb", "sh"):
        assert getattr(a, f).dtype == np.float32
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    lam, aa, k, z = (a.shape[..., i] for i in range(4))
    assert lam.min() >= 1 and lam.max() <= 1e3 and aa.min() >= 1 and aa.max() <= 1e3
    assert k.min() >= 0 and k.max() <= 16 and z.min() >= 0 and z.max() <= 2 * np.pi


def test_camera_geometry():
    w = W.draw_workload(9, 1000, 2, 5)
    np.testing.assert_allclose(np.linalg.norm(w.cams, axis=1), 10, rtol=1e-6)
    assert np.abs(w.means).max() <= 5
    assert w.grad_rgb.shape == (5, 1000, 3)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(100000).astype(np.float32) * 100
    bits = W.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(bits, ref)
    back = W.bf16_bits_to_f32(bits)
    np.testing.assert_array_equal(back, torch.from_numpy(x).to(torch.bfloat16).float().numpy())


def test_take_primitives():
    w = W.draw_workload(3, 50, 3, 2, dtype="bf16")
    idx = np.array([4, 0, 49])
    s = W.take_primitives(w, idx)
    np.testing.assert_array_equal(s.quat, w.quat[:, idx])
    np.testing.assert_array_equal(s.rgbw_bits, w.rgbw_bits[:, :, idx])
    np.testing.assert_array_equal(s.grad_rgb, w.grad_rgb[:, idx])


def test_config4_scene_table():
    sc = W.config4(scale=0.001)
    assert len(sc) == 32
    assert {s.workload.k for s in sc} <= {4, 8, 16}
    assert {s.workload.v for s in sc} <= {1, 4, 16}
