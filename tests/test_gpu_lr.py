"""GPU parity of the camera-spacing statistic (Section 4, implementation
details) that scales the appearance learning rates: ``nasg_camera_knn``
through the C ABI and through ``lr.camera_knn`` against the FP64 oracle.

* closed forms: cube corners, an even ring, a line (whose end cameras see one
  neighbour at twice the spacing), coincident centres (distance 0);
* seeded rigs in the layouts of the paper's captures (shell, walk-around,
  forward-facing grid), camera counts around one 256-camera tile (one, one
  exactly full, one plus a ragged tail, several), k from 1 to 32;
* the largest accepted rig (65536 cameras, k = 32) on sampled cameras and the
  mean against the exactly rounded average of the kernel's per-camera values;
* identical bits on repeated calls.

Bar: relative error <= 1e-14 per camera and for the mean. A distance here is
the square root of an FMA chain (a few ulp against the oracle's math.dist),
averaged over k values; the mean is a fixed tree sum over at most 65536
values (relative error below log2(65536) ulp).
"""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from oracle import lr_ref as Q
from paper_2606_09794_amd import _lib as L
from paper_2606_09794_amd import lr
from workloads.gen import CAMERA_LAYOUTS, draw_camera_centres

pytestmark = pytest.mark.gpu
TOL = 1e-14


def abi_knn(centres, k):
    """Call the C ABI directly: (per-camera values, mean) as numpy."""
    c = torch.as_tensor(np.ascontiguousarray(centres, dtype=np.float64), device="cuda")
    n = int(c.shape[0])
    per = torch.empty(n, dtype=torch.float64, device="cuda")
    mean = torch.empty(1, dtype=torch.float64, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(L.lib().nasg_camera_knn(C.c_void_p(c.data_ptr()), n, k, C.c_void_p(per.data_ptr()),
                                    C.c_void_p(mean.data_ptr()), st), "nasg_camera_knn")
    torch.cuda.synchronize()
    return per.cpu().numpy(), float(mean.item())


def check(per, mean, ref_per, what):
    ref_per = np.asarray(ref_per)
    rel = np.abs(per - ref_per) / np.maximum(np.abs(ref_per), 1e-300)
    print(f"{what}: max rel {rel.max():.2e}", flush=True)
    assert rel.max() <= TOL, what
    ref_mean = math.fsum(ref_per) / len(ref_per)
    assert abs(mean - ref_mean) <= TOL * abs(ref_mean), what


def test_closed_forms():
    s = 2.5
    cube = np.array([[x, y, z] for x in (0, s) for y in (0, s) for z in (0, s)], float)
    per, mean = abi_knn(cube, 3)
    assert np.allclose(per, s, rtol=TOL, atol=0) and abs(mean - s) <= TOL * s

    n, r = 12, 4.0
    a = 2 * np.pi * np.arange(n) / n
    ring = np.stack([r * np.cos(a), r * np.sin(a), np.zeros(n)], -1)
    ref = (2 * 2 * r * math.sin(math.pi / n) + 2 * r * math.sin(2 * math.pi / n)) / 3
    per, mean = abi_knn(ring, 3)
    assert np.allclose(per, ref, rtol=TOL, atol=0) and abs(mean - ref) <= TOL * ref

    n, h = 9, 0.75
    line = np.stack([h * np.arange(n), np.zeros(n), np.zeros(n)], -1)
    per, _ = abi_knn(line, 2)
    assert per[0] == per[-1] == 1.5 * h and np.all(per[1:-1] == h)

    per, mean = abi_knn([[0, 0, 0], [0, 0, 0], [3, 4, 0]], 2)
    assert per.tolist() == [2.5, 2.5, 5.0] and mean == pytest.approx(10 / 3, rel=TOL)


@pytest.mark.parametrize("layout", CAMERA_LAYOUTS)
@pytest.mark.parametrize("n,ks", [(4, (1, 3)), (57, (1, 3, 5, 8)), (256, (3, 16)),
                                  (300, (3, 32)), (700, (2, 17))])
def test_rigs_against_oracle(layout, n, ks):
    c = draw_camera_centres(7 + n, n, layout)
    for k in ks:
        per, mean = abi_knn(c, k)
        check(per, mean, Q.knn_per_camera(c, k), f"{layout} n={n} k={k}")


def test_package_entry_and_rates():
    c = draw_camera_centres(3, 120, "orbit")
    per, d = lr.camera_knn(torch.as_tensor(c), 3)
    assert per.is_cuda and per.dtype == torch.float64 and per.shape == (120,)
    ref = Q.knn_distance(c, 3)
    assert abs(d - ref) <= TOL * ref
    assert lr.knn_distance(c) == d
    d_ref = 0.8
    assert lr.rate_scales(d, d_ref) == pytest.approx(Q.rate_scales(ref, d_ref), rel=1e-13)


def test_largest_rig_sampled():
    n, k = L.KNN_MAX_CAMERAS, L.KNN_MAX_K
    c = draw_camera_centres(11, n, "sphere")
    per, mean = abi_knn(c, k)
    for i in np.random.default_rng(0).choice(n, 12, replace=False).tolist() + [0, n - 1]:
        ref = Q.knn_one(c, i, k)
        assert abs(per[i] - ref) <= TOL * ref, i
    exact = math.fsum(per.tolist()) / n
    assert abs(mean - exact) <= TOL * exact


def test_repeatable_bits():
    c = draw_camera_centres(5, 1000, "forward")
    a = abi_knn(c, 5)
    b = abi_knn(c, 5)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
