"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/nasg.h, and rejects invalid arguments on the host before
any launch (fake device addresses are never dereferenced on these paths)."""
import ctypes as C
import os
import re

import pytest

from paper_2606_09794_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "nasg.h")
FAKE = 0x10000          # aligned fake device address (validation fails before use)


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(nasg_\w+|sh3_\w+)\s*\(", src, re.M)))


def test_exports_match_header(lib):
    names = declared_functions()
    assert {"nasg_eval_fwd", "nasg_eval_bwd", "sh3_eval_fwd", "sh3_eval_bwd"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.EXPORTS, n


def params(**kw):
    d = dict(quat=FAKE, shape=FAKE, rgbw=FAKE, c0=FAKE, n=10, k=4, dtype=0)
    d.update(kw)
    return L.NasgParams(**d)


def views(**kw):
    d = dict(means=FAKE, cams=FAKE, dirs=None, v=2)
    d.update(kw)
    return L.NasgViews(**d)


def fwd(lib, p, v, rgb=FAKE, norm=0):
    return lib.nasg_eval_fwd(C.byref(p) if p is not None else None,
                             C.byref(v) if v is not None else None, rgb, norm, None)


@pytest.mark.parametrize("case,code", [
    (dict(p=None), -1), (dict(k=0), -2), (dict(k=65), -2), (dict(n=-1), -2), (dict(dtype=2), -4),
    (dict(quat=None), -1), (dict(quat=FAKE + 4), -3), (dict(c0=FAKE + 2), -3),
    (dict(v=0), -2), (dict(v=5000), -2), (dict(dirs=FAKE, v=2), -2), (dict(cams=None), -1),
    (dict(rgb=None), -1), (dict(rgb=FAKE + 1), -3), (dict(norm=7), -5),
    (dict(param=2), -5), (dict(param=-1), -5), (dict(family=6), -5), (dict(family=-1), -5),
    (dict(param=1, family=2), -5), (dict(param=1, family=5), -5),
])
def test_fwd_rejects(lib, case, code):
    case = dict(case)
    if "p" in case:
        assert fwd(lib, None, views()) == code
        return
    vkeys = {"v", "dirs", "cams", "means"}
    pk = {k: v for k, v in case.items() if k not in vkeys | {"rgb", "norm"}}
    vk = {k: v for k, v in case.items() if k in vkeys}
    extra = {k: v for k, v in case.items() if k in ("rgb", "norm")}
    assert fwd(lib, params(**pk), views(**vk), **extra) == code


def test_bf16_alignment_is_8_bytes(lib):
    p = params(dtype=1, quat=FAKE + 8, shape=FAKE + 8, rgbw=FAKE + 2)
    # valid alignment for bf16: reaches the mode check and stops there
    assert fwd(lib, p, views(), norm=9) == -5
    assert fwd(lib, params(dtype=1, quat=FAKE + 4), views(), norm=0) == -3


def test_empty_input_needs_no_pointers(lib):
    p = L.NasgParams(None, None, None, None, 0, 4, 0)
    v = L.NasgViews(None, None, None, 3)
    assert lib.nasg_eval_fwd(C.byref(p), C.byref(v), None, 0, None) == 0
    g = L.NasgGrads()
    assert lib.nasg_eval_bwd(C.byref(p), C.byref(v), None, C.byref(g), None, 0, 0, None) == 0
    assert lib.sh3_eval_fwd(None, 0, C.byref(v), None, None) == 0
    assert lib.sh3_eval_bwd(None, 0, C.byref(v), None, None, None, None, 0, None) == 0


def test_bwd_rejects(lib):
    p, v, g = params(), views(), L.NasgGrads(FAKE, FAKE, FAKE, FAKE, FAKE)
    bwd = lambda **kw: lib.nasg_eval_bwd(C.byref(p), C.byref(v), kw.get("grad_rgb", FAKE),  # noqa: E731
                                         kw.get("g", C.byref(g)), kw.get("rgb", None),
                                         kw.get("norm", 0), kw.get("mode", 0), None)
    assert bwd(mode=3) == -5
    assert bwd(norm=-1) == -5
    assert bwd(grad_rgb=None) == -1
    assert bwd(g=None) == -1
    g2 = L.NasgGrads(FAKE + 4, FAKE, FAKE, FAKE, FAKE)
    assert bwd(g=C.byref(g2)) == -3


def test_sh_rejects(lib):
    v = views()
    assert lib.sh3_eval_fwd(None, 5, C.byref(v), FAKE, None) == -1
    assert lib.sh3_eval_fwd(FAKE, -1, C.byref(v), FAKE, None) == -2
    assert lib.sh3_eval_fwd(FAKE + 1, 5, C.byref(v), FAKE, None) == -3
    assert lib.sh3_eval_bwd(FAKE, 5, C.byref(v), FAKE, None, None, None, 2, None) == -5


def test_status_strings_and_tuning(lib):
    for code in range(-7, 1):
        assert lib.nasg_status_string(code)
    t = L.NasgTuning(3, 1, 256)
    assert lib.nasg_set_tuning(1, 8, 16, 0, C.byref(t)) == -2      # 3 lanes unsupported
    t = L.NasgTuning(4, 2, 128)
    assert lib.nasg_set_tuning(1, 8, 16, 0, C.byref(t)) == 0
    out = L.NasgTuning()
    assert lib.nasg_get_tuning(1, 8, 16, 0, C.byref(out)) == 0
    assert (out.lanes, out.views_per_lane, out.block) == (4, 2, 128)
    assert lib.nasg_set_tuning(1, 8, 16, 0, C.byref(L.NasgTuning(0, 0, 0))) == 0
    assert lib.nasg_get_tuning(1, 8, 16, 0, C.byref(out)) == 0
    assert (out.lanes, out.views_per_lane) == (4, 4)           # built-in choice for V = 16
    assert lib.nasg_set_tuning(9, 8, 16, 0, C.byref(t)) == -5


def test_batched_rejects(lib):
    sc = (L.NasgScene * 1)()
    sc[0] = L.NasgScene(params(), views(), FAKE, L.NasgGrads(FAKE, FAKE, FAKE, FAKE, FAKE), None)
    out = L.NasgBatch()
    t = L.NasgBatchTuning(4, 2)
    need = lib.nasg_batched_workspace_bytes(sc, 1, C.byref(t))
    assert need > 64
    plan = lambda ws=FAKE, nbytes=need, norm=0, tt=C.byref(t), o=C.byref(out): \
        lib.nasg_batched_plan(sc, 1, norm, tt, ws, nbytes, o, None)  # noqa: E731
    assert plan(o=None) == -1
    assert plan(norm=4) == -5
    assert plan(tt=C.byref(L.NasgBatchTuning(0, 2))) == -2
    assert plan(tt=C.byref(L.NasgBatchTuning(4, 9))) == -2
    assert plan(ws=None) == -7
    assert plan(nbytes=need - 1) == -7
    assert plan(ws=FAKE + 16) == -7
    sc[0].p.dtype = 1
    assert plan() == -4
    sc[0].p.dtype = 0
    sc[0].p.family = 2                                   # only NASGabor lobes are batched
    assert plan() == -5
    sc[0].p.family = 0
    sc[0].grad_rgb = None
    assert plan() == -1
    assert lib.nasg_batched_run(None, None) == -1
    empty = L.NasgBatch(FAKE, 0, 0, 0, 1, 0, 0)
    assert lib.nasg_batched_run(C.byref(empty), None) == 0      # nothing to launch
    bad = L.NasgBatch(FAKE, 0, 5, 1, 1, 0, 1, 2)                # raw-values flag neither 0 nor 1
    assert lib.nasg_batched_run(C.byref(bad), None) == -7
    assert C.sizeof(L.NasgBatch) == 48                          # the C layout of nasg_batch
    # the work list grows with the tile count: at V = 2 a primitive has one lane,
    # so one tile is 4 passes x 256 primitives
    sc[0].grad_rgb = FAKE
    sc[0].p.n = 1024 * 3 + 1
    assert lib.nasg_batched_workspace_bytes(sc, 1, C.byref(t)) == need + 3 * 16


def test_raster_rejects(lib):
    cam = L.NasgCamera((C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1), (C.c_double * 3)(0, 0, 0),
                       100.0, 100.0, 32.0, 24.0, 64, 48)
    need = lib.nasg_raster_workspace_bytes(10, C.byref(cam), 256)
    # 4 x 3 tiles: header, cursors, lists [12][256] of 8-byte keys, 64-byte render
    # and 16-byte bin records, per-pixel FP64 (t, E), FP64 accumulators [N][10],
    # each part 256-byte aligned
    assert need == 256 + 256 + 12 * 256 * 8 + 768 + 256 + 64 * 48 * 2 * 8 + 10 * 80
    assert lib.nasg_raster_workspace_bytes(10, C.byref(cam), 0) == 0
    assert lib.nasg_raster_workspace_bytes(10, C.byref(cam), 4097) == 0
    assert lib.nasg_raster_workspace_bytes(-1, C.byref(cam), 256) == 0
    assert lib.nasg_raster_workspace_bytes(10, None, 256) == 0
    g = L.NasgGaussians(FAKE, FAKE, FAKE, FAKE, FAKE, 10)
    fwd = lambda gg=C.byref(g), cc=C.byref(cam), cap=256, ws=FAKE, nb=need, img=FAKE: \
        lib.nasg_raster_fwd(gg, cc, cap, ws, nb, img, None)  # noqa: E731
    assert fwd(gg=None) == -1
    assert fwd(cc=None) == -1
    assert fwd(cap=0) == -2
    assert fwd(ws=None) == -1
    assert fwd(nb=need - 1) == -7
    assert fwd(ws=FAKE + 64) == -3
    assert fwd(img=None) == -1
    assert fwd(img=FAKE + 2) == -3
    bad = L.NasgCamera(cam.rot, cam.t, 1.0, 1.0, 0.0, 0.0, 0, 48)
    assert fwd(cc=C.byref(bad)) == -2
    g.opac = None
    assert fwd() == -1
    g.opac = FAKE
    g.rots = FAKE + 1
    assert fwd() == -3
    g.rots = FAKE
    bwd = lambda nb=need, gi=FAKE, gc=FAKE, go=FAKE, gm=None, gs=None, gr=None: \
        lib.nasg_raster_bwd(C.byref(g), C.byref(cam), 256, FAKE, nb, gi, gc, go, gm, gs, gr,  # noqa: E731
                            None)
    assert bwd(gi=None) == -1
    assert bwd(nb=need - 8) == -7
    assert bwd(gc=FAKE + 1) == -3
    assert bwd(go=FAKE + 2) == -3
    assert bwd(gm=FAKE + 2) == -3
    assert bwd(gs=FAKE + 1) == -3
    assert bwd(gr=FAKE + 3) == -3


def test_hbm_stream_rejects(lib):
    s = lambda mode=2, src=FAKE, dst=FAKE + 4096, nb=4096, blocks=256, unroll=4, nt=0: \
        lib.nasg_hbm_stream(mode, src, dst, nb, blocks, unroll, nt, None)  # noqa: E731
    assert s(mode=3) == -5
    assert s(mode=-1) == -5
    assert s(nb=4095) == -2                 # not a multiple of 16 bytes
    assert s(nb=-16) == -2
    assert s(blocks=0) == -2
    assert s(blocks=(1 << 20) + 1) == -2
    assert s(unroll=3) == -2
    assert s(nt=2) == -2
    assert s(src=None) == -1
    assert s(dst=None) == -1
    assert s(mode=1, src=None, dst=FAKE + 8) == -3    # write: src unused, dst misaligned
    assert s(src=FAKE + 4) == -3
    assert s(nb=0) == 0                      # nothing to stream, nothing launched


def test_camera_knn_rejects(lib):
    f = lambda c=FAKE, n=40, k=3, per=FAKE + 4096, mean=FAKE + 8192: \
        lib.nasg_camera_knn(c, n, k, per, mean, None)  # noqa: E731
    assert f(k=0) == -2
    assert f(k=L.KNN_MAX_K + 1) == -2
    assert f(n=3) == -2                      # needs more than k cameras
    assert f(n=L.KNN_MAX_CAMERAS + 1) == -2
    assert f(c=None) == -1
    assert f(per=None) == -1
    assert f(mean=None) == -1
    assert f(c=FAKE + 4) == -3
    assert f(mean=FAKE + 8196) == -3


def test_raster_fwd_noalloc_rejects(lib):
    """Invalid arguments, and a workspace beyond the fixed scratch, are refused
    on the host before the runtime is touched."""
    cam = L.NasgCamera((C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1), (C.c_double * 3)(0, 0, 0),
                       100.0, 100.0, 32.0, 24.0, 64, 48)
    g = L.NasgGaussians(FAKE, FAKE, FAKE, FAKE, FAKE, 10)
    f = lambda gg=C.byref(g), cc=C.byref(cam), cap=256, img=FAKE, ov=None: \
        lib.nasg_raster_fwd_noalloc(gg, cc, cap, img, ov, None)  # noqa: E731
    assert f(gg=None) == -1
    assert f(cc=None) == -1
    assert f(cap=0) == -2
    assert f(img=None) == -1
    assert f(img=FAKE + 2) == -3
    assert f(ov=FAKE + 1) == -3
    g.opac = None
    assert f() == -1
    g.opac = FAKE
    # 1920 x 1080 at capacity 4096 needs 0.27 GB of lists alone: beyond the 64 MiB
    big = L.NasgCamera(cam.rot, cam.t, 1000.0, 1000.0, 960.0, 540.0, 1920, 1080)
    need = lib.nasg_raster_workspace_bytes(10, C.byref(big), 4096)
    assert need > L.NOALLOC_SCRATCH_BYTES
    assert f(cc=C.byref(big), cap=4096) == -7
