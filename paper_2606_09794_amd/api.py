"""Torch-facing wrappers of the C ABI and the autograd Functions.

PyTorch provides device memory and the current HIP stream; every step of the
evaluation runs in libnasg's kernels. Inputs must be contiguous device
tensors in the layouts of ``include/nasg.h``:

    quat [K][N][4], shape [K][N][4], rgbw [K][3][N]   float32 or bfloat16
    c0 [N][3], means [N][3], cams [V][3] or dirs [N][3], grad_rgb [V][N][3]
    sh [16][3][N]                                       float32

``family`` picks the lobe ("nasgabor" default, or "nasg", "sg", "sb", "sc",
"asg"; see include/nasg.h for each family's shape values).
``param="quat"`` (default) reads quat / shape / rgbw as a quaternion frame,
(lambda, a, k, zeta) and weights; ``param="angles"`` reads the paper's raw
pre-activation values in the same slots (frame cosines tanh(u), lambda and a
e^u, k = 20 (tanh u + 1), weights tanh u) and returns gradients with respect
to those raw values.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

import torch

from . import _lib as L

_NORMS = {"exact": L.NORM_EXACT, "approx": L.NORM_APPROX}
_PARAMS = {"quat": L.PARAM_QUAT, "angles": L.PARAM_ANGLES}


def _param_code(param) -> int:
    if isinstance(param, str):
        if param not in _PARAMS:
            raise ValueError(f"param must be one of {sorted(_PARAMS)}")
        return _PARAMS[param]
    return int(param)


def _norm_code(norm) -> int:
    if isinstance(norm, str):
        if norm not in _NORMS:
            raise ValueError(f"norm must be one of {sorted(_NORMS)}")
        return _NORMS[norm]
    return int(norm)


def _dev(t: Optional[torch.Tensor], name: str, dtype=torch.float32) -> Optional[torch.Tensor]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _out(t: Optional[torch.Tensor], name: str, shape) -> Optional[torch.Tensor]:
    """A caller-supplied output buffer: float32, on the device, contiguous and
    of exactly `shape` (the kernels write that many elements through a raw
    pointer, so a smaller buffer would be overrun)."""
    if t is None:
        return None
    _dev(t, name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _grad_shapes(k: int, n: int):
    return {"quat": (k, n, 4), "shape": (k, n, 4), "rgbw": (k, 3, n), "c0": (n, 3),
            "geom": (n, 3)}


def _check_grads(grads, k: int, n: int, where: str = "grads") -> None:
    shapes = _grad_shapes(k, n)
    for name, t in grads.items():
        if name not in shapes:
            raise ValueError(f"{where}: unknown gradient {name!r} (expected {sorted(shapes)})")
        _out(t, f"{where}[{name}]", shapes[name])


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _views(n: int, means, cams, dirs):
    if dirs is not None:
        dirs = _dev(dirs, "dirs")
        if tuple(dirs.shape) != (n, 3):
            raise ValueError("dirs must be [N][3]")
        return L.NasgViews(None, None, dirs.data_ptr(), 1), 1
    means = _dev(means, "means")
    cams = _dev(cams, "cams")
    if means is None or cams is None:
        raise ValueError("give either dirs or both means and cams")
    if tuple(means.shape) != (n, 3) or cams.dim() != 2 or cams.shape[1] != 3:
        raise ValueError("means must be [N][3] and cams [V][3]")
    v = int(cams.shape[0])
    return L.NasgViews(means.data_ptr(), cams.data_ptr(), None, v), v


def _family_code(family) -> int:
    if isinstance(family, str):
        if family not in L.FAMILIES:
            raise ValueError(f"family must be one of {sorted(L.FAMILIES)}")
        return L.FAMILIES[family]
    return int(family)


def _params(quat, shape, rgbw, c0, param="quat", family="nasgabor"):
    dt = quat.dtype
    if dt not in (torch.float32, torch.bfloat16):
        raise ValueError("lobe parameters must be float32 or bfloat16")
    _dev(quat, "quat", dt)
    _dev(shape, "shape", dt)
    _dev(rgbw, "rgbw", dt)
    _dev(c0, "c0")
    k, n = int(quat.shape[0]), int(quat.shape[1])
    if (tuple(quat.shape) != (k, n, 4) or tuple(shape.shape) != (k, n, 4)
            or tuple(rgbw.shape) != (k, 3, n) or tuple(c0.shape) != (n, 3)):
        raise ValueError("expected quat/shape [K][N][4], rgbw [K][3][N], c0 [N][3]")
    code = L.NASG_F32 if dt == torch.float32 else L.NASG_BF16
    return L.NasgParams(quat.data_ptr(), shape.data_ptr(), rgbw.data_ptr(), c0.data_ptr(),
                        n, k, code, _param_code(param), _family_code(family)), k, n


def nasg_eval_fwd(quat, shape, rgbw, c0, *, means=None, cams=None, dirs=None, norm="exact",
                  out: Optional[torch.Tensor] = None, param="quat", family="nasgabor"
                  ) -> torch.Tensor:
    """Per-view colours rgb[V][N][3] (Section 4.2 model; NASGabor lobes or
    another family of the distribution table, ``family``)."""
    p, k, n = _params(quat, shape, rgbw, c0, param, family)
    vw, v = _views(n, means, cams, dirs)
    if out is None:
        out = torch.empty((v, n, 3), device=quat.device, dtype=torch.float32)
    _out(out, "out", (v, n, 3))
    L.check(L.lib().nasg_eval_fwd(C.byref(p), C.byref(vw), _p(out), _norm_code(norm), _stream()),
            "nasg_eval_fwd")
    return out


def nasg_grad_buffers(k: int, n: int, device) -> Dict[str, torch.Tensor]:
    f = dict(device=device, dtype=torch.float32)
    return {"quat": torch.empty((k, n, 4), **f), "shape": torch.empty((k, n, 4), **f),
            "rgbw": torch.empty((k, 3, n), **f), "c0": torch.empty((n, 3), **f),
            "geom": torch.empty((n, 3), **f)}


def nasg_eval_bwd(quat, shape, rgbw, c0, grad_rgb, *, means=None, cams=None, dirs=None,
                  norm="exact", grads: Optional[Dict[str, torch.Tensor]] = None,
                  accumulate: bool = False, rgb_out: Optional[torch.Tensor] = None,
                  param="quat", family="nasgabor") -> Dict[str, torch.Tensor]:
    """Gradients of sum(grad_rgb * rgb) w.r.t. quat, shape, rgbw, c0 and the
    means (or dirs) as float32 tensors (dict keys quat, shape, rgbw, c0, geom).
    With ``rgb_out`` the forward colours are written in the same pass."""
    p, k, n = _params(quat, shape, rgbw, c0, param, family)
    vw, v = _views(n, means, cams, dirs)
    _dev(grad_rgb, "grad_rgb")
    if tuple(grad_rgb.shape) != (v, n, 3):
        raise ValueError("grad_rgb must be [V][N][3]")
    if grads is None:
        grads = nasg_grad_buffers(k, n, quat.device)
    _check_grads(grads, k, n)
    _out(rgb_out, "rgb_out", (v, n, 3))
    g = L.NasgGrads(*(grads[x].data_ptr() if grads.get(x) is not None else None
                      for x in ("quat", "shape", "rgbw", "c0", "geom")))
    L.check(L.lib().nasg_eval_bwd(C.byref(p), C.byref(vw), _p(grad_rgb), C.byref(g), _p(rgb_out),
                                  _norm_code(norm),
                                  L.GRAD_ACCUMULATE if accumulate else L.GRAD_OVERWRITE,
                                  _stream()), "nasg_eval_bwd")
    return grads


def sh3_eval_fwd(sh, *, means=None, cams=None, dirs=None,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Degree-3 SH colours rgb[V][N][3] (Section 3.2)."""
    _dev(sh, "sh")
    if sh.dim() != 3 or tuple(sh.shape[:2]) != (16, 3):
        raise ValueError("sh must be [16][3][N]")
    n = int(sh.shape[2])
    vw, v = _views(n, means, cams, dirs)
    if out is None:
        out = torch.empty((v, n, 3), device=sh.device, dtype=torch.float32)
    _out(out, "out", (v, n, 3))
    L.check(L.lib().sh3_eval_fwd(_p(sh), n, C.byref(vw), _p(out), _stream()), "sh3_eval_fwd")
    return out


def sh3_eval_bwd(sh, grad_rgb, *, means=None, cams=None, dirs=None,
                 grads: Optional[Dict[str, torch.Tensor]] = None, accumulate: bool = False,
                 rgb_out: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
    """Gradients w.r.t. sh and the means (or dirs): dict keys sh, geom."""
    _dev(sh, "sh")
    if sh.dim() != 3 or tuple(sh.shape[:2]) != (16, 3):
        raise ValueError("sh must be [16][3][N]")
    n = int(sh.shape[2])
    vw, v = _views(n, means, cams, dirs)
    _dev(grad_rgb, "grad_rgb")
    if tuple(grad_rgb.shape) != (v, n, 3):
        raise ValueError("grad_rgb must be [V][N][3]")
    if grads is None:
        grads = {"sh": torch.empty_like(sh), "geom": torch.empty((n, 3), device=sh.device)}
    shapes = {"sh": (16, 3, n), "geom": (n, 3)}
    for name, t in grads.items():
        if name not in shapes:
            raise ValueError(f"grads: unknown gradient {name!r} (expected ['geom', 'sh'])")
        _out(t, f"grads[{name}]", shapes[name])
    _out(rgb_out, "rgb_out", (v, n, 3))
    L.check(L.lib().sh3_eval_bwd(_p(sh), n, C.byref(vw), _p(grad_rgb), _p(grads.get("sh")),
                                 _p(grads.get("geom")), _p(rgb_out),
                                 L.GRAD_ACCUMULATE if accumulate else L.GRAD_OVERWRITE,
                                 _stream()), "sh3_eval_bwd")
    return grads


class NasgBatchPlan:
    """A planned multi-scene fused forward+backward (one persistent launch).

    ``scenes`` is a list of dicts with device tensors quat, shape, rgbw, c0,
    means, cams, grad_rgb, the float32 gradient buffers ``grads`` (dict as
    returned by nasg_grad_buffers) and optionally ``rgb`` [V][N][3]. The plan
    keeps references to every tensor it points at; ``run()`` only launches
    kernels and can be captured into a CUDA/HIP graph. ``tile_iters`` and
    ``blocks_per_cu`` default to the tuner's cached choice (autotune.tune_batch)."""

    def __init__(self, scenes, norm="exact", tile_iters=None, blocks_per_cu=None):
        if tile_iters is None or blocks_per_cu is None:
            from .autotune import batch_defaults
            dt, db = batch_defaults()
            tile_iters = dt if tile_iters is None else tile_iters
            blocks_per_cu = db if blocks_per_cu is None else blocks_per_cu
        arr = (L.NasgScene * len(scenes))()
        self._keep = []
        for idx, sc in enumerate(scenes):
            p, k, n = _params(sc["quat"], sc["shape"], sc["rgbw"], sc["c0"], sc.get("param", "quat"))
            vw, v = _views(n, sc.get("means"), sc.get("cams"), sc.get("dirs"))
            _dev(sc["grad_rgb"], "grad_rgb")
            if tuple(sc["grad_rgb"].shape) != (v, n, 3):
                raise ValueError("grad_rgb must be [V][N][3]")
            g = sc["grads"]
            _check_grads(g, k, n, f"scene {idx} grads")
            _out(sc.get("rgb"), f"scene {idx} rgb", (v, n, 3))
            arr[idx] = L.NasgScene(p, vw, sc["grad_rgb"].data_ptr(),
                                   L.NasgGrads(*(g[x].data_ptr() if g.get(x) is not None else None
                                                 for x in ("quat", "shape", "rgbw", "c0", "geom"))),
                                   sc["rgb"].data_ptr() if sc.get("rgb") is not None else None)
            self._keep.append(sc)
        self._scenes = arr
        tun = L.NasgBatchTuning(tile_iters, blocks_per_cu)
        nbytes = L.lib().nasg_batched_workspace_bytes(arr, len(scenes), C.byref(tun))
        if nbytes == 0 and len(scenes) > 0:
            raise ValueError("invalid scenes or tuning for a batched plan")
        dev = scenes[0]["quat"].device if scenes else torch.device("cuda")
        self.workspace = torch.empty(max(nbytes, 64), dtype=torch.uint8, device=dev)
        self.batch = L.NasgBatch()
        L.check(L.lib().nasg_batched_plan(arr, len(scenes), _norm_code(norm), C.byref(tun),
                                          C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                          C.byref(self.batch), _stream()), "nasg_batched_plan")

    @property
    def n_items(self) -> int:
        return self.batch.n_items

    def run(self) -> None:
        L.check(L.lib().nasg_batched_run(C.byref(self.batch), _stream()), "nasg_batched_run")


def set_tuning(kernel: int, k: int, v: int, dtype: int, lanes: int, views_per_lane: int,
               block: int = 256, bcast: int = 0) -> None:
    t = L.NasgTuning(lanes, views_per_lane, block, bcast)
    L.check(L.lib().nasg_set_tuning(kernel, k, v, dtype, C.byref(t)), "nasg_set_tuning")


def get_tuning(kernel: int, k: int, v: int, dtype: int):
    """(lanes, views_per_lane, block, bcast) a call with this key would use."""
    t = L.NasgTuning()
    L.check(L.lib().nasg_get_tuning(kernel, k, v, dtype, C.byref(t)), "nasg_get_tuning")
    return (t.lanes, t.views_per_lane, t.block, t.bcast)


# ------------------------------------------------------------------ autograd

class NasgEval(torch.autograd.Function):
    """rgb = NasgEval.apply(quat, shape, rgbw, c0, means, cams, dirs, norm, param).

    Backward calls the analytic backward kernel; cams get no gradient. With
    bfloat16 lobe parameters the float32 gradients are rounded to bfloat16 to
    match the parameter dtype. With param="angles" the lobe tensors are the
    paper's raw values and so are their gradients."""

    @staticmethod
    def forward(ctx, quat, shape, rgbw, c0, means, cams, dirs, norm="exact", param="quat"):
        rgb = nasg_eval_fwd(quat, shape, rgbw, c0, means=means, cams=cams, dirs=dirs, norm=norm,
                            param=param)
        ctx.save_for_backward(quat, shape, rgbw, c0, means, cams, dirs)
        ctx.norm = norm
        ctx.param = param
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        quat, shape, rgbw, c0, means, cams, dirs = ctx.saved_tensors
        g = nasg_eval_bwd(quat, shape, rgbw, c0, grad_rgb.contiguous(), means=means, cams=cams,
                          dirs=dirs, norm=ctx.norm, param=ctx.param)
        dt = quat.dtype
        gm = g["geom"] if dirs is None else None
        gd = g["geom"] if dirs is not None else None
        return (g["quat"].to(dt), g["shape"].to(dt), g["rgbw"].to(dt), g["c0"], gm, None, gd,
                None, None)


class SH3Eval(torch.autograd.Function):
    """rgb = SH3Eval.apply(sh, means, cams, dirs)."""

    @staticmethod
    def forward(ctx, sh, means, cams, dirs):
        rgb = sh3_eval_fwd(sh, means=means, cams=cams, dirs=dirs)
        ctx.save_for_backward(sh, means, cams, dirs)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        sh, means, cams, dirs = ctx.saved_tensors
        g = sh3_eval_bwd(sh, grad_rgb.contiguous(), means=means, cams=cams, dirs=dirs)
        gm = g["geom"] if dirs is None else None
        gd = g["geom"] if dirs is not None else None
        return g["sh"], gm, None, gd


# ------------------------------------------------------------- compositing

class Camera:
    """Pinhole camera for compositing: x_cam = rot @ x + t (rot = world-to-
    camera rotation), pixel u = fx X/Z + cx, v = fy Y/Z + cy."""

    def __init__(self, rot, t, fx, fy, cx, cy, width, height):
        self.rot = [float(x) for x in torch.as_tensor(rot, dtype=torch.float64).reshape(9)]
        self.t = [float(x) for x in torch.as_tensor(t, dtype=torch.float64).reshape(3)]
        self.fx, self.fy, self.cx, self.cy = float(fx), float(fy), float(cx), float(cy)
        self.width, self.height = int(width), int(height)

    def struct(self) -> L.NasgCamera:
        c = L.NasgCamera()
        c.rot[:] = self.rot
        c.t[:] = self.t
        c.fx, c.fy, c.cx, c.cy = self.fx, self.fy, self.cx, self.cy
        c.width, c.height = self.width, self.height
        return c

    def centre(self, device) -> torch.Tensor:
        """Camera centre o = -rot^T t as a [1][3] float32 device tensor (the
        view input of the appearance evaluation)."""
        r = torch.tensor(self.rot, dtype=torch.float64).reshape(3, 3)
        o = -(r.T @ torch.tensor(self.t, dtype=torch.float64))
        return o.to(torch.float32).reshape(1, 3).to(device)


def _gaussians(means, scales, rots, opac, colors) -> L.NasgGaussians:
    n = means.shape[0]
    for t, name, shape in ((means, "means", (n, 3)), (scales, "scales", (n, 3)),
                           (rots, "rots", (n, 4)), (opac, "opac", (n,)),
                           (colors, "colors", (n, 3))):
        _dev(t, name)
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    return L.NasgGaussians(_p(means), _p(scales), _p(rots), _p(opac), _p(colors), n)


def raster_workspace_bytes(n: int, cam: Camera, tile_capacity: int = 1024) -> int:
    b = L.lib().nasg_raster_workspace_bytes(n, C.byref(cam.struct()), tile_capacity)
    if b == 0:
        raise ValueError("invalid compositing size (n, image side or tile capacity)")
    return int(b)


def raster_fwd(means, scales, rots, opac, colors, cam: Camera, tile_capacity: int = 1024,
               workspace: Optional[torch.Tensor] = None, check_overflow: bool = True):
    """image [H][W][3] and the workspace the backward needs. With
    check_overflow the call waits for the device and raises if a tile list
    overflowed (the image would miss primitives)."""
    g = _gaussians(means, scales, rots, opac, colors)
    cs = cam.struct()
    nb = raster_workspace_bytes(g.n, cam, tile_capacity)
    if workspace is not None:
        _dev(workspace, "workspace", torch.uint8)   # its numel() is its size in bytes
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=means.device)
    img = torch.empty(cam.height, cam.width, 3, dtype=torch.float32, device=means.device)
    L.check(L.lib().nasg_raster_fwd(C.byref(g), C.byref(cs), tile_capacity,
                                    _p(workspace), workspace.numel(), _p(img), _stream()),
            "nasg_raster_fwd")
    if check_overflow and int(workspace[:4].view(torch.int32).item()) != 0:
        raise L.NasgError(f"a tile holds more than {tile_capacity} primitives; "
                          "raise tile_capacity")
    return img, workspace


def raster_bwd(means, scales, rots, opac, colors, cam: Camera, workspace, grad_image,
               tile_capacity: int = 1024, geometry: bool = False):
    """(grad_colors [N][3], grad_opac [N]) of L = sum(grad_image * image),
    with the workspace of the forward on the same inputs; with geometry=True
    also (grad_means [N][3], grad_scales [N][3], grad_rots [N][4])."""
    g = _gaussians(means, scales, rots, opac, colors)
    cs = cam.struct()
    _dev(grad_image, "grad_image")
    _dev(workspace, "workspace", torch.uint8)
    if tuple(grad_image.shape) != (cam.height, cam.width, 3):
        raise ValueError(f"grad_image must have shape {(cam.height, cam.width, 3)}")
    gc = torch.empty_like(colors)
    go = torch.empty_like(opac)
    geo = [torch.empty_like(t) for t in (means, scales, rots)] if geometry else [None] * 3
    L.check(L.lib().nasg_raster_bwd(C.byref(g), C.byref(cs), tile_capacity, _p(workspace),
                                    workspace.numel(), _p(grad_image), _p(gc), _p(go),
                                    *(_p(t) for t in geo), _stream()), "nasg_raster_bwd")
    return (gc, go, *geo) if geometry else (gc, go)


class Rasterize(torch.autograd.Function):
    """image = Rasterize.apply(means, scales, rots, opac, colors, cam,
    tile_capacity). Gradients flow to opac and colors (the colours carry them
    on to the appearance model) and, when any of them requires it, to means,
    scales and rots through the projection."""

    @staticmethod
    def forward(ctx, means, scales, rots, opac, colors, cam, tile_capacity=1024):
        img, ws = raster_fwd(means, scales, rots, opac, colors, cam, tile_capacity)
        ctx.save_for_backward(means, scales, rots, opac, colors, ws)
        ctx.cam = cam
        ctx.cap = tile_capacity
        return img

    @staticmethod
    def backward(ctx, grad_image):
        means, scales, rots, opac, colors, ws = ctx.saved_tensors
        geometry = any(ctx.needs_input_grad[:3])
        out = raster_bwd(means, scales, rots, opac, colors, ctx.cam, ws,
                         grad_image.contiguous(), ctx.cap, geometry=geometry)
        gm, gs, gr = out[2:] if geometry else (None, None, None)
        return gm, gs, gr, out[1], out[0], None, None


def render_view(quat, shape, rgbw, c0, means, scales, rots, opac, cam: Camera, *,
                norm="exact", param="quat", tile_capacity=1024):
    """One training view: the central-ray colour of every primitive for this
    camera (one appearance evaluation per primitive, Section 5.2), composited
    into the image (Section 3.1). Differentiable in the lobe parameters, c0,
    the opacities, and the means (through the view direction and the
    projection), scales and rotations (through the projection)."""
    rgb = NasgEval.apply(quat, shape, rgbw, c0, means, cam.centre(means.device), None, norm,
                         param)
    return Rasterize.apply(means, scales, rots, opac, rgb[0], cam, tile_capacity)
