"""MI355X-native NASGabor / degree-3 SH appearance evaluation.

The compute path is libnasg.so (hand-written HIP for gfx950, C ABI in
``include/nasg.h``); this package is its thin binding. Build the library with
``python -m paper_2606_09794_amd.build``.
"""
from .api import (  # noqa: F401
    Camera,
    NasgBatchPlan,
    NasgEval,
    SH3Eval,
    get_tuning,
    nasg_eval_bwd,
    nasg_eval_fwd,
    nasg_grad_buffers,
    raster_bwd,
    raster_fwd,
    raster_workspace_bytes,
    Rasterize,
    render_view,
    set_tuning,
    sh3_eval_bwd,
    sh3_eval_fwd,
)
from ._lib import LIB_PATH, NasgError, lib  # noqa: F401
