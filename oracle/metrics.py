"""Error metric for parity against the FP64 oracle (test infrastructure).

For an output or gradient element y with oracle value y_ref, the error is
    e = |y - y_ref| / S,
where S is the sum of the absolute values of the elementary terms that the
oracle adds up to form y_ref (for a colour, |c0| + sum_l |w_l G_l|; for a
gradient, the absolute per-view, per-lobe and per-product-rule-term
contributions). S is the natural scale of the rounding error of a sum, and it
stays meaningful where terms cancel or where a lobe underflows.
"""
from __future__ import annotations

import numpy as np


def scaled_error(y, y_ref, scale, floor=1e-30):
    y = np.asarray(y, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    return np.abs(y - y_ref) / (np.asarray(scale, np.float64) + floor)


def summarize(err):
    err = np.asarray(err, np.float64).ravel()
    if err.size == 0:
        return {"max": 0.0, "p99": 0.0, "median": 0.0, "n": 0}
    return {"max": float(err.max()), "p99": float(np.percentile(err, 99)),
            "median": float(np.median(err)), "n": int(err.size)}
