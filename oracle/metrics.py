"""Error metric for parity against the FP64 oracle (test infrastructure).

For an output or gradient element y with oracle value y_ref, the error is
    e = |y - y_ref| / S,
where S is the sum of the absolute values of the elementary terms that the
oracle adds up to form y_ref (for a colour, |c0| + sum_l |w_l G_l|; for a
gradient, the absolute per-view, per-lobe and per-product-rule-term
contributions). S is the natural scale of the rounding error of a sum, and it
stays meaningful where terms cancel or where a lobe underflows.

The secondary metric is the plain relative error |y - y_ref| / |y_ref| on the
elements whose |y_ref| exceeds 1e-3 of the tensor's largest |y_ref| (elements
far below that are left out: their plain relative error measures the
cancellation in the sum, not the evaluation). Both are reported as
max / p99 / median per output and per gradient.
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


def plain_relative(y, y_ref, rel_floor=1e-3):
    """|y - y_ref| / |y_ref| on the elements with |y_ref| > rel_floor * max |y_ref|."""
    y = np.asarray(y, np.float64).ravel()
    y_ref = np.asarray(y_ref, np.float64).ravel()
    if y_ref.size == 0:
        return np.zeros(0)
    a = np.abs(y_ref)
    keep = a > rel_floor * a.max()
    return np.abs(y[keep] - y_ref[keep]) / a[keep]


def report(y, y_ref, scale):
    """Both metrics of one output or gradient tensor, summarised."""
    return {"scaled": summarize(scaled_error(y, y_ref, scale)),
            "plain_rel": summarize(plain_relative(y, y_ref))}
