"""Helpers shared by the GPU parity tests: upload a workload, call the oracle on
the same stored values, compare with the scale-normalised error."""
import numpy as np
import torch

from oracle import families as F
from oracle import metrics as M
from oracle import nasg_paper as Pp
from oracle import nasg_ref as R
from oracle import sh3_ref as S

NORMS = {"exact": R.NORM_EXACT, "approx": R.NORM_APPROX}


def upload(w, device="cuda"):
    """Device tensors of a workload (lobe params in their storage dtype)."""
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
    if w.dtype == "bf16":
        lob = {k: torch.from_numpy(getattr(w, k + "_bits").view(np.int16)).to(device).view(torch.bfloat16)
               for k in ("quat", "shape", "rgbw")}
    else:
        lob = {k: t(getattr(w, k)) for k in ("quat", "shape", "rgbw")}
    return dict(lob, c0=t(w.c0), means=t(w.means), cams=t(w.cams), dirs=t(w.dirs),
                grad_rgb=t(w.grad_rgb), sh=t(w.sh))


def geo(w):
    return {"dirs": w.dirs} if w.dirs is not None else {"means": w.means, "cams": w.cams}


def dgeo(d):
    return {"dirs": d["dirs"]} if d["dirs"] is not None else {"means": d["means"], "cams": d["cams"]}


FAMILY_CODES = {"nasg": F.NASG, "sg": F.SG, "sb": F.SB, "sc": F.SC, "asg": F.ASG}


def oracle_nasg(w, norm):
    """The oracle for the workload's lobe family and parametrisation
    (quaternion or the paper's raw values)."""
    fam = getattr(w, "family", "nasgabor")
    if fam != "nasgabor":
        out, scale = F.forward_backward(FAMILY_CODES[fam], w.quat, w.shape, w.rgbw, w.c0,
                                        w.grad_rgb, param=w.param, **geo(w))
    else:
        fb = Pp.forward_backward if getattr(w, "param", "quat") == "angles" else R.forward_backward
        out, scale = fb(w.quat, w.shape, w.rgbw, w.c0, w.grad_rgb, NORMS[norm], **geo(w))
    key = "dirs" if w.dirs is not None else "means"
    out["geom"], scale["geom"] = out.pop(key), scale.pop(key)
    return out, scale


def oracle_sh(w):
    out, scale = S.forward_backward(w.sh, w.grad_rgb, **geo(w))
    key = "dirs" if w.dirs is not None else "means"
    out["geom"], scale["geom"] = out.pop(key), scale.pop(key)
    return out, scale


def compare(got, ref, scale, name, tol):
    """Scaled error (gated at `tol`) and the plain relative error (reported)
    of one output or gradient; prints both as max / p99 / median."""
    rep = M.report(got, ref, scale)
    s = rep["scaled"]
    p = rep["plain_rel"]
    print(f"  {name:>12s}: scaled max {s['max']:.2e} p99 {s['p99']:.2e} median {s['median']:.2e}"
          f" | plain rel max {p['max']:.2e} p99 {p['p99']:.2e} median {p['median']:.2e}"
          f" ({p['n']} of {s['n']})")
    assert np.isfinite(np.asarray(got)).all(), f"{name}: non-finite values"
    assert s["max"] <= tol, f"{name}: scaled error {s} above {tol}"
    return s
