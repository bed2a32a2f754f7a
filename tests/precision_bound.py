"""Check of the quantised-moment states against dense FP64 Adam.

The oracle's quantised models (``DeferredF32(..., track_bound=True)``) carry,
per element, an a-posteriori bound of |w - w64| along their own trajectory:
bounds of the stored moments' deviation from the exact ones (decayed old bound
+ the actual rounding of every store and block re-encode + FP32 slack), the
largest ratio difference over every exact moment pair inside them (exact
ratios clipped by the Cauchy-Schwarz bound of Adam moments grown from zero,
the model's ratios by its clamp), times lr c_k per step, plus the FP32
rounding of w.  Nothing is assumed about the ratio's size, so subnormal E4M3
codes and lost second moments are covered (the bound then falls back towards
lr c_k (rb + 7.27) per step).  The GPU path equals the model bit for bit, so
the same bound applies to it.
"""
import numpy as np


def check_bound(w_got, model, dense, steps, lrs, tag, rows=None):
    """Assert |w_got - w64| <= bound for every element of both groups.
    w_got: (geo, app) parameter arrays (the model's own or the GPU's);
    rows: optional row selection of the dense model and the bound arrays.
    Returns [(max error, max bound)] per group in units of lr * steps."""
    out = []
    for k, lr in enumerate(lrs):
        ref = dense.w[k] if rows is None else dense.w[k][rows]
        bnd = model.bw[k] if rows is None else model.bw[k][rows]
        err = np.abs(np.asarray(w_got[k], np.float64) - ref)
        bad = np.nonzero(err > bnd)
        assert bad[0].size == 0, (tag, k, bad[0][:5], bad[1][:5], err[bad][:5], bnd[bad][:5])
        scale = lr.astype(np.float64) * steps
        out.append((float((err / scale).max()), float((bnd / scale).max())))
    return out
