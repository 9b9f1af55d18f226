"""Evaluation metrics of Sec. 4.4 -- test infrastructure only."""
from __future__ import annotations

import numpy as np


def error_pixel_percent(ell, gt, eps, sel=None):
    """Eqs. (33), (35): percentage of pixels with |l - l~| > eps."""
    e = np.abs(np.asarray(ell, np.float64) - gt)
    if sel is not None:
        e = e[sel]
    return float(np.mean(e > eps) * 100.0)


def rms_error(ell, gt, sel=None):
    """Eq. (34): root mean squared disparity error."""
    e = np.asarray(ell, np.float64) - gt
    if sel is not None:
        e = e[sel]
    return float(np.sqrt(np.mean(e * e)))


def mde_per_s(u_max, v_max, d_max, t_seconds):
    """Eq. (36): millions of disparity evaluations per second."""
    return u_max * v_max * d_max / t_seconds * 1e-6


def iou(pred, truth, sel=None):
    """Intersection over union of two boolean masks (optionally restricted to
    sel); 1.0 when both are empty."""
    a = np.asarray(pred, bool)
    b = np.asarray(truth, bool)
    if sel is not None:
        a, b = a[sel], b[sel]
    union = np.count_nonzero(a | b)
    return 1.0 if union == 0 else float(np.count_nonzero(a & b) / union)


def sigma_d(values):
    """Eq. (37): population standard deviation of transformed disparities."""
    s = np.asarray(values, np.float64).ravel()
    m = s.size
    return float(np.sqrt(np.sum((s - s.sum() / m) ** 2) / m))
