"""Comparison rules between the GPU path (FP32) and the FP64 oracle.

  * integer WTA levels: bit-exact, except where the oracle's two smallest
    aggregated costs are within TIE_GAP (absolute; E lies in [0, 2]);
  * valid mask: exact, except pixels whose own or matched-target level is
    such a near-tie;
  * costs C and E: |gpu - oracle| <= COST_TOL * max(|oracle|, 1);
  * sub-pixel level and disparity, where the level matches:
    |gpu - oracle| <= max(SUB_TOL * max(|oracle|, 1), 2 E_TOL / (a + b)).
    The second term is error propagation through Eq. (13): with
    delta = (a - b) / (2 (a + b)), a = E(d-1) - E(d), b = E(d+1) - E(d), and
    each E known to E_TOL, |d delta| <= 2 E_TOL / (a + b).  It matters only
    where the parabola is nearly flat (e.g. at the left border, where many
    levels read identical clamped blocks).
"""
import numpy as np

TIE_GAP = 1e-5
COST_TOL = 1e-4
SUB_TOL = 1e-4
E_TOL = 1e-5


def top2_gap(E):
    s = np.sort(E, axis=0)
    return s[1] - s[0]


def assert_cost_close(gpu, ref, name="cost"):
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - ref) / np.maximum(np.abs(ref), 1.0)
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= COST_TOL, f"{name}: max rel err {err.max():.3g} at {worst}"
    return float(err.max())


def parabola_curvature(E, dint):
    D = E.shape[0]
    dm = np.clip(dint - 1, 0, D - 1)
    dp = np.clip(dint + 1, 0, D - 1)
    e0 = np.take_along_axis(E, dint[None], 0)[0]
    a = np.take_along_axis(E, dm[None], 0)[0] - e0
    b = np.take_along_axis(E, dp[None], 0)[0] - e0
    return a + b


def compare_levels(gpu_dint, ora_dint, gap):
    """Returns (mismatch mask outside near-ties, near-tie mask)."""
    tie = gap < TIE_GAP
    bad = (np.asarray(gpu_dint) != ora_dint) & ~tie
    return bad, tie


def subpixel_tol(ora, curv):
    with np.errstate(divide="ignore"):
        noise = np.where(curv > 0, 2.0 * E_TOL / np.maximum(curv, 1e-300), np.inf)
    return np.maximum(SUB_TOL * np.maximum(np.abs(ora), 1.0), noise)


def assert_subpixel_close(gpu, ora, same, curv, name="subpixel"):
    gpu = np.asarray(gpu, np.float64)
    tol = subpixel_tol(ora, curv)
    err = np.abs(gpu - ora)
    bad = same & ~(err <= tol)
    assert not bad.any(), f"{name}: {bad.sum()} pixels out of tolerance, max err {err[same].max():.3g}"
