"""Comparison rules between the GPU path (FP32) and the FP64 oracle.

  * integer WTA levels: bit-exact, except where the oracle's two smallest
    aggregated costs are within TIE_GAP (absolute; E lies in [0, 2]);
  * valid mask: exact, except pixels whose own or matched-target level is
    such a near-tie;
  * costs C and E: |gpu - oracle| <= COST_TOL * max(|oracle|, 1);
  * sub-pixel level and disparity, where the level matches:
    |gpu - oracle| <= max(SUB_TOL * max(|oracle|, 1), min(2 E_TOL / (a + b), SUB_CAP)).
    The second term is error propagation through Eq. (13): with
    delta = (a - b) / (2 (a + b)), a = E(d-1) - E(d), b = E(d+1) - E(d), and
    each E known to E_TOL, |d delta| <= 2 E_TOL / (a + b).  It is capped at
    SUB_CAP = 1e-2 px, the fixed band for ill-conditioned parabolas, so that
    a nearly flat parabola is still checked to 1/100 px.  Where the oracle's
    curvature a + b is below CURV_FLAT = 4 E_TOL, errors of E_TOL in the three
    costs can change the sign of the curvature, so Eq. (13) has no stable
    value in FP32: such pixels (e.g. at the left border, where many levels
    read identical clamped blocks) are counted, not compared, like near ties.
"""
import numpy as np

TIE_GAP = 1e-5
COST_TOL = 1e-4
SUB_TOL = 1e-4
E_TOL = 1e-5
SUB_CAP = 1e-2
CURV_FLAT = 4 * E_TOL


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
    curv = np.asarray(curv, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        noise = np.where(curv > 0, np.minimum(2.0 * E_TOL / np.maximum(curv, 1e-300), SUB_CAP),
                         SUB_CAP)
    return np.maximum(SUB_TOL * np.maximum(np.abs(ora), 1.0), noise)


def assert_subpixel_close(gpu, ora, same, curv, name="subpixel"):
    """Checks every pixel of `same` outside the flat-parabola set; returns the
    counts: compared, within the relative term, relying on the (capped)
    noise term, and flat parabolas left unchecked."""
    gpu = np.asarray(gpu, np.float64)
    curv = np.asarray(curv, np.float64)
    flat = curv < CURV_FLAT
    check = np.asarray(same, bool) & ~flat
    tol = subpixel_tol(ora, curv)
    err = np.abs(gpu - ora)
    bad = check & ~(err <= tol)
    assert not bad.any(), (f"{name}: {bad.sum()} pixels out of tolerance, max err "
                           f"{err[check].max():.3g}, first at {np.argwhere(bad)[:3].tolist()}")
    rel = check & (err <= SUB_TOL * np.maximum(np.abs(ora), 1.0))
    return dict(compared=int(check.sum()), relative=int(rel.sum()),
                noise=int((check & ~rel).sum()), flat=int((np.asarray(same, bool) & flat).sum()))


def check_selection(w, ora, dR, dT, dsub, valid, disp):
    """Every output against the oracle: levels bit-exact outside near ties,
    validity exact outside excused pixels, sub-pixel levels and disparities
    within the sub-pixel rule.  `ora` holds the oracle's volumes, or (for the
    banded full-frame oracle) the tie gaps and parabola curvature directly.
    Returns the sub-pixel counts."""
    gapR = ora["gapR"] if "gapR" in ora else top2_gap(ora["E_R"])
    gapT = ora["gapT"] if "gapT" in ora else top2_gap(ora["E_T"])
    badR, tieR = compare_levels(dR, ora["dint_R"], gapR)
    badT, tieT = compare_levels(dT, ora["dint_T"], gapT)
    assert not badR.any(), f"dint_R differs at {np.argwhere(badR)[:5].tolist()}"
    assert not badT.any(), f"dint_T differs at {np.argwhere(badT)[:5].tolist()}"
    same = dR == ora["dint_R"]
    curv = ora["curv"] if "curv" in ora else parabola_curvature(ora["E_R"], ora["dint_R"])
    # at the ends of the range Eq. (13) is not applied on either side
    D = w.num_disp
    curv = np.where((ora["dint_R"] > 0) & (ora["dint_R"] < D - 1), curv, np.inf)
    counts = assert_subpixel_close(dsub, ora["ell"], same, curv, "dsub")
    counts["ties"] = int(tieR.sum())
    if valid is None:
        return counts
    H, W = dR.shape
    v, u = np.mgrid[0:H, 0:W]
    x = np.clip(u - ora["dint_R"], 0, W - 1)
    excused = tieR | tieT[v, x] | ~same
    vb = (valid.astype(bool) != ora["valid"]) & ~excused
    assert not vb.any(), f"valid differs at {np.argwhere(vb)[:5].tolist()}"
    both = ora["valid"] & valid.astype(bool) & same
    assert np.all(np.isnan(disp[~valid.astype(bool)]))
    assert_subpixel_close(disp, np.where(both, ora["disp"], 0.0), both, curv, "disp")
    counts["valid_excused"] = int((excused & (valid.astype(bool) != ora["valid"])).sum())
    return counts


def flat_share_ok(counts, w):
    """Flat parabolas must stay an exception: at most 1 % of the compared
    pixels beyond the left band, where every level past u + R + r reads the
    same clamped blocks (there they are structural)."""
    return counts["flat"] <= 0.01 * (counts["compared"] + counts["flat"]) + \
        w.height * (w.num_disp + w.bil_radius + w.ncc_radius)
