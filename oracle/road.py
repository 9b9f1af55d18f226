"""FP64 oracle of the disparity transformation (Sec. 3.3) -- test infrastructure only.

  energy(psi)     E_t,min(psi) = d'd - d'Y (Y'Y)^-1 Y'd,  Eq. (23), with
                  Y(psi) = [1, y(psi)], y = v cos psi - u sin psi (Eq. 19)
  gradient(psi)   Eq. (26): -2 d' W(psi) d, W = (I - Y J) dY J (Eq. 27),
                  evaluated without forming the n x n matrix: with the
                  residual r = d - Y alpha, d'(I - YJ) = r', so the gradient is
                  -2 r' dY alpha = -2 alpha_1 sum_i r_i y'_i
  alpha(psi)      Eq. (21): alpha = J(psi) d
  fit_roll        gradient descent on psi, Eq. (25), with the adaptive rate of
                  Eq. (28), from psi0 (0, or the previous frame's psi)
  transform       Eq. (29): l' = l - a0 + a1 (u sin psi - v cos psi) + delta_t

Readings where the paper is silent (also in the design notes):
  * the energy is minimised in normalised form E / (n s^2 a1(psi0)^2) with
    s = max(W, H); this is the scale at which the paper's lambda0 = 10 is a
    sensible first step (for a roll error dpsi the raw energy grows like
    n a1^2 var(x) dpsi^2).  When |a1(psi0)| < 1e-6 the scale uses a1 = 1 and
    the fit returns psi0 unchanged (no slope, no roll information);
  * safeguard: a step is halved while it raises the energy (by more than a
    relative 1e-9, the rounding level of Eq. (23) evaluated in FP64 for maps
    whose plane explains most of the variance) or exceeds pi/4;
    a non-positive or non-finite rate from Eq. (28) restarts at lambda0;
  * psi is wrapped into (-pi/2, pi/2] (E_min has period pi);
  * the iteration stops when |psi_k+1 - psi_k| < delta_psi, when the gradient
    no longer changes, or after max_iter steps (then "not converged").
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

F64 = np.float64
DELTA_PSI = math.pi / 1.8e6      # Sec. 4.4.2: 0.0001 degree
LAMBDA0 = 10.0                   # Sec. 4.4.2


@dataclass
class RoadFit:
    psi: float
    alpha0: float
    alpha1: float
    e_min: float
    iters: int
    converged: bool
    flat: bool

    @property
    def plane(self):
        """Road disparity plane implied by the fit: a0 + a1 y(psi)."""
        return (self.alpha0, -self.alpha1 * math.sin(self.psi),
                self.alpha1 * math.cos(self.psi))


def road_points(disp, valid=None, mask=None):
    """(u, v, d) of the pixels used by the fit: valid, finite and in the mask."""
    disp = np.asarray(disp, F64)
    H, W = disp.shape
    v, u = np.mgrid[0:H, 0:W]
    sel = np.isfinite(disp)
    if valid is not None:
        sel &= np.asarray(valid, bool)
    if mask is not None:
        sel &= np.asarray(mask, bool)
    return u[sel].astype(F64), v[sel].astype(F64), disp[sel]


def _Y(u, v, psi):
    y = v * math.cos(psi) - u * math.sin(psi)
    return np.stack([np.ones_like(y), y], axis=1)


def alpha(u, v, d, psi):
    """Eq. (21): alpha(psi) = (Y'Y)^-1 Y' d."""
    Y = _Y(u, v, psi)
    return np.linalg.solve(Y.T @ Y, Y.T @ d)


def energy(u, v, d, psi):
    """Eq. (23): E_min(psi) = d'd - d'Y (Y'Y)^-1 Y'd."""
    Y = _Y(u, v, psi)
    b = Y.T @ d
    return float(d @ d - b @ np.linalg.solve(Y.T @ Y, b))


def gradient(u, v, d, psi):
    """Eq. (26) through the residual: -2 alpha_1 sum_i r_i y'_i(psi)."""
    a = alpha(u, v, d, psi)
    y = v * math.cos(psi) - u * math.sin(psi)
    yp = -v * math.sin(psi) - u * math.cos(psi)
    r = d - a[0] - a[1] * y
    return float(-2.0 * a[1] * (r @ yp))


def _wrap(psi):
    """Into (-pi/2, pi/2]."""
    w = math.fmod(psi + math.pi / 2.0, math.pi)
    if w <= 0.0:
        w += math.pi
    return w - math.pi / 2.0


def fit_roll(u, v, d, width, height, psi0=0.0, lambda0=LAMBDA0,
             delta_psi=DELTA_PSI, max_iter=100):
    """Roll angle by Eq. (25) with the adaptive rate of Eq. (28)."""
    if len(d) < 3:          # too few points to fit a line: nothing to estimate
        a0 = float(np.mean(d)) if len(d) else 0.0
        return RoadFit(psi0, a0, 0.0, 0.0, 0, True, True)
    a_init = alpha(u, v, d, psi0)
    s = float(max(width, height))
    flat = abs(a_init[1]) < 1e-6
    a1s = 1.0 if flat else a_init[1]
    scale = 1.0 / (len(d) * s * s * a1s * a1s)
    if flat:
        a = a_init
        return RoadFit(psi0, float(a[0]), float(a[1]), energy(u, v, d, psi0),
                       0, True, True)

    def En(psi):
        return energy(u, v, d, psi) * scale

    def Gn(psi):
        return gradient(u, v, d, psi) * scale

    psi, lam = psi0, lambda0
    E, g = En(psi), Gn(psi)
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        step = -lam * g
        for _ in range(64):
            if abs(step) <= math.pi / 4.0 and En(_wrap(psi + step)) <= E * (1.0 + 1e-9):
                break
            lam *= 0.5
            step = -lam * g
        psi_new = _wrap(psi + step)
        g_new = Gn(psi_new)
        done = abs(step) < delta_psi
        if g_new == g:
            psi, E, g = psi_new, En(psi_new), g_new
            converged = True
            break
        lam = lam * g / (g - g_new)            # Eq. (28)
        if not (lam > 0.0 and math.isfinite(lam)):
            lam = lambda0
        psi, E, g = psi_new, En(psi_new), g_new
        if done:
            converged = True
            break
    a = alpha(u, v, d, psi)
    return RoadFit(psi, float(a[0]), float(a[1]), energy(u, v, d, psi), it,
                   converged, False)


def transform(disp, fit: RoadFit, delta_t=0.0):
    """Eq. (29): l' = l - a0 + a1 (u sin psi - v cos psi) + delta_t."""
    disp = np.asarray(disp, F64)
    H, W = disp.shape
    v, u = np.mgrid[0:H, 0:W]
    return (disp - fit.alpha0
            + fit.alpha1 * (u * math.sin(fit.psi) - v * math.cos(fit.psi))
            + delta_t)


def plane_from_fit(fit: RoadFit):
    """The road model of the fit, d = a0 + a1 (v cos psi - u sin psi), as the
    plane c = (c0, c1, c2) of d_road = c0 + c1 u + c2 v (Sec. 3.1 / 3.3)."""
    return (fit.alpha0, -fit.alpha1 * math.sin(fit.psi), fit.alpha1 * math.cos(fit.psi))


def damage_mask(disp_t, delta_t=0.0, tau=0.5):
    """Damage on the transformed map (Sec. 4.4.3): after Eq. (29) the road is
    flat at delta_t and potholes / cracks (farther away, smaller disparity)
    lie below it.  A pixel is damage when its finite transformed disparity is
    more than tau below delta_t.  The comparison is taken in FP32 (a float
    decides a boolean; the kernel's precision), with delta_t - tau rounded to
    FP32 once."""
    d = np.asarray(disp_t, np.float32)
    level = np.float32(np.float32(delta_t) - np.float32(tau))
    with np.errstate(invalid="ignore"):
        return np.isfinite(d) & (d < level)


def road_transform(disp, valid=None, mask=None, psi0=0.0, lambda0=LAMBDA0,
                   delta_psi=DELTA_PSI, max_iter=100, delta_t=0.0):
    H, W = np.shape(disp)
    u, v, d = road_points(disp, valid, mask)
    fit = fit_roll(u, v, d, W, H, psi0, lambda0, delta_psi, max_iter)
    return fit, transform(disp, fit, delta_t)
