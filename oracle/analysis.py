"""Dose comparison tools for the parity tests (test infrastructure).

* ``gamma_pass_rate``: 3D global gamma index (Low et al. 1998) as used for
  the paper's validation (2%/2mm and 1%/1mm above the 10% isodose, Table 1).
  The paper does not state its gamma variant; this one is global (dose
  criterion relative to the reference maximum), evaluates reference voxels
  at or above the threshold, and searches the trilinearly interpolated
  evaluated dose on a sub-voxel grid of offsets inside the DTA sphere, which
  decides pass/fail (gamma <= 1) exactly up to the search resolution.
* ``zscore_stats``: per-voxel z = (a - b) / sqrt(sa^2 + sb^2) above a dose
  threshold.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage


def gamma_pass_rate(ref, ev, voxel, dose_crit=0.02, dta=0.2,
                    threshold=0.1, step=None, region=None):
    """Fraction of reference voxels (dose >= threshold * max, and inside
    ``region`` if given) with gamma <= 1.  ``voxel`` and ``dta`` in the same
    length unit; arrays (z, y, x)."""
    ref = np.asarray(ref, np.float64)
    g2 = gamma_squared(ref, ev, voxel, dose_crit, dta, step)
    sel = ref >= threshold * ref.max()
    if region is not None:
        sel &= region
    if not sel.any():
        return 1.0
    return float((g2[sel] <= 1.0).mean())


def gamma_squared(ref, ev, voxel, dose_crit=0.02, dta=0.2, step=None):
    """min over the DTA sphere of gamma^2 (values above 1 are only bounds)."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    vz, vy, vx = (voxel,) * 3 if np.isscalar(voxel) else voxel
    dd = dose_crit * ref.max()
    step = step or dta / 5.0
    r = np.arange(-dta, dta + 1e-12, step)
    best = np.full(ref.shape, np.inf)
    for oz in r:
        for oy in r:
            for ox in r:
                d2 = ox * ox + oy * oy + oz * oz
                if d2 > dta * dta + 1e-12:
                    continue
                sh = ndimage.shift(ev, (-oz / vz, -oy / vy, -ox / vx),
                                   order=1, mode="nearest", prefilter=False)
                g2 = d2 / (dta * dta) + ((sh - ref) / dd) ** 2
                np.minimum(best, g2, out=best)
    return best


def zscore_stats(a, sa, b, sb, ref_for_threshold=None, threshold=0.1):
    ref = a if ref_for_threshold is None else ref_for_threshold
    sel = ref >= threshold * ref.max()
    den = np.sqrt(sa[sel] ** 2 + sb[sel] ** 2)
    ok = den > 0
    z = (a[sel][ok] - b[sel][ok]) / den[ok]
    return {"n": int(z.size), "frac_le3": float((np.abs(z) <= 3).mean()),
            "mean": float(z.mean()), "sd": float(z.std()),
            "max_abs": float(np.abs(z).max())}


def time_to_uncertainty(t_run, dose, sigma, target=0.01, level=0.5):
    """T_target = T_run (sigma_bar / target)^2, sigma_bar the mean relative
    batch uncertainty over voxels at or above ``level`` of the maximum."""
    sel = dose >= level * dose.max()
    rel = sigma[sel] / dose[sel]
    s = float(rel.mean())
    return t_run * (s / target) ** 2, s
