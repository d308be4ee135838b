"""Oracle of the walk calibration (Sec. IV, ToT-ToF Correlation Correction,
Eq. 1).  TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's
reference leg call it; the library never imports it.  Plain numpy / scipy in
float64, following the paper's steps in its order:

1. select one ion peak: the pixels whose ToF (ToA - trigger of their shot)
   lies in a narrow window [tof_lo, tof_hi] (ticks, inclusive);
2. for every ToT value of the slice, the centre of its ToF distribution.  The
   paper fits a Gaussian to each ToT slice; the centre is read here as the
   Gaussian's maximum-likelihood centre, i.e. the mean ToF of the slice's
   pixels of that ToT (ns);
3. fit Eq. (1), <ToF>(ToT) = a / (ToT + b)^d + c, by least squares over the
   pixels of the slice: the residual of a pixel is its ToF minus the model, so
   each ToT value enters with weight = its pixel count (the within-value
   scatter does not depend on the parameters).  ToT values with fewer than
   `min_count` pixels are left out;
4. the correction applied to every pixel is the ToT-dependent part,
   walk(ToT) = a / (ToT + b)^d (true ToF = measured - walk); c is the ToF of
   the selected peak.
"""
from __future__ import annotations

import numpy as np

TICK_NS = 1.5625


def slice_centres(tot, tof_ticks, tof_lo, tof_hi):
    """Per ToT value 0..1023 of the pixels with tof_lo <= ToF <= tof_hi: the
    pixel count and the mean ToF in ns (NaN where there is none)."""
    tot = np.asarray(tot, np.int64)
    tof = np.asarray(tof_ticks, np.int64)
    sel = (tof >= tof_lo) & (tof <= tof_hi)
    n = np.bincount(tot[sel], minlength=1024)[:1024].astype(np.int64)
    s = np.bincount(tot[sel], weights=tof[sel].astype(np.float64), minlength=1024)[:1024]
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(n > 0, s / np.maximum(n, 1) * TICK_NS, np.nan)
    return n, mean


def model(t, a, b, d, c):
    """Eq. (1)."""
    return a / np.power(np.asarray(t, np.float64) + b, d) + c


def fit_centres(t, mean, count, x0=None):
    """Least-squares fit of Eq. (1) to centres `mean` at ToT values `t` with
    weights `count`; returns (a, b, c, d)."""
    from scipy.optimize import least_squares

    t = np.asarray(t, np.float64)
    mean = np.asarray(mean, np.float64)
    w = np.sqrt(np.asarray(count, np.float64))
    if x0 is None:
        x0 = initial_guess(t, mean)
    a0, b0, c0, d0 = x0

    def res(p):
        a, b, d, c = p
        return w * (model(t, a, b, d, c) - mean)

    lo = np.array([-np.inf, -t.min() + 1e-6, 0.05, -np.inf])
    hi = np.array([np.inf, np.inf, 8.0, np.inf])
    r = least_squares(res, np.array([a0, max(b0, lo[1] + 1e-3), d0, c0]), bounds=(lo, hi),
                      method="trf", x_scale="jac", xtol=1e-14, ftol=1e-14, gtol=1e-14,
                      max_nfev=20000)
    a, b, d, c = r.x
    return float(a), float(b), float(c), float(d)


def initial_guess(t, mean):
    """Start of the fit: d = 1, b = 1, c from the brightest fifth of the ToT
    values, a from the dimmest one."""
    order = np.argsort(t)
    t, mean = np.asarray(t, np.float64)[order], np.asarray(mean, np.float64)[order]
    k = max(1, t.size // 5)
    c0 = float(np.mean(mean[-k:]))
    b0 = 1.0
    a0 = float((mean[0] - c0) * (t[0] + b0))
    return a0, b0, c0, 1.0


def walk_fit(ev, trig, tof_lo, tof_hi, min_count=20):
    """Steps 1-3 on decoded events (x, y, tot, shot, toa) and trigger times:
    dict(params=(a, b, c, d), count, mean)."""
    tof = np.asarray(ev["toa"], np.int64) - np.asarray(trig, np.int64)[np.asarray(ev["shot"], np.int64)]
    n, mean = slice_centres(ev["tot"], tof, tof_lo, tof_hi)
    use = np.nonzero(n >= min_count)[0]
    if use.size < 4:
        raise ValueError("fewer than 4 ToT values with enough pixels")
    p = fit_centres(use, mean[use], n[use])
    return dict(params=p, count=n, mean=mean)


def walk_table(params):
    """Step 4: walk(ToT) = a / (ToT + b)^d for ToT = 0..1023 (ns); ToT
    values at or below -b take the value of the smallest ToT above it."""
    a, b, c, d = params
    t = np.arange(1024, dtype=np.float64)
    ok = t + b > 0
    out = np.empty(1024)
    out[ok] = a / np.power(t[ok] + b, d)
    if not ok.all():
        out[~ok] = out[ok][0] if ok.any() else 0.0
    return out
