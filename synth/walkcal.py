"""Seeded calibration runs for the time-walk correction (inputs only).

A calibration run holds hits of one ion species, all arriving at the same true
time of flight after their shot's trigger.  Each hit is a Gaussian spot on the
pixel grid (sigma U(0.6, 1.5) px); a pixel's ToT is rint(scale * amplitude),
clipped to 1..1023, and it reports the ion's arrival later by a walk that
depends on its ToT through the paper's calibration model (Sec. IV, ToT-ToF
Correlation Correction, Eq. 1), a / (ToT + b)^d + c, plus Gaussian jitter.
The module only fabricates these events (event arrays and trigger times); it
fits nothing.
"""
from __future__ import annotations

import numpy as np

from .vmi import SHOT_PERIOD_TICKS, TICK_NS

# default walk model of a run, in ns: about 22 ns of walk at ToT 10 falling
# towards 1.6 ns at ToT 1023 (a / (ToT + b)^d + c)
WALK_DEFAULT = dict(a=300.0, b=4.0, d=1.05, c=1.2)


def walk_ns(tot, a, b, d, c):
    """The generator's walk in ns of pixels of the given ToT."""
    return a / np.power(np.asarray(tot, np.float64) + b, d) + c


def calibration_run(seed, n_hits, tof0_ns=5000.0, walk=None, jitter_ns=1.5, tot_scale=(150, 900),
                    hits_per_shot=10):
    """Events of `n_hits` single-ion hits of one species at true ToF
    `tof0_ns`.  Returns (events dict x, y, tot, shot, toa in ticks, trigger
    times in ticks)."""
    walk = dict(WALK_DEFAULT if walk is None else walk)
    rng = np.random.default_rng(seed)
    n_shots = max(1, -(-n_hits // hits_per_shot))
    trig = (10_000_000 + SHOT_PERIOD_TICKS * np.arange(n_shots)).astype(np.int64)
    shot = np.arange(n_hits) // hits_per_shot
    cx = rng.uniform(16, 240, n_hits)
    cy = rng.uniform(16, 240, n_hits)
    sig = rng.uniform(0.6, 1.5, n_hits)
    scale = rng.uniform(*tot_scale, n_hits)
    xs, ys, tots, shots = [], [], [], []
    for dx in range(-5, 6):
        for dy in range(-5, 6):
            px = np.floor(cx).astype(np.int64) + dx
            py = np.floor(cy).astype(np.int64) + dy
            amp = np.exp(-((px - cx) ** 2 + (py - cy) ** 2) / (2 * sig ** 2))
            keep = amp >= 0.05
            t = np.clip(np.rint(scale * amp), 1, 1023).astype(np.int64)
            xs.append(px[keep])
            ys.append(py[keep])
            tots.append(t[keep])
            shots.append(shot[keep])
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    tot = np.concatenate(tots)
    sh = np.concatenate(shots)
    t_ns = tof0_ns + walk_ns(tot, **walk) + rng.normal(0.0, jitter_ns, tot.size)
    toa = trig[sh] + np.rint(t_ns / TICK_NS).astype(np.int64)
    order = np.lexsort((toa, sh))
    ev = dict(x=x[order].astype(np.uint16), y=y[order].astype(np.uint16),
              tot=tot[order].astype(np.uint16), shot=sh[order].astype(np.uint32),
              toa=toa[order].astype(np.uint64))
    return ev, trig.astype(np.uint64)
