"""Seeded single clusters with known truth, for training and evaluating a
learned centroider / multiplicity splitter.

Each sample is one cluster: one particle hit, or (with probability
`pair_frac`) two overlapping hits, rendered with the same detector model as
the stream workloads (Gaussian spot, pixels kept at amplitude >= 5 % of peak,
ToT = rint(scale * summed amplitude), ToA = earliest contributing hit time +
20 ns * (1 - amplitude) + N(0, 1.5 ns) jitter, in 1.5625 ns ticks).  Every
sample is its own shot with its trigger at tick 0, so ToA is also ToF.

The module fabricates inputs only: it returns the pixel events of every
sample (contiguous, sample by sample), the index of each sample's first event
(the grouping the generator made, used as the cluster label), and the truth
(hit positions in pixel units with pixel centres at integer coordinates, hit
times in ns, multiplicity).
"""
from __future__ import annotations

import math

import numpy as np

from .vmi import AMP_KEEP, GRID, TICK_NS


def _render(rng, n, pair_frac, sigma, tot_scale, sep_px, pair_dt_ns, t_window_ns, walk_ns,
            jitter_ns):
    mult = np.where(rng.random(n) < pair_frac, 2, 1).astype(np.uint8)
    # hit A anywhere on the grid away from the edges, hit B at a random offset
    ax = 16.0 + rng.random(n) * (GRID - 32.0)
    ay = 16.0 + rng.random(n) * (GRID - 32.0)
    at = rng.random(n) * t_window_ns
    asg = sigma[0] + (sigma[1] - sigma[0]) * rng.random(n)
    sep = sep_px[0] + (sep_px[1] - sep_px[0]) * rng.random(n)
    phi = rng.random(n) * 2.0 * math.pi
    bx = ax + sep * np.cos(phi)
    by = ay + sep * np.sin(phi)
    bt = at + pair_dt_ns[0] + (pair_dt_ns[1] - pair_dt_ns[0]) * rng.random(n)
    bsg = sigma[0] + (sigma[1] - sigma[0]) * rng.random(n)
    pair = mult == 2

    # render both spots on one box per sample (A's box widened by the largest
    # separation), summing the light of the spots that reach 5 % of their peak
    R = int(math.ceil(sigma[1] * math.sqrt(2.0 * math.log(1.0 / AMP_KEEP))))
    M = int(math.ceil(sep_px[1]))
    offs = np.arange(-R - M, R + M + 2)
    ox, oy = np.meshgrid(offs, offs, indexing="ij")
    px = np.floor(ax).astype(np.int64)[:, None] + ox.ravel()[None, :]
    py = np.floor(ay).astype(np.int64)[:, None] + oy.ravel()[None, :]
    cut = 2.0 * math.log(1.0 / AMP_KEEP)
    da = ((px - ax[:, None]) ** 2 + (py - ay[:, None]) ** 2) / asg[:, None] ** 2
    db = ((px - bx[:, None]) ** 2 + (py - by[:, None]) ** 2) / bsg[:, None] ** 2
    a_on = da <= cut
    b_on = (db <= cut) & pair[:, None]
    keep = a_on | b_on
    sample = np.nonzero(keep)[0]
    a_on, b_on = a_on[keep], b_on[keep]
    amp_sum = np.where(a_on, np.exp(-0.5 * da[keep]), 0.0) + \
        np.where(b_on, np.exp(-0.5 * db[keep]), 0.0)
    t_first = np.where(a_on & b_on, np.minimum(at, bt)[sample],
                       np.where(a_on, at[sample], bt[sample]))
    ex, ey = px[keep], py[keep]
    tot = np.clip(np.rint(tot_scale * amp_sum), 1, 1023).astype(np.uint16)
    t_ns = t_first + walk_ns * (1.0 - np.minimum(amp_sum, 1.0)) + rng.normal(0.0, jitter_ns,
                                                                             sample.size)
    toa = np.maximum(0, np.rint(t_ns / TICK_NS)).astype(np.uint64)
    truth = np.zeros((n, 2, 3), np.float64)
    truth[:, 0] = np.stack([ax, ay, at], 1)
    truth[:, 1] = np.stack([bx, by, bt], 1)
    truth[~pair, 1] = truth[~pair, 0]
    return ex, ey, tot, toa, sample, truth, mult


def make_clusters(seed, n, pair_frac=0.3, sigma=(0.5, 2.5), tot_scale=400.0,
                  sep_px=(0.5, 3.0), pair_dt_ns=(0.0, 50.0), t_window_ns=10_000.0,
                  walk_ns=20.0, jitter_ns=1.5, block=4000, first_block=0):
    """n samples in blocks of `block`; block b draws from PCG64 seeded with
    (seed, b), so any range of blocks can be generated on its own (and in
    parallel) with the same result."""
    parts = []
    for k, lo in enumerate(range(0, n, block)):
        m = min(block, n - lo)
        rng = np.random.default_rng([seed, first_block + k])
        ex, ey, tot, toa, sample, truth, mult = _render(rng, m, pair_frac, sigma, tot_scale,
                                                         sep_px, pair_dt_ns, t_window_ns,
                                                         walk_ns, jitter_ns)
        parts.append((ex.astype(np.uint16), ey.astype(np.uint16), tot, toa,
                      (sample + lo).astype(np.uint32), truth, mult))
    cat = [np.concatenate([p[k] for p in parts]) for k in range(7)]
    x, y, tot, toa, shot, truth, mult = cat
    counts = np.bincount(shot, minlength=n)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    ev = dict(x=x, y=y, tot=tot, shot=shot, toa=toa)
    return dict(events=ev, labels=start[shot].astype(np.uint32), first=start, counts=counts,
                truth=truth, mult=mult, n=n)


MLP_SHAPES = [((256, 98), 98), ((256,), 0), ((256, 256), 256), ((256,), 0), ((8, 256), 256),
              ((8,), 0)]


def init_mlp_params(seed, zero_last=False):
    """Initial parameters of the 98 -> 256 -> 256 -> 8 network, packed
    W1, b1, W2, b2, W3, b3 with W as [out][in]: He-uniform weights
    (U(-sqrt(6 / fan_in), +sqrt(6 / fan_in))), zero biases, from PCG64(seed),
    as float32; zero_last leaves the output layer at zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (shape, fan_in) in enumerate(MLP_SHAPES):
        if fan_in and zero_last and k == 4:
            rng.uniform(-1, 1, shape)
            parts.append(np.zeros(shape).ravel())
        elif fan_in:
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts).astype(np.float32)
