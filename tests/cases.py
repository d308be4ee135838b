"""Seeded test inputs shared by the GPU parity tests and the host-emulation
tests (inputs only; no processing)."""
import numpy as np

import synth


def tiny_cluster_case(seed):
    """The random event-mode clustering case of a seed: events on a small
    grid with frequent neighbours, repeats and shot boundaries, a radius and a
    time window."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 300))
    ev = synth.tiny_events(rng, n, grid=int(rng.integers(2, 12)), t_span=int(rng.integers(0, 800)),
                           n_shots=int(rng.integers(1, 5)), sort_by_shot=bool(seed % 2))
    dxy = int(rng.integers(0, 4))
    dt = int(rng.choice([0, 1, 64, 128, 500]))
    return ev, dxy, dt


def many_components_packets(n_iso):
    """One shot whose pixels are all isolated (spacing 2 on the grid, so no
    two are neighbours) plus one 3x3 blob, as packets: n_iso = 1500 gives more
    components in one segment than LDS accumulators hold, 3000 a segment
    beyond the LDS event capacity, 20000 one shot spanning many strides."""
    rng = np.random.default_rng(n_iso)
    trig = np.array([1_000_000, 1_000_000 + synth.SHOT_PERIOD_TICKS])
    k = np.arange(n_iso)
    x = 2 * (k % 128)
    y = 2 * ((k // 128) % 128)
    t = trig[0] + 100 + (k // 16384) * 1000 + rng.integers(0, 50_000, n_iso)
    bx, by = np.meshgrid(np.arange(3) + 1, np.arange(3) + 1)
    x = np.concatenate([x, bx.ravel()])
    y = np.concatenate([y, by.ravel()])
    t = np.concatenate([t, np.full(9, trig[0] + 60_000)])
    tot = rng.integers(0, 400, x.size)
    tot[:5] = 0
    order = np.argsort(t, kind="stable")
    return np.concatenate([synth.encode_tdc(trig[:1], [0]),
                           synth.encode_pixels(x[order], y[order], tot[order], t[order]),
                           synth.encode_tdc(trig[1:], [1])])


def big_component_packets(side=136, layers=2):
    """One component of side^2 * layers pixels: a square at ToT 1023 with x
    and y up to 255, fired `layers` times 50 ticks apart (the default gives
    36,992 pixels whose sum of ToT * x exceeds 32 bits)."""
    trig = np.array([1_000_000, 1_000_000 + synth.SHOT_PERIOD_TICKS])
    bx, by = np.meshgrid(np.arange(256 - side, 256), np.arange(256 - side, 256))
    x = np.tile(bx.ravel(), layers)
    y = np.tile(by.ravel(), layers)
    t = np.repeat(trig[0] + 1000 + 50 * np.arange(layers), bx.size)
    tot = np.full(x.size, 1023)
    return np.concatenate([synth.encode_tdc(trig[:1], [0]),
                           synth.encode_pixels(x, y, tot, t),
                           synth.encode_tdc(trig[1:], [1])])


def shuffled_shapes_packets(seed, width=40):
    """One shot of connected shapes whose pixels arrive in a random order, so
    that the smallest-neighbour forest of each shape has many local minima
    and trees must be joined many times over: a serpentine path one pixel
    wide (every other row of a width x width box, joined at alternating
    ends), a filled 20 x 20 square, a ring, and a few isolated pixels; times
    spread over 100 ticks (every pair of neighbours within the window)."""
    rng = np.random.default_rng(5000 + seed)
    trig = np.array([1_000_000, 1_000_000 + synth.SHOT_PERIOD_TICKS])
    pts = []
    for r in range(0, width, 2):  # serpentine
        pts += [(10 + c, 10 + r) for c in range(width)]
        if r + 2 < width:
            pts.append((10 + (width - 1 if (r // 2) % 2 == 0 else 0), 10 + r + 1))
    pts += [(100 + c, 100 + r) for r in range(20) for c in range(20)]  # square
    for a in range(0, 360, 3):  # ring of radius 15
        p = (200 + int(round(15 * np.cos(np.radians(a)))), 60 + int(round(15 * np.sin(np.radians(a)))))
        if p not in pts:
            pts.append(p)
    pts += [(2 * k, 250) for k in range(20)]  # isolated
    xy = np.array(pts)
    order = rng.permutation(len(xy))
    x, y = xy[order, 0], xy[order, 1]
    t = trig[0] + 1000 + rng.integers(0, 100, x.size)
    tot = rng.integers(1, 600, x.size)
    return np.concatenate([synth.encode_tdc(trig[:1], [0]),
                           synth.encode_pixels(x, y, tot, t),
                           synth.encode_tdc(trig[1:], [1])])
