"""Properties the centroiding of Sec. V must have, checked on the oracle:
conservation of ToT and pixel count, exact centres of symmetric spots,
translation and permutation invariance, one-to-one recovery of isolated hits,
and agreement with a textbook connected-component labelling (scipy) when time
plays no role."""
import numpy as np
import pytest
from scipy import ndimage

import synth


def _run_events(orc, ev, dxy=1, dt=128):
    lab, nc = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"], dxy=dxy, dt_ticks=dt)
    h = orc.centroid(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], lab, ev["trig"])
    return lab, h


def test_conservation_c1(orc):
    w = synth.make_config("c1", n_shots=300)
    r = orc.process(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ev, h = r["events"], r["hits"]
    assert int(h["npix"].sum()) == ev["x"].size
    assert int(h["tot_sum"].sum()) == int(ev["tot"].astype(np.int64).sum())
    # every hit lies inside the bounding box of its pixels
    lab = r["labels"]
    for hh in h[:200]:
        m = lab == hh["label"]
        assert ev["x"][m].min() <= hh["x"] <= ev["x"][m].max()
        assert ev["y"][m].min() <= hh["y"] <= ev["y"][m].max()
    s = r["stats"]
    assert s["n_pixels"] == s["n_pre_trigger"] + s["n_tof_cut"] + s["n_events"]
    assert s["n_packets"] == s["n_pixels"] + s["n_tdc"] + s["n_other"]


def _spot(x0, y0, t0, weights):
    """Pixels around (x0, y0) with ToT given by a dict {(dx, dy): tot}."""
    xs, ys, tots = [], [], []
    for (dx, dy), w in weights.items():
        xs.append(x0 + dx)
        ys.append(y0 + dy)
        tots.append(w)
    n = len(xs)
    return dict(x=np.array(xs, np.uint16), y=np.array(ys, np.uint16),
                tot=np.array(tots, np.uint16), shot=np.zeros(n, np.uint32),
                toa=np.full(n, t0, np.uint64), trig=np.array([t0 - 640], np.uint64))


def test_symmetric_spot_is_centred_exactly(orc):
    w = {(0, 0): 400, (1, 0): 120, (-1, 0): 120, (0, 1): 120, (0, -1): 120,
         (1, 1): 37, (1, -1): 37, (-1, 1): 37, (-1, -1): 37, (2, 0): 5, (-2, 0): 5,
         (0, 2): 5, (0, -2): 5}
    _, h = _run_events(orc, _spot(100, 57, 10_000, w))
    assert h.size == 1
    assert h["x"][0] == 100.0 and h["y"][0] == 57.0
    assert h["tof_ns"][0] == 640 * 1.5625


def test_two_by_two_block_is_half_pixel(orc):
    _, h = _run_events(orc, _spot(10, 20, 5000, {(0, 0): 9, (1, 0): 9, (0, 1): 9, (1, 1): 9}))
    assert h["x"][0] == 10.5 and h["y"][0] == 20.5


def test_symmetric_times_give_exact_mean(orc):
    ev = _spot(10, 20, 5000, {(0, 0): 7, (1, 0): 7})
    ev["toa"] = np.array([5000 - 4, 5000 + 4], np.uint64)
    _, h = _run_events(orc, ev)
    assert h["tof_ns"][0] == 640 * 1.5625


def test_translation_invariance(orc):
    rng = np.random.default_rng(7)
    ev = synth.tiny_events(rng, 60, grid=12, t_span=500, n_shots=3)
    lab, h = _run_events(orc, ev)
    ev2 = dict(ev)
    ev2["x"] = (ev["x"] + 37).astype(np.uint16)
    ev2["y"] = (ev["y"] + 101).astype(np.uint16)
    ev2["toa"] = ev["toa"] + np.uint64(123_456)
    ev2["trig"] = ev["trig"] + np.uint64(123_456)
    lab2, h2 = _run_events(orc, ev2)
    assert np.array_equal(lab, lab2)
    # integer moments shift exactly; only the final division rounds
    assert np.allclose(h2["x"] - 37, h["x"], rtol=0, atol=1e-12)
    assert np.allclose(h2["y"] - 101, h["y"], rtol=0, atol=1e-12)
    assert np.array_equal(h2["tof_ns"], h["tof_ns"])
    assert np.array_equal(h2["tot_sum"], h["tot_sum"]) and np.array_equal(h2["npix"], h["npix"])
    assert np.array_equal(h2["toa_first"] - 123_456, h["toa_first"])


def test_permutation_invariance(orc):
    rng = np.random.default_rng(11)
    ev = synth.tiny_events(rng, 80, grid=10, t_span=500, n_shots=2, sort_by_shot=False)
    lab, _ = _run_events(orc, ev)
    perm = rng.permutation(ev["x"].size)
    evp = {k: (v[perm] if k != "trig" else v) for k, v in ev.items()}
    labp, _ = _run_events(orc, evp)
    # same partition: i ~ j before  <=>  perm^-1(i) ~ perm^-1(j) after
    a = lab[perm]
    b = labp
    pairs = {}
    for u, v in zip(a.tolist(), b.tolist()):
        assert pairs.setdefault(u, v) == v
    assert len(set(pairs.values())) == len(pairs)
    # and labels are the smallest member index
    for v in set(b.tolist()):
        assert v == np.nonzero(b == v)[0].min()


def test_isolated_planted_hits_recovered_one_to_one(orc):
    """Hits separated by more than the spot size plus the radius, or in time
    by more than the window plus the time-walk span, come back as one hit
    each, with exactly their own pixels."""
    rng = np.random.default_rng(3)
    xs, ys, tots, toas, hid = [], [], [], [], []
    k = 0
    for gx in range(6, 250, 12):
        for gy in range(6, 250, 24):
            cx, cy = gx + rng.random(), gy + rng.random()
            t0 = 20_000 + int(rng.integers(0, 6000))
            for dx in range(-3, 5):
                for dy in range(-3, 5):
                    px, py = int(np.floor(cx)) + dx, int(np.floor(cy)) + dy
                    a = np.exp(-((px - cx) ** 2 + (py - cy) ** 2) / (2 * 0.8 ** 2))
                    if a >= 0.05:
                        xs.append(px); ys.append(py); tots.append(int(round(400 * a)))
                        toas.append(t0 + int(round(12.8 * (1 - a))))
                        hid.append(k)
            k += 1
    perm = rng.permutation(len(xs))
    ev = dict(x=np.array(xs, np.uint16)[perm], y=np.array(ys, np.uint16)[perm],
              tot=np.array(tots, np.uint16)[perm], toa=np.array(toas, np.uint64)[perm],
              shot=np.zeros(len(xs), np.uint32), trig=np.array([0], np.uint64))
    hid = np.array(hid)[perm]
    lab, h = _run_events(orc, ev)
    assert h.size == k
    for lv in np.unique(lab):
        assert np.unique(hid[lab == lv]).size == 1
    for hv in range(k):
        assert np.unique(lab[hid == hv]).size == 1


@pytest.mark.parametrize("seed", range(5))
def test_single_time_slab_matches_scipy_label(orc, seed):
    """All ToA equal and addresses unique: the partition is plain 8-connected
    labelling of the occupancy image."""
    rng = np.random.default_rng(seed)
    img = rng.random((40, 40)) < 0.45
    ys, xs = np.nonzero(img)
    perm = rng.permutation(xs.size)
    xs, ys = xs[perm], ys[perm]
    n = xs.size
    lab, nc = orc.cluster(xs.astype(np.uint16), ys.astype(np.uint16), np.zeros(n, np.uint32),
                          np.full(n, 777, np.uint64))
    ref, nref = ndimage.label(img, structure=np.ones((3, 3)))
    assert nc == nref
    refl = ref[ys, xs]
    m = {}
    for a, b in zip(lab.tolist(), refl.tolist()):
        assert m.setdefault(b, a) == a
    assert len(set(m.values())) == len(m)


def test_walk_table_is_subtracted_per_pixel(orc):
    """Eq. (1) maps measured to true ToF: each pixel's ToF loses
    Delta ToF(ToT) before the ToT-weighted mean."""
    walk = np.zeros(1024)
    walk[10] = 3.0
    walk[30] = 7.5
    ev = _spot(5, 5, 10_000, {(0, 0): 10, (1, 0): 30})
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    h = orc.centroid(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], lab, ev["trig"],
                     walk_ns=walk)
    expect = (10 * (640 * 1.5625 - 3.0) + 30 * (640 * 1.5625 - 7.5)) / 40
    assert h["tof_ns"][0] == expect
    h0 = orc.centroid(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], lab, ev["trig"])
    assert h0["tof_ns"][0] == 640 * 1.5625
