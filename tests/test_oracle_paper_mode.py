"""Pins of the oracle's paper-mode hits (Sec. V, Local Maxima and Centroiding:
Eqs. 6-7 and Eq. 9 evaluated on A itself): the worked example's printed
numbers, the dense matrix formulation of tests/bruteforce.py on random tiny
inputs, the tie-break, and closed-form cases."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import bruteforce as bf
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_worked_example(orc):
    """The paper's five pixels on x with r = 5 (Sec. V): local maxima are
    pixels 2 and 3 (1-based) and their rows give 7000 / 350 and 29300 / 325."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_example.json")))
    x = np.array(g["X"])
    tot = np.array(g["ToT"])
    n = x.size
    h = orc.local_maxima(x, np.zeros(n), tot, np.zeros(n), np.full(n, 5000), np.array([0]),
                         dxy=g["radius"], dt_ticks=0)
    assert list(h["label"] + 1) == g["local_maxima_1based"]
    for k, (num, den) in enumerate(zip(g["centroid_num"], g["centroid_den"])):
        assert h["x"][k] == num / den
        assert h["tot_sum"][k] == den
    assert list(h["npix"]) == [3, 2]


def _dense(x, y, tot, shot, toa, trig, r, dt):
    """Local maxima and row centroids from the dense formulation (Eqs. 3-7, 9),
    on inputs whose ToT values are distinct (no tie-break needed)."""
    t = np.asarray(toa, np.int64) - int(np.min(toa))
    A = bf.adjacency(x, y, t, shot, r, dt)
    _, _, maxima = bf.local_maxima(tot, A)
    tof = np.asarray(toa, np.int64) - np.asarray(trig, np.int64)[np.asarray(shot, np.int64)]
    rows = bf.centroid_rows(x, y, tof, tot, A)
    order = sorted(maxima, key=lambda i: (shot[i], i))
    return order, rows, A


@pytest.mark.parametrize("seed", range(40))
def test_matches_dense_formulation(orc, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 90))
    ev = synth.tiny_events(rng, n, grid=int(rng.integers(2, 9)), t_span=int(rng.integers(0, 600)),
                           n_shots=int(rng.integers(1, 4)), sort_by_shot=bool(seed % 2))
    tot = rng.permutation(np.arange(1, n + 1) * 3).astype(np.uint16)  # distinct
    trig = np.zeros(int(ev["shot"].max()) + 1, np.uint64)
    r = int(rng.integers(0, 3))
    dt = int(rng.choice([0, 64, 128, 400]))
    order, rows, A = _dense(ev["x"], ev["y"], tot, ev["shot"], ev["toa"], trig, r, dt)
    h = orc.local_maxima(ev["x"], ev["y"], tot, ev["shot"], ev["toa"], trig, dxy=r, dt_ticks=dt)
    assert list(h["label"]) == [int(i) for i in order]
    for k, i in enumerate(order):
        cx, cy, ct, flagged = rows[i]
        assert abs(h["x"][k] - float(cx)) <= 1e-12
        assert abs(h["y"][k] - float(cy)) <= 1e-12
        assert abs(h["tof_ns"][k] - 1.5625 * float(ct)) <= 1e-6
        assert h["npix"][k] == int(A[i].sum())
        assert h["tot_sum"][k] == int(A[i] @ tot.astype(np.int64))


def test_ties_break_by_index(orc):
    """Equal ToT on two neighbours: only the later index is a maximum (the
    paper's +0.001 i), and its row holds both pixels."""
    x = np.array([10, 11, 40])
    y = np.array([5, 5, 5])
    tot = np.array([100, 100, 7])
    h = orc.local_maxima(x, y, tot, np.zeros(3), np.array([10, 20, 30]), np.array([0]))
    assert list(h["label"]) == [1, 2]
    assert h["x"][0] == 10.5 and h["npix"][0] == 2
    assert h["x"][1] == 40.0 and h["npix"][1] == 1


def test_closed_forms(orc):
    """A plus-shaped spot (centre brightest, four equal arms) gives exactly
    its centre; an isolated pixel is its own hit; a pixel out of time (> r_t)
    is not a neighbour; the row of a maximum is its direct neighbourhood only
    (a chain of three along x yields the middle pixel's row, not the chain)."""
    x = np.array([50, 49, 51, 50, 50, 200])
    y = np.array([60, 60, 60, 59, 61, 10])
    tot = np.array([400, 90, 90, 90, 90, 3])
    toa = np.array([1000, 1010, 1020, 1005, 1015, 1000])
    h = orc.local_maxima(x, y, tot, np.zeros(6), toa, np.array([0]))
    assert list(h["label"]) == [0, 5]
    assert (h["x"][0], h["y"][0]) == (50.0, 60.0) and h["npix"][0] == 5
    assert (h["x"][1], h["y"][1], h["npix"][1]) == (200.0, 10.0, 1)
    # time: the right arm 200 ticks late is no neighbour and becomes a hit
    toa2 = toa.copy()
    toa2[2] = 1000 + 200
    h2 = orc.local_maxima(x, y, tot, np.zeros(6), toa2, np.array([0]))
    assert list(h2["label"]) == [0, 2, 5]
    assert h2["npix"][0] == 4
    # a chain 1-2-3 with the middle brightest: one hit over all three; with the
    # left end brightest, the left end's row is only itself and the middle
    xs = np.array([10, 11, 12])
    h3 = orc.local_maxima(xs, np.zeros(3), np.array([5, 9, 5]), np.zeros(3), np.zeros(3),
                          np.array([0]))
    assert list(h3["label"]) == [1] and h3["npix"][0] == 3
    h4 = orc.local_maxima(xs, np.zeros(3), np.array([9, 5, 7]), np.zeros(3), np.zeros(3),
                          np.array([0]))
    assert list(h4["label"]) == [0, 2]
    # FP64 division of exact integer moments: the correctly rounded quotient
    assert h4["x"][0] == float(Fraction(9 * 10 + 5 * 11, 14)) and h4["npix"][0] == 2
    assert h4["x"][1] == float(Fraction(5 * 11 + 7 * 12, 12)) and h4["npix"][1] == 2


def test_zero_tot_row_is_plain_mean(orc):
    h = orc.local_maxima(np.array([3, 4]), np.array([0, 0]), np.array([0, 0]), np.zeros(2),
                         np.array([7, 7]), np.array([0]))
    assert list(h["label"]) == [1] and h["flags"][0] == 1 and h["x"][0] == 3.5
