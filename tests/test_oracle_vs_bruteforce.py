"""The oracle's clustering and centroids equal the dense formulation of the
paper (Eqs. 3-5 closed transitively, Eq. 9) on many tiny inputs."""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import bruteforce as bf
from synth import tiny_events


def _check(orc, ev, dxy, dt):
    x, y, tot, shot, toa, trig = (ev[k] for k in ("x", "y", "tot", "shot", "toa", "trig"))
    lab, nc = orc.cluster(x, y, shot, toa, dxy=dxy, dt_ticks=dt)
    ref = bf.labels(x.astype(np.int64), y.astype(np.int64), toa.astype(np.int64),
                    shot.astype(np.int64), dxy, dt)
    assert lab.astype(np.int64).tolist() == ref.tolist()
    assert nc == len(set(ref.tolist()))
    hits = orc.centroid(x, y, tot, shot, toa, lab, trig)
    refh = bf.hits(x.astype(np.int64), y.astype(np.int64), tot.astype(np.int64),
                   shot.astype(np.int64), toa.astype(np.int64), trig.astype(np.int64), dxy, dt)
    assert len(hits) == len(refh)
    for h, r in zip(hits, refh):
        assert (int(h["shot"]), int(h["label"]), int(h["npix"]), int(h["tot_sum"]),
                int(h["toa_first"])) == (r["shot"], r["label"], r["npix"], r["tot_sum"],
                                         r["toa_first"])
        assert bool(h["flags"] & 1) == r["flagged"]
        # exact rational reference vs one double division
        assert abs(Fraction(float(h["x"])) - r["x"]) <= abs(r["x"]) * Fraction(1, 2**52)
        assert abs(Fraction(float(h["y"])) - r["y"]) <= abs(r["y"]) * Fraction(1, 2**52)
        tof_ns = r["tof_ticks"] * Fraction(25, 16)
        assert abs(Fraction(float(h["tof_ns"])) - tof_ns) <= abs(tof_ns) * Fraction(1, 2**50)


@pytest.mark.parametrize("seed", range(400))
def test_random_tiny(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 48))
    ev = tiny_events(rng, n, grid=int(rng.integers(2, 9)), t_span=int(rng.integers(0, 600)),
                     n_shots=int(rng.integers(1, 4)), sort_by_shot=bool(rng.integers(0, 2)))
    dxy = int(rng.integers(0, 3))
    dt = int(rng.choice([0, 1, 50, 128, 300]))
    _check(orc, ev, dxy, dt)


@settings(max_examples=300, deadline=None)
@given(st.integers(0, 2**31), st.integers(1, 40), st.integers(2, 7), st.integers(0, 400))
def test_hypothesis_tiny(orc, seed, n, grid, span):
    rng = np.random.default_rng(seed)
    ev = tiny_events(rng, n, grid=grid, t_span=span, n_shots=2, sort_by_shot=False)
    _check(orc, ev, 1, 128)


def _ev(x, y, toa, shot=None, tot=None, trig=(0,)):
    n = len(x)
    return dict(x=np.array(x, np.uint16), y=np.array(y, np.uint16),
                toa=np.array(toa, np.uint64),
                shot=np.zeros(n, np.uint32) if shot is None else np.array(shot, np.uint32),
                tot=np.full(n, 10, np.uint16) if tot is None else np.array(tot, np.uint16),
                trig=np.array(trig, np.uint64))


def test_time_chain_is_transitive(orc):
    # A-B and B-C within 128 ticks, A-C not: one hit
    ev = _ev([5, 5, 5], [5, 5, 5], [0, 128, 256])
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    assert lab.tolist() == [0, 0, 0]
    ev = _ev([5, 5], [5, 5], [0, 129])
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    assert lab.tolist() == [0, 1]
    _check(orc, _ev([5, 5, 5, 6], [5, 5, 5, 6], [0, 128, 256, 384]), 1, 128)


def test_diagonal_chain_and_gap(orc):
    ev = _ev([0, 1, 2, 3, 5], [0, 1, 2, 3, 5], [0] * 5)
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    assert lab.tolist() == [0, 0, 0, 0, 4]
    _check(orc, ev, 1, 128)


def test_same_address_repeat(orc):
    # a re-fired pixel (Chebyshev distance 0) joins within dt, not beyond
    ev = _ev([3, 3, 3], [3, 3, 3], [0, 100, 400])
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    assert lab.tolist() == [0, 0, 2]


def test_shots_never_merge(orc):
    ev = _ev([1, 1], [1, 1], [50, 50], shot=[0, 1], trig=(0, 0))
    lab, nc = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    assert lab.tolist() == [0, 1] and nc == 2


def test_zero_tot_hit_is_flagged(orc):
    ev = _ev([1, 2], [1, 1], [10, 20], tot=[0, 0])
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    h = orc.centroid(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], lab, ev["trig"])
    assert h.size == 1 and h["flags"][0] == 1
    assert h["x"][0] == 1.5 and h["y"][0] == 1.0 and h["tof_ns"][0] == 15 * 1.5625
    _check(orc, ev, 1, 128)


def test_unsorted_shots_order_of_hits(orc):
    ev = _ev([1, 9, 1], [1, 9, 1], [700, 5, 700], shot=[1, 0, 1], trig=(0, 600))
    lab, _ = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"])
    assert lab.tolist() == [0, 1, 0]
    h = orc.centroid(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], lab, ev["trig"])
    assert h["shot"].tolist() == [0, 1] and h["label"].tolist() == [1, 0]
    assert h["tof_ns"].tolist() == [5 * 1.5625, 100 * 1.5625]
