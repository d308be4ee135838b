"""Pins of the walk-calibration oracle (oracle/walkfit.py, Sec. IV ToT-ToF
Correlation Correction, Eq. 1) against what the mathematics and the generator
fix: exact recovery of Eq. (1) from noise-free centres, equality of the
count-weighted fit over ToT values with a direct fit over the individual
pixels, recovery of the generator's walk from a calibration run, the window
selection, and the shift of c alone under a shift of every ToF."""
import numpy as np
import pytest

import synth
from oracle import walkfit as W

TRUE = dict(a=300.0, b=4.0, d=1.05, c=1.2)


def test_exact_centres_recover_the_parameters():
    t = np.arange(5, 1000, 7)
    mean = W.model(t, TRUE["a"], TRUE["b"], TRUE["d"], TRUE["c"])
    a, b, c, d = W.fit_centres(t, mean, np.full(t.size, 50))
    assert a == pytest.approx(TRUE["a"], rel=1e-6)
    assert b == pytest.approx(TRUE["b"], rel=1e-6)
    assert c == pytest.approx(TRUE["c"], rel=1e-6, abs=1e-7)
    assert d == pytest.approx(TRUE["d"], rel=1e-7)


def test_weighted_centres_equal_a_direct_fit_over_pixels():
    """Least squares over pixels = least squares over ToT values weighted by
    their counts (a fit that ignored the counts would differ)."""
    from scipy.optimize import least_squares
    rng = np.random.default_rng(3)
    tot = rng.integers(6, 400, 4000)
    tot[:3000] = rng.integers(6, 30, 3000)          # very uneven counts
    tof_ns = W.model(tot, 250.0, 3.0, 1.0, 2.0) + rng.normal(0, 3.0, tot.size)
    tof = np.rint(tof_ns / W.TICK_NS).astype(np.int64)
    n, mean = W.slice_centres(tot, tof, -10**9, 10**9)
    use = np.nonzero(n > 0)[0]
    p = W.fit_centres(use, mean[use], n[use])
    y = tof * W.TICK_NS
    x0 = W.initial_guess(use, mean[use])
    r = least_squares(lambda q: W.model(tot, q[0], q[1], q[2], q[3]) - y,
                      np.array([x0[0], x0[1], x0[3], x0[2]]), method="lm", xtol=1e-15, ftol=1e-15,
                      gtol=1e-15, max_nfev=20000)
    a, b, d, c = r.x
    assert p[0] == pytest.approx(a, rel=1e-5)
    assert p[1] == pytest.approx(b, rel=1e-5, abs=1e-6)
    assert p[2] == pytest.approx(c, rel=1e-5, abs=1e-6)
    assert p[3] == pytest.approx(d, rel=1e-6)
    unweighted = W.fit_centres(use, mean[use], np.ones(use.size))
    assert abs(unweighted[0] - a) > 1e-3 * abs(a) or abs(unweighted[3] - d) > 1e-4


def test_calibration_run_recovers_the_generator_walk():
    ev, trig = synth.calibration_run(7, 40_000, tof0_ns=5000.0)
    lo, hi = int(4950 / W.TICK_NS), int(5200 / W.TICK_NS)
    r = W.walk_fit(ev, trig, lo, hi, min_count=30)
    a, b, c, d = r["params"]
    tab = W.walk_table(r["params"])
    t = np.nonzero(r["count"] >= 30)[0]
    true_walk = synth.walk_ns(t, **TRUE) - TRUE["c"]
    # the fitted walk matches the generator's (up to the constant, which
    # goes into c) within the statistics of the run and the tick rounding
    assert np.abs((tab[t] + c) - (true_walk + TRUE["c"] + 5000.0)).max() < 0.3
    assert c == pytest.approx(5000.0 + TRUE["c"], abs=0.5)
    # corrected ToF of the slice no longer depends on ToT
    tof = ev["toa"].astype(np.int64) - trig.astype(np.int64)[ev["shot"].astype(np.int64)]
    sel = (tof >= lo) & (tof <= hi)
    corr = tof[sel] * W.TICK_NS - tab[ev["tot"][sel].astype(np.int64)]
    lowt = ev["tot"][sel] < 40
    assert abs(corr[lowt].mean() - corr[~lowt].mean()) < 0.3


def test_window_and_shift():
    ev, trig = synth.calibration_run(8, 12_000, tof0_ns=5000.0)
    lo, hi = int(4950 / W.TICK_NS), int(5200 / W.TICK_NS)
    base = W.walk_fit(ev, trig, lo, hi)
    # pixels outside the window change nothing
    extra = {k: np.concatenate([v, v[:500]]) for k, v in ev.items()}
    extra["toa"][-500:] += np.uint64(hi + 10_000)
    again = W.walk_fit(extra, trig, lo, hi)
    assert np.allclose(again["params"], base["params"], rtol=0, atol=0)
    # every ToF later by 64 ticks: c moves by 100 ns, the walk does not
    sh = dict(ev)
    sh["toa"] = ev["toa"] + np.uint64(64)
    moved = W.walk_fit(sh, trig, lo + 64, hi + 64)
    a, b, c, d = moved["params"]
    assert c == pytest.approx(base["params"][2] + 100.0, abs=1e-4)
    assert np.allclose([a, b, d], [base["params"][0], base["params"][1], base["params"][3]],
                       rtol=1e-5)
