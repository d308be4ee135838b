"""The input generator: seeded, deterministic, with the shapes the configs
describe (pixels per hit, hits per shot, noise share, wrap placement)."""
import numpy as np

import synth


def test_deterministic_and_worker_independent():
    a = synth.make_config("c2", n_shots=2500, workers=1)
    b = synth.make_config("c2", n_shots=2500, workers=2)
    assert np.array_equal(a.packets, b.packets)
    assert np.array_equal(a.t_abs, b.t_abs)


def test_shapes_of_the_configs():
    stats = {}
    for name, shots in (("c1", 1000), ("c2", 2000), ("c3", 4000), ("c5", 300)):
        w = synth.make_config(name, n_shots=shots)
        km = w.kept_mask()
        sig = km & (w.hit >= 0)
        stats[name] = dict(events=int(km.sum()), hits=int(w.hit_x.size),
                           px_per_hit=float(sig.sum() / max(w.hit_x.size, 1)),
                           hits_per_shot=float(w.hit_x.size / shots))
        print(name, stats[name])
        # report order: packet stream is sorted by report time, so the kept
        # pixels of one shot never precede that shot's trigger word
        trig_pos = np.nonzero(w.kind == synth.KIND_TRIGGER)[0]
        first_ev = np.array([np.argmax((w.shot == s) & (w.kind == synth.KIND_PIXEL)) for s in range(0, shots, max(shots // 50, 1))])
        assert np.all(trig_pos[np.arange(0, shots, max(shots // 50, 1))] < first_ev)
    assert 11.0 < stats["c1"]["px_per_hit"] < 13.0          # sigma 0.8
    assert 9.5 < stats["c1"]["hits_per_shot"] < 10.5         # Poisson(10)
    assert 19.0 < stats["c2"]["px_per_hit"] < 24.0           # sigma U(0.6, 1.5)
    assert 29.0 < stats["c2"]["hits_per_shot"] < 31.0        # Poisson(30)
    assert 25.0 < stats["c3"]["px_per_hit"] < 40.0
    assert 21.0 < stats["c3"]["hits_per_shot"] < 26.0        # mixture mean 23.5


def test_noise_and_cut_fractions():
    w = synth.make_config("c1")
    pix = w.kind == synth.KIND_PIXEL
    noise = pix & (w.hit < 0)
    assert abs(noise.sum() / pix.sum() - 0.01) < 0.002
    cut = noise & (w.tof > 64_000)
    assert 0.85 < cut.sum() / noise.sum() < 0.95       # ~90 % of dark counts cut


def test_c5_wrap_inside_replay():
    w = synth.make_config("c5", n_shots=2500)
    t = w.t_abs[w.kind == synth.KIND_PIXEL]
    assert t.min() < synth.PIX_WRAP_TICKS < t.max()
    assert w.pix_epoch0 == 0
