"""Decode, unwrap and shot assignment in the oracle (Sec. III, Sec. IV),
pinned by hand-built words, by the generator's ground truth and by streams
constructed around the wrap of the ToA counters."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

W34, W36 = 1 << 34, 1 << 36
J = 12_800_000_000            # 20 s in 1.5625 ns ticks


def _pix_word(x, y, toa14, tot, ftoa, spidr):
    # written out field by field, independently of the generator's encoder
    return (0xB << 60) | ((x // 2) << 53) | ((y // 4) << 47) | (((x % 2) * 4 + y % 4) << 44) \
        | (toa14 << 30) | (tot << 20) | (ftoa << 16) | spidr


def _tdc_word(stamp35, subtype=0xF, counter=0):
    return (0x6 << 60) | (subtype << 56) | (counter << 44) | (stamp35 << 9)


def test_hand_built_words(orc):
    w = _pix_word(201, 77, 0x1234, 0x2AB, 9, 0xBEEF)
    k, x, y, tot, raw = orc.decode_word(w)
    assert (k, x, y, tot) == (0, 201, 77, 0x2AB)
    assert raw == (((0xBEEF << 14) | 0x1234) * 16 - 9) % W34
    # fine ToA below a zero coarse counter lands just before the wrap
    assert orc.decode_word(_pix_word(0, 0, 0, 1, 5, 0))[4] == W34 - 5
    assert orc.decode_word(_pix_word(255, 255, 0x3FFF, 0x3FF, 0, 0xFFFF))[1:4] == (255, 255, 1023)
    k, *_, raw = orc.decode_word(_tdc_word((1 << 35) - 1, counter=0xABC))
    assert k == 1 and raw == W36 - 2
    assert orc.decode_word(_tdc_word(12345, subtype=0xA))[0] == 2      # falling edge
    assert orc.decode_word(0x4 << 60 | 0xDEADBEEF)[0] == 2
    assert orc.decode_word(0)[0] == 2


@pytest.mark.parametrize("name,shots", [("c1", 1000), ("c2", 600), ("c3", 300)])
def test_roundtrip_with_generator(orc, name, shots):
    w = synth.make_config(name, n_shots=shots)
    pix = w.kind == synth.KIND_PIXEL
    sub = np.array([orc.decode_word(int(p)) for p in w.packets[:3000]])
    m = pix[:3000]
    assert np.array_equal(sub[m, 1], w.x[:3000][m])
    assert np.array_equal(sub[m, 2], w.y[:3000][m])
    assert np.array_equal(sub[m, 3], w.tot[:3000][m])
    assert np.array_equal(sub[m, 4], w.t_abs[:3000][m] % W34)
    r = orc.decode(w.packets, want_times=True, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    both = w.kind != synth.KIND_OTHER
    assert np.array_equal(r["t"][both], w.t_abs[both])          # unwrapped = true time
    assert np.array_equal(r["trig"], w.trig_ticks)
    km = w.kept_mask()
    ev = r["events"]
    for f in ("x", "y", "tot", "shot"):
        assert np.array_equal(ev[f].astype(np.int64), getattr(w, f)[km])
    assert np.array_equal(ev["toa"].astype(np.int64), w.t_abs[km])
    s = r["stats"]
    assert s["n_pre_trigger"] == int(np.sum(pix & (w.shot < 0)))
    assert s["n_tof_cut"] == int(np.sum(pix & (w.shot >= 0) & (w.tof > 64_000)))
    assert s["n_other"] == int(np.sum(w.kind == synth.KIND_OTHER))
    assert s["n_tdc"] == w.trig_ticks.size


def test_unwrap_across_coincident_wraps(orc):
    """Shot 100 straddles the instant where the pixel counter (2^34) and the
    trigger counter (2^36) wrap together; late reporters from before the wrap
    arrive after pixels from after it."""
    spec = dataclasses.replace(synth.SPECS["c1"], n_shots=200, seed=77,
                               t0_ticks=W36 - 3000 - 100 * synth.SHOT_PERIOD_TICKS)
    w = synth.generate(spec)
    r = orc.decode(w.packets, want_times=True, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    both = w.kind != synth.KIND_OTHER
    assert np.array_equal(r["t"][both], w.t_abs[both])
    s = r["stats"]
    assert s["n_tdc_wraps"] == 1 and s["n_tdc_backjumps"] == 0
    assert s["n_pix_backjumps"] >= 1
    assert s["n_pix_wraps"] - s["n_pix_backjumps"] == 1
    assert w.pix_epoch0 == 3 and w.tdc_epoch0 == 0


def _pix_at(t, x=1, y=1, tot=5):
    raw = t % W34
    coarse = -(-raw // 16)
    ftoa = coarse * 16 - raw
    coarse %= 1 << 30
    return _pix_word(x, y, coarse & 0x3FFF, tot, ftoa, coarse >> 14)


def _trig_at(t):
    return _tdc_word((t % W36) // 2)


def test_late_reporter_by_hand(orc):
    T = W34 - 1000                                   # trigger just before the wrap
    ts = [T + 10, W34 + 5, T + 900, W34 + 40, T + 950, W34 + 41]
    pk = np.array([_trig_at(T)] + [_pix_at(t) for t in ts], np.uint64)
    r = orc.decode(pk, want_times=True)
    assert r["t"][1:].tolist() == ts
    s = r["stats"]
    assert (s["n_pix_wraps"], s["n_pix_backjumps"]) == (3, 2)
    assert r["events"]["toa"].tolist() == ts        # all within the ToF window


def test_assignment_boundaries(orc):
    T0, T1 = 1_000_000, 1_640_000
    pk = [_pix_at(T0 - 1), _trig_at(T0), _pix_at(T0), _pix_at(T0 + 64_000),
          _pix_at(T0 + 64_001), _pix_at(T1 + 3), _trig_at(T1), _pix_at(T1 - 1)]
    r = orc.decode(np.array(pk, np.uint64))
    s = r["stats"]
    assert s["n_pre_trigger"] == 1 and s["n_tof_cut"] == 2
    ev = r["events"]
    # the pixel reported before its trigger word still belongs to shot 1
    assert ev["toa"].tolist() == [T0, T0 + 64_000, T1 + 3]
    assert ev["shot"].tolist() == [0, 0, 1]
    r = orc.decode(np.array(pk, np.uint64), tof_max_ticks=64_001)
    assert r["stats"]["n_tof_cut"] == 1


def test_stream_errors(orc):
    # triggers must not go back in time
    with pytest.raises(oracle.OracleError) as e:
        orc.decode(np.array([_trig_at(5000), _trig_at(1000)], np.uint64))
    assert e.value.rc == oracle.ESTREAM
    # a late reporter before the first wrap would need a negative wrap count
    with pytest.raises(oracle.OracleError) as e:
        orc.decode(np.array([_pix_at(100), _pix_at(W34 - 100)], np.uint64))
    assert e.value.rc == oracle.ESTREAM
    # ...which is legal when the stream starts in a later epoch
    r = orc.decode(np.array([_pix_at(W34 + 100), _pix_at(W34 - 100)], np.uint64),
                   want_times=True, pix_epoch0=1)
    assert r["t"].tolist() == [W34 + 100, W34 - 100]
