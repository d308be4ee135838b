"""Parity of tpx_local_maxima (the paper's local-maximum hits, Eqs. 6-7 and
Eq. 9 on A) with the oracle through the C ABI: integers bit-exact, centroids
within 1e-4 px and 0.1 ns."""
import json
import os
import sys

import numpy as np
import pytest

import synth
from test_gpu_parity import assert_hits_match

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tpx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_04942_amd as t
    t.load()
    return t


def _run(tpx, ev, trig, **kw):
    import torch
    d = tpx.to_device_events(ev)
    return tpx.local_maxima(d, torch.from_numpy(np.asarray(trig, np.uint64).view(np.int64)).cuda(),
                            params=tpx.make_params(**kw))


def test_worked_example(tpx, orc):
    g = json.load(open(os.path.join(HERE, "golden", "paper_example.json")))
    n = len(g["X"])
    ev = dict(x=np.array(g["X"], np.uint16), y=np.zeros(n, np.uint16),
              tot=np.array(g["ToT"], np.uint16), shot=np.zeros(n, np.uint32),
              toa=np.full(n, 5000, np.uint64))
    h = _run(tpx, ev, [0], dxy=g["radius"], dt_ticks=0)
    assert list(h["label"] + 1) == g["local_maxima_1based"]
    assert list(h["tot_sum"]) == g["centroid_den"]
    assert np.allclose(h["x"], np.array(g["centroid_num"]) / np.array(g["centroid_den"]), atol=1e-4)


@pytest.mark.parametrize("name,shots", [("c1", 1000), ("c2", 200), ("c5", 60)])
def test_decoded_workloads(tpx, orc, name, shots):
    _say(f"paper mode {name} shots={shots}")
    w = synth.make_config(name, n_shots=shots)
    d = orc.decode(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    e = d["events"]
    ref = orc.local_maxima(e["x"], e["y"], e["tot"], e["shot"], e["toa"], d["trig"])
    h = _run(tpx, e, d["trig"])
    assert_hits_match(h, ref)


@pytest.mark.parametrize("seed", range(24))
def test_tiny_with_ties(tpx, orc, seed):
    """Few distinct ToT values (many ties), radii 0-2, several windows, shots
    in and out of order."""
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 400))
    ev = synth.tiny_events(rng, n, grid=int(rng.integers(2, 20)), t_span=int(rng.integers(0, 800)),
                           n_shots=int(rng.integers(1, 5)), sort_by_shot=bool(seed % 3))
    ev["tot"] = rng.integers(0, 6, n).astype(np.uint16)
    S = int(ev["shot"].max()) + 1
    first = [int(ev["toa"][ev["shot"] == k].min()) if np.any(ev["shot"] == k) else 0 for k in range(S)]
    trig = np.array(first, np.uint64) - rng.integers(0, 50000, S).astype(np.uint64)
    dxy = int(rng.integers(0, 3))
    dt = int(rng.choice([0, 64, 128, 500]))
    ref = orc.local_maxima(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], trig, dxy=dxy,
                           dt_ticks=dt)
    h = _run(tpx, ev, trig, dxy=dxy, dt_ticks=dt)
    assert_hits_match(h, ref)


def test_walk_table_and_permutation(tpx, orc):
    import torch
    w = synth.make_config("c1", n_shots=300)
    d = orc.decode(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    e = d["events"]
    walk32 = (180.0 / (np.arange(1024) + 9.0) - 0.4).astype(np.float32)
    perm = np.random.default_rng(11).permutation(e["x"].size)
    ep = {k: v[perm] for k, v in e.items()}
    ref = orc.local_maxima(ep["x"], ep["y"], ep["tot"], ep["shot"], ep["toa"], d["trig"],
                           walk_ns=walk32.astype(np.float64))
    h = _run(tpx, ep, d["trig"], walk_lut_ns=torch.from_numpy(walk32).cuda())
    assert_hits_match(h, ref)


def test_errors(tpx):
    ev = dict(x=np.array([1], np.uint16), y=np.array([1], np.uint16), tot=np.array([1], np.uint16),
              shot=np.array([3], np.uint32), toa=np.array([0], np.uint64))
    with pytest.raises(tpx.TpxError) as e:
        _run(tpx, ev, [0, 0])            # shot 3 has no trigger time
    assert e.value.rc == tpx.EINVAL
    ev["shot"][0] = 0
    h = _run(tpx, ev, [0])
    assert h.size == 1 and h["npix"][0] == 1


def test_groups_beyond_lds(tpx, orc):
    """Shot groups larger than the 2,048 events a workgroup holds in LDS take
    the global-memory path: the uneven-shot workload (its Poisson(200) shots
    hold several thousand events), one shot of 3,009 events (isolated pixels
    and a blob) and one of 7,200 equal-ToT pixels (every decision a tie)."""
    from cases import big_component_packets, many_components_packets
    w = synth.make_config("c3", n_shots=150)
    cases = [("c3", w.packets, dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)),
             ("iso3000", many_components_packets(3000), {}),
             ("square", big_component_packets(side=60, layers=2), {})]
    for name, pk, kw in cases:
        d = orc.decode(pk, **kw)
        e = d["events"]
        counts = np.bincount(e["shot"].astype(np.int64))
        _say(f"paper mode {name}: {e['x'].size} events, largest shot {counts.max()}")
        assert counts.max() > 2048
        ref = orc.local_maxima(e["x"], e["y"], e["tot"], e["shot"], e["toa"], d["trig"])
        h = _run(tpx, e, d["trig"])
        assert_hits_match(h, ref)
