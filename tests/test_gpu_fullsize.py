"""Parity at full workload size, in the configuration the benchmark times: the
whole c2 stream (100,000 shots, ~6.4e7 packets) and the whole c3 stream
(200,000 shots of uneven multiplicity, ~1.5e8 packets) as one flushed chunk
through tpx_process_stream, compared hit by hit with the oracle on the same
packets (integers bit-exact, centroids within 1e-4 px and 0.1 ns)."""
import os
import sys
import time

import numpy as np
import pytest

import synth
from test_gpu_parity import assert_hits_match

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tpx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_04942_amd as t
    t.load()
    return t


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_stream_full_size(tpx, orc, name):
    workers = min(16, os.cpu_count() or 1)
    t = time.perf_counter()
    w = synth.make_config(name, with_truth=False, workers=workers)
    print(f"{name}: {w.n_packets} packets generated in {time.perf_counter() - t:.1f} s", flush=True)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    t = time.perf_counter()
    h, st = tpx.process_stream(w.packets, **kw)
    print(f"{name}: GPU {h.size} hits in {time.perf_counter() - t:.1f} s", flush=True)
    t = time.perf_counter()
    ref, rst = orc.run(w.packets, **kw)
    print(f"{name}: oracle {ref.size} hits in {time.perf_counter() - t:.1f} s", flush=True)
    sys.stdout.flush()
    for f in ("n_pixels", "n_tdc", "n_other", "n_pre_trigger", "n_tof_cut", "n_events"):
        assert st[f] == rst[f], f
    assert st["n_late_drop"] == 0
    assert_hits_match(h, ref)
    # conservation over the whole stream
    assert int(h["npix"].astype(np.int64).sum()) == st["n_events"]


def test_paper_mode_full_size_sampled(tpx, orc):
    """tpx_local_maxima over the whole decoded c2 stream (the configuration
    the benchmark times); the oracle recomputes 250 randomly drawn shots one
    by one and their hits must match those of the full run."""
    workers = min(16, os.cpu_count() or 1)
    w = synth.make_config("c2", with_truth=False, workers=workers)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ev, trig, _, _ = tpx.decode(w.packets, params=tpx.make_params(**kw))
    h = tpx.local_maxima(ev, trig)
    print(f"c2 paper mode: {h.size} hits from {ev['x'].numel()} events", flush=True)
    shot = ev["shot"].cpu().numpy().view(np.uint32)
    host = {k: v.cpu().numpy() for k, v in ev.items()}
    trig_h = trig.cpu().numpy().view(np.uint64)
    picks = np.sort(np.random.default_rng(2603).choice(int(shot.max()) + 1, 250, replace=False))
    for s in picks:
        idx = np.nonzero(shot == s)[0]
        e = dict(x=host["x"][idx].view(np.uint16), y=host["y"][idx].view(np.uint16),
                 tot=host["tot"][idx].view(np.uint16), shot=shot[idx],
                 toa=host["toa"][idx].view(np.uint64))
        ref = orc.local_maxima(e["x"], e["y"], e["tot"], e["shot"], e["toa"], trig_h)
        ref["label"] = idx[ref["label"].astype(np.int64)]
        got = h[h["shot"] == s]
        assert_hits_match(got, ref)


def test_learned_full_size_sampled(tpx):
    """Patches and the forward pass over 10^6 generated clusters (the
    held-out set the benchmark scores); the oracle recomputes 300 randomly
    drawn clusters from their own events: patches bit-exact, outputs within
    the bfloat16 tolerance of the learned-part parity tests."""
    import torch

    from oracle import learned as L
    from paper_2603_04942_amd.learned import prepare
    from test_gpu_learned import REL_TOL, _rand_params
    import oracle
    orc = oracle.get()
    n = 1_000_000
    cl = synth.make_clusters(4002, n, block=50_000)
    feat, hits, _, _ = prepare(cl)
    p = _rand_params(11)
    out = tpx.Mlp(p, batch=16).forward(feat).cpu().numpy()
    got = feat.cpu().numpy().view(np.uint16)
    print(f"learned full size: {n} clusters, {cl['events']['x'].size} events", flush=True)
    picks = np.sort(np.random.default_rng(77).choice(n, 300, replace=False))
    e = cl["events"]
    ref_feat = []
    for s in picks:
        lo, m = int(cl["first"][s]), int(cl["counts"][s])
        sl = slice(lo, lo + m)
        lab = (cl["labels"][sl] - lo).astype(np.uint32)     # indices into the slice
        h = orc.centroid(e["x"][sl], e["y"][sl], e["tot"][sl], e["shot"][sl], e["toa"][sl],
                         lab, np.zeros(n, np.uint64))
        ref_feat.append(L.patches(e["x"][sl], e["y"][sl], e["tot"][sl], e["toa"][sl],
                                  e["shot"][sl], lab, h)[0])
    ref_feat = np.array(ref_feat)
    assert np.array_equal(got[picks], ref_feat)
    ref, _ = L.forward(p, ref_feat)
    rms = float(np.sqrt(np.mean(ref ** 2)))
    assert np.abs(out[picks] - ref).max() <= REL_TOL * rms
