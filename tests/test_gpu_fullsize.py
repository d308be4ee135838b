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
