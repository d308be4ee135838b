"""Segment stride and clustering kernel of the stream path and their
autotuner, through the C ABI: the hits equal the oracle's at every stride and
with every kernel (small strides send large shots to the global-memory path,
large ones fill the LDS), and an autotune run leaves the stream state as it
was."""
import sys

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


@pytest.fixture(scope="module")
def c3(orc):
    w = synth.make_config("c3", n_shots=300)
    ref, rst = orc.run(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    return w, ref, rst


@pytest.mark.parametrize("q", [64, 100, 333, 512, 2048, 4096])
def test_stride_parity_uneven_shots(tpx, c3, q):
    w, ref, rst = c3
    # every kernel in separate launches, then the persistent launch (None)
    for k in list(range(-1, tpx.kernel_count())) + [None]:
        print(f"c3 300 shots, stride {q}, kernel {k}", flush=True)
        sys.stdout.flush()
        s = tpx.Stream(w.n_packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0,
                       kernel=1 if k is None else k, persistent=k is None)
        try:
            s.set_segment(q)
            assert s.segment() == q and s.kernel() == (1 if k is None else k)
            h, st = s.process(w.packets, flush=True)
        finally:
            s.close()
        assert st["n_events"] == rst["n_events"]
        assert_hits_match(h, ref)


def test_stride_parity_chunked(tpx, orc):
    w = synth.make_config("c5", n_shots=80)
    ref, _ = orc.run(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    s = tpx.Stream(20_000, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    try:
        s.set_segment(64)
        out = []
        for a in range(0, w.n_packets, 20_000):
            h, _ = s.process(w.packets[a:a + 20_000], flush=a + 20_000 >= w.n_packets)
            out.append(h)
    finally:
        s.close()
    assert_hits_match(np.concatenate(out), ref)


def test_stride_bounds(tpx):
    s = tpx.Stream(1000)
    try:
        for q in (0, 63, 4097):
            with pytest.raises(tpx.TpxError) as e:
                s.set_segment(q)
            assert e.value.rc == tpx.EINVAL
        assert s.segment() == 1024
    finally:
        s.close()


def test_autotune_keeps_state(tpx, c3):
    import torch
    w, ref, _ = c3
    half = w.n_packets // 2
    s = tpx.Stream(w.n_packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    try:
        h1, _ = s.process(w.packets[:half])                   # state with open shots
        hits = torch.empty((w.n_packets, 48), dtype=torch.uint8, device="cuda")
        pk = torch.from_numpy(w.packets[half:].view(np.int64)).cuda()
        kernels = list(range(-1, tpx.kernel_count()))
        best, best_k, ms = s.autotune(pk, True, [64, 256, 1024, 4096], hits, w.n_packets, reps=2,
                                      kernels=kernels)
        print(f"autotune: best {best}, kernel {best_k}, {ms}", flush=True)
        assert best in (64, 256, 1024, 4096) and s.segment() == best
        assert best_k in kernels and s.kernel() == best_k
        assert len(ms) == 4 * len(kernels) and all(v > 0 for v in ms.values())
        h2, _ = s.process(w.packets[half:], flush=True)
    finally:
        s.close()
    assert_hits_match(np.concatenate([h1, h2]), ref)


def test_kernel_bounds(tpx):
    s = tpx.Stream(1000)
    try:
        k0 = s.kernel()
        for k in (-2, tpx.kernel_count()):
            with pytest.raises(tpx.TpxError) as e:
                s.set_kernel(k)
            assert e.value.rc == tpx.EINVAL
        assert s.kernel() == k0
    finally:
        s.close()
