"""Several independent request streams served at once (tpx_server), through
the C ABI: slots are admitted against the HBM budget and return their memory
when closed; three slots with different workloads, each driven from its own
host thread (chunks submitted and batches run as they come, runs on
different HIP streams), give exactly the hits each gives alone, which equal
the oracle's.  And the native paced replay of the service processes every
chunk of a stream."""
import sys
import threading

import numpy as np
import pytest

import synth
from test_gpu_parity import assert_hits_match

pytestmark = pytest.mark.gpu


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


def test_admission_against_the_budget(tpx):
    probe = tpx.Server(1 << 40, n_streams=2)
    _, one = probe.open(20_000)
    probe.close()
    sr = tpx.Server(2 * one + one // 2, n_streams=2)
    try:
        a, _ = sr.open(20_000)
        b, _ = sr.open(20_000)
        assert (a, b) == (0, 1)
        assert sr.free_bytes == one // 2
        with pytest.raises(tpx.TpxError) as e:
            sr.open(20_000)
        assert e.value.rc == tpx.ECAPACITY
        assert sr.free_bytes == one // 2             # nothing stays allocated
        sr.close_slot(a)
        c, _ = sr.open(20_000)
        assert c == 0                                # the lowest free slot
        with pytest.raises(tpx.TpxError):
            sr.submit(5, np.zeros(4, np.uint64))    # no such slot
    finally:
        sr.close()


def test_slots_in_the_mix_equal_alone(tpx, orc):
    work = []
    for name, shots, chunk, seed in (("c5", 120, 9_000, 1), ("c1", 500, 2_500, 2),
                                     ("c3", 60, 60_000, 3)):
        w = synth.make_config(name, n_shots=shots)
        kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
        ref, _ = orc.run(w.packets, **kw)
        rng = np.random.default_rng(seed)
        sizes = rng.integers(chunk // 4, chunk + 1, w.n_packets // (chunk // 4) + 2)
        cuts = np.cumsum(sizes)
        parts = np.split(w.packets, cuts[cuts < w.n_packets])
        assert sum(p.size for p in parts) == w.n_packets and max(p.size for p in parts) <= chunk
        work.append((name, kw, ref, parts, chunk))
    import paper_2603_04942_amd as T

    def drive(sr, slot, parts, out, errors):
        try:
            got, done = [], 0
            for i, p in enumerate(parts):
                sr.submit(slot, p)
                if i % 2 == 1:            # a run takes two parts or more: no backlog
                    h, done = sr.run(slot)
                    got.append(h)
            # a run takes at most max_batch words: drain the rest, and end
            # the stream with a flushing run (possibly of no new words)
            while True:
                h, done = sr.run(slot, flush=True)
                got.append(h)
                if done == len(parts):
                    break
            out.append(np.concatenate(got))
        except Exception as e:  # reported by the main thread
            errors.append(e)

    alone = []
    for name, kw, ref, parts, chunk in work:
        sr = T.Server(1 << 40, n_streams=1, **kw)
        slot, _ = sr.open(2 * chunk)
        out, errors = [], []
        drive(sr, slot, parts, out, errors)
        sr.close()
        assert not errors, errors
        assert_hits_match(out[0], ref)
        alone.append(out[0])
        _say(f"{name}: {out[0].size} hits alone")
    # all three at once: one server, three slots (each with its own epochs),
    # three host threads, runs on three HIP streams
    sr = T.Server(1 << 40, n_streams=3)
    try:
        slots = [sr.open(2 * chunk, **kw)[0] for name, kw, ref, parts, chunk in work]
        assert slots == [0, 1, 2]
        outs = [[] for _ in work]
        errors = []
        th = [threading.Thread(target=drive, args=(sr, slots[k], work[k][3], outs[k], errors))
              for k in range(len(work))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        for k in range(len(work)):
            assert outs[k][0].tobytes() == alone[k].tobytes()
    finally:
        sr.close()


def test_native_paced_replay(tpx):
    import torch
    w = synth.make_config("c5", n_shots=600)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    pk = torch.from_numpy(w.packets.view(np.int64)).cuda()
    sv = tpx.Service(1 << 18, 1 << 20, **kw)
    try:
        rate = w.n_packets / 0.6 * 50.0              # 50x the acquisition rate
        lat, runs = sv.replay(pk, 8192, rate)
        n_chunks = -(-w.n_packets // 8192)
        _say(f"replay: {n_chunks} chunks in {runs} runs, p50 {np.percentile(lat, 50):.3f} ms, "
             f"p99 {np.percentile(lat, 99):.3f} ms")
        assert lat.size == n_chunks and 1 <= runs <= n_chunks
        assert np.all(lat > 0) and np.all(np.isfinite(lat))
        # the service is drained and reusable: the same stream again from
        # a fresh service gives the same number of hits as one whole call
        h_all, _ = tpx.process_stream(w.packets, **kw)
        sv2 = tpx.Service(1 << 18, 1 << 20, **kw)
        sv2.set_segment(256)                          # results do not depend on the stride
        total = 0
        for a in range(0, w.n_packets, 8192):
            sv2.submit(pk[a:a + 8192])
            h, _, _ = sv2.run(flush=a + 8192 >= w.n_packets)
            total += h.size
        sv2.close()
        assert total == h_all.size
    finally:
        sv.close()
