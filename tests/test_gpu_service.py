"""tpx_service (continuous batching over one stream) through the C ABI: any
admission pattern and any run schedule give the hits of the whole stream
processed at once, compared with the oracle (integers bit-exact, centroids
within 1e-4 px and 0.1 ns); ring wrap-around, staging, and the error paths."""
import sys

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


@pytest.fixture(scope="module")
def c5(orc):
    w = synth.make_config("c5", n_shots=150)
    ref, rst = orc.run(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    return w, ref, rst


def _drive(tpx, sv, chunks, run_after, on_device):
    """Submit every chunk (running first when the ring is full), run where
    asked, then flush until every chunk is done; returns hits and stats."""
    import torch
    out, n_ev, n_runs = [], 0, 0

    def run(flush):
        nonlocal n_ev, n_runs
        h, nd, st = sv.run(flush=flush, hit_cap=1 << 16)
        out.append(h)
        n_ev += st["n_events"]
        n_runs += 1
        return nd

    for k, c in enumerate(chunks):
        arg = torch.from_numpy(c.view(np.int64)).cuda() if on_device[k] else c
        try:
            assert sv.submit(arg) == k
        except tpx.TpxError as e:
            assert e.rc == tpx.ECAPACITY
            run(False)
            assert sv.submit(arg) == k
        if run_after[k]:
            run(False)
    while run(True) < len(chunks):
        pass
    return np.concatenate(out), n_ev, n_runs


@pytest.mark.parametrize("seed", range(6))
def test_random_batching_matches_whole_stream(tpx, c5, seed):
    w, ref, rst = c5
    rng = np.random.default_rng(4100 + seed)
    k = int(rng.integers(4, 40))
    cuts = np.sort(rng.choice(np.arange(1, w.n_packets), k, replace=False))
    chunks = np.split(w.packets, cuts)
    sizes = [c.size for c in chunks]
    max_batch = int(max(sizes) * rng.choice([1, 2, 5]))
    ring = int(max_batch + rng.integers(0, 2 * max_batch))   # small rings force wraps
    _say(f"service seed={seed} chunks={len(chunks)} max_batch={max_batch} ring={ring}")
    sv = tpx.Service(max_batch, ring, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    try:
        h, n_ev, n_runs = _drive(tpx, sv, chunks, rng.random(len(chunks)) < 0.35,
                                 rng.random(len(chunks)) < 0.5)
    finally:
        sv.close()
    _say(f"  {n_runs} runs, {h.size} hits")
    assert n_ev == rst["n_events"]
    assert_hits_match(h, ref)


def test_one_chunk_per_run_and_empty_chunks(tpx, c5):
    """Runs that take one chunk each (batch limit = chunk size) and empty
    chunks in between give the same hits."""
    w, ref, _ = c5
    step = 5000
    chunks = []
    for a in range(0, w.n_packets, step):
        chunks.append(w.packets[a:a + step])
        chunks.append(w.packets[:0])
    sv = tpx.Service(step, 3 * step + 7, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    try:
        h, _, n_runs = _drive(tpx, sv, chunks, [True] * len(chunks), [k % 3 == 0 for k in
                                                                       range(len(chunks))])
    finally:
        sv.close()
    assert n_runs >= len(chunks) // 2
    assert_hits_match(h, ref)


def test_errors_leave_the_service_unchanged(tpx, c5):
    w, ref, _ = c5
    import paper_2603_04942_amd as t
    with pytest.raises(t.TpxError) as e:
        t.Service(1000, 999)
    assert e.value.rc == t.EINVAL
    n = w.n_packets
    half = n // 2
    sv = t.Service(n - half + 1, n - half + 1, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    try:
        with pytest.raises(t.TpxError) as e:
            sv.submit(np.zeros(n - half + 2, np.uint64))        # larger than the batch limit
        assert e.value.rc == t.EINVAL
        assert sv.submit(w.packets[:half]) == 0
        with pytest.raises(t.TpxError) as e:
            sv.submit(w.packets[half:])                          # ring full
        assert e.value.rc == t.ECAPACITY
        # a hit buffer that is too small: status and count, batch stays admitted
        import torch
        small = torch.empty((1, 48), dtype=torch.uint8, device="cuda")
        rc, nh, nd, _ = sv.run_raw(False, small, 0)
        assert rc == t.ECAPACITY and nh > 0 and nd == 0
        h1, nd, _ = sv.run(False, hit_cap=1 << 16)
        assert nd == 1
        assert sv.submit(w.packets[half:]) == 1                  # wraps the ring
        h2, nd, _ = sv.run(True, hit_cap=1 << 16)
        assert nd == 2
    finally:
        sv.close()
    assert_hits_match(np.concatenate([h1, h2]), ref)


@pytest.mark.parametrize("seed", range(3))
def test_submit_from_another_thread_while_running(tpx, c5, seed):
    """A producer thread admits chunks (host and device memory, a small ring
    that fills and wraps) while the main thread runs batches: the copies of
    new chunks overlap the batch on the GPU, and the hits equal the whole
    stream's."""
    import threading
    import time

    import torch
    w, ref, rst = c5
    rng = np.random.default_rng(5100 + seed)
    cuts = np.sort(rng.choice(np.arange(1, w.n_packets), int(rng.integers(10, 60)), replace=False))
    chunks = np.split(w.packets, cuts)
    dev = [torch.from_numpy(c.view(np.int64)).cuda() if k % 2 else c for k, c in enumerate(chunks)]
    torch.cuda.synchronize()
    max_batch = int(max(c.size for c in chunks) * 3)
    sv = tpx.Service(max_batch, int(max_batch * 1.5), pix_epoch0=w.pix_epoch0,
                     tdc_epoch0=w.tdc_epoch0)
    done = threading.Event()
    errors = []

    def producer():
        try:
            for c in dev:
                while True:
                    try:
                        sv.submit(c)
                        break
                    except tpx.TpxError as e:
                        if e.rc != tpx.ECAPACITY:
                            raise
                        time.sleep(1e-4)
        except Exception as e:  # noqa: BLE001 - reported by the main thread
            errors.append(e)
        finally:
            done.set()

    t = threading.Thread(target=producer)
    out, n_ev, runs = [], 0, 0
    try:
        t.start()
        while True:
            fin = done.is_set()
            h, nd, st = sv.run(flush=fin, hit_cap=1 << 16)
            out.append(h)
            n_ev += st["n_events"]
            runs += 1
            if (fin and nd == len(chunks)) or errors:
                break
            assert runs < 100_000
    finally:
        t.join()
        sv.close()
    assert not errors, errors
    _say(f"  threaded: {len(chunks)} chunks in {runs} runs")
    assert n_ev == rst["n_events"]
    assert_hits_match(np.concatenate(out), ref)
