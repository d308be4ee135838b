"""Parity of the HIP path (through the C ABI) with the oracle on the same
seeded inputs.  Integer results (events, triggers, labels, hit membership)
must be bit-exact; centroids within 1e-4 px and 0.1 ns of the oracle's FP64
values."""
import dataclasses
import sys

import numpy as np
import pytest

import synth
from cases import big_component_packets, many_components_packets, shuffled_shapes_packets

pytestmark = pytest.mark.gpu

TOL_PX = 1e-4
TOL_NS = 0.1


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


def _np_events(ev):
    return dict(x=ev["x"].cpu().numpy().view(np.uint16), y=ev["y"].cpu().numpy().view(np.uint16),
                tot=ev["tot"].cpu().numpy().view(np.uint16),
                shot=ev["shot"].cpu().numpy().view(np.uint32),
                toa=ev["toa"].cpu().numpy().view(np.uint64))


def assert_hits_match(h, ref, tol_px=TOL_PX, tol_ns=TOL_NS):
    assert h.size == ref.size, (h.size, ref.size)
    for f in ("shot", "label", "npix", "tot_sum", "toa_first", "flags"):
        a = h[f].astype(np.uint64)
        b = ref[f].astype(np.uint64)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{f} differs at {bad[:5]}: {a[bad[:5]]} vs {b[bad[:5]]}"
    for f, tol in (("x", tol_px), ("y", tol_px), ("tof_ns", tol_ns)):
        d = np.abs(h[f].astype(np.float64) - ref[f])
        assert d.max(initial=0) <= tol, f"{f}: max err {d.max()} at {np.argmax(d)}"


# ------------------------------------------------------------------ decode
@pytest.mark.parametrize("name,shots", [("c1", 1000), ("c2", 400), ("c3", 200)])
def test_decode_parity(tpx, orc, name, shots):
    _say(f"decode parity {name} shots={shots}")
    w = synth.make_config(name, n_shots=shots)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref = orc.decode(w.packets, **kw)
    ev, trig, stats, _ = tpx.decode(w.packets, params=tpx.make_params(**kw))
    got = _np_events(ev)
    for f in ("x", "y", "tot", "shot", "toa"):
        assert np.array_equal(got[f], ref["events"][f]), f
    assert np.array_equal(trig.cpu().numpy().view(np.uint64), ref["trig"])
    for f in ("n_pixels", "n_tdc", "n_other", "n_pre_trigger", "n_tof_cut", "n_events",
              "n_pix_wraps", "n_pix_backjumps", "n_tdc_wraps", "n_tdc_backjumps"):
        assert stats[f] == ref["stats"][f], f


def test_decode_across_wraps_and_calls(tpx, orc):
    """Coincident pixel/trigger wrap inside shot 100; the stream is decoded
    whole and in 7 pieces with the carried state; both equal the oracle."""
    _say("decode across wraps")
    W36 = 1 << 36
    spec = dataclasses.replace(synth.SPECS["c1"], n_shots=200, seed=77,
                               t0_ticks=W36 - 3000 - 100 * synth.SHOT_PERIOD_TICKS)
    w = synth.generate(spec)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref = orc.decode(w.packets, **kw)
    assert ref["stats"]["n_pix_backjumps"] >= 1
    ev, trig, stats, _ = tpx.decode(w.packets, params=tpx.make_params(**kw))
    got = _np_events(ev)
    assert np.array_equal(got["toa"], ref["events"]["toa"])
    assert np.array_equal(got["shot"], ref["events"]["shot"])
    assert stats["n_pix_backjumps"] == ref["stats"]["n_pix_backjumps"]
    # piecewise with carried state
    cuts = np.sort(np.random.default_rng(5).choice(w.n_packets, 6, replace=False))
    parts = np.split(w.packets, cuts)
    st = None
    evs, trigs = [], []
    p = tpx.make_params(**kw)
    for part in parts:
        e, t, s, st = tpx.decode(part, state=st, params=p)
        evs.append(_np_events(e))
        trigs.append(t.cpu().numpy().view(np.uint64))
    cat = {f: np.concatenate([e[f] for e in evs]) for f in evs[0]}
    for f in ("x", "y", "tot", "shot", "toa"):
        assert np.array_equal(cat[f], ref["events"][f]), f
    assert np.array_equal(np.concatenate(trigs), ref["trig"])


# ------------------------------------------------------------------ stream
@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("name,shots", [("c1", 1000), ("c2", 300), ("c3", 120), ("c5", 150)])
def test_stream_whole(tpx, orc, name, shots, persistent):
    """Whole streams as one chunk, in one persistent launch (these chunks
    are small enough) and in separate launches."""
    _say(f"stream whole {name} shots={shots} persistent={persistent}")
    w = synth.make_config(name, n_shots=shots)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, rst = orc.run(w.packets, **kw)
    h, st = tpx.process_stream(w.packets, persistent=persistent, **kw)
    assert_hits_match(h, ref)
    for f in ("n_pixels", "n_tdc", "n_other", "n_pre_trigger", "n_tof_cut", "n_events"):
        assert st[f] == rst[f], f
    assert st["n_hits"] == ref.size and st["n_late_drop"] == 0


@pytest.mark.parametrize("seed", range(6))
def test_stream_chunked(tpx, orc, seed):
    """Random splits of a stream (odd seeds in separate launches, even ones
    in persistent launches); chunks may be empty of triggers or pixels."""
    w = synth.make_config("c5", n_shots=120)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 40))
    cuts = np.sort(rng.choice(np.arange(1, w.n_packets), k, replace=False))
    parts = np.split(w.packets, cuts)
    s = tpx.Stream(max(len(p) for p in parts), persistent=seed % 2 == 0, **kw)
    out = []
    for i, part in enumerate(parts):
        h, st = s.process(part, flush=(i == len(parts) - 1))
        out.append(h)
        assert st["n_late_drop"] == 0
    h = np.concatenate(out)
    assert_hits_match(h, ref)
    assert s.fallback_count == 0


def test_stream_persistent_near_the_tile_limit(tpx, orc):
    """A chunk of about 500 tiles in one persistent launch (one tile per
    thread in the prefix item, hundreds of segments taken by ticket), and the
    same stream as chunks above the limit, which take the separate launches."""
    w = synth.make_config("c2", n_shots=3200)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    tiles = -(-w.n_packets // 4096)
    _say(f"persistent limit: {w.n_packets} packets, {tiles} tiles")
    assert 400 < tiles <= 512
    h, _ = tpx.process_stream(w.packets, persistent=512, **kw)
    assert_hits_match(h, ref)
    s = tpx.Stream(w.n_packets, persistent=tiles - 1, **kw)   # every chunk above the limit
    h2, _ = s.process(w.packets, flush=True)
    s.close()
    assert h2.tobytes() == h.tobytes()


@pytest.mark.parametrize("persistent", [True, False])
def test_stream_ends_with_empty_flush(tpx, orc, persistent):
    """A stream whose last call flushes no new words: the open shots carried
    so far are closed by a call with no tiles (in the persistent launch every
    item then waits for the prefix over tiles directly)."""
    w = synth.make_config("c1", n_shots=500)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    s = tpx.Stream(5000, persistent=persistent, **kw)
    out = []
    for a in range(0, w.n_packets, 5000):
        h, _ = s.process(w.packets[a:a + 5000], flush=False)
        out.append(h)
    h, st = s.process(w.packets[:0], flush=True)
    out.append(h)
    assert h.size > 0 and st["n_events"] == 0
    assert_hits_match(np.concatenate(out), ref)


@pytest.mark.parametrize("n_iso", [1500, 3000, 20000])
def test_stream_many_components(tpx, orc, n_iso):
    """One shot whose pixels are all isolated plus one 3x3 blob: more
    components in one segment than the LDS accumulators hold (n_iso = 1500), a
    segment beyond the LDS event capacity (3000), and one shot of 20000 events
    spanning many segment strides; every clustering kernel."""
    _say(f"many components n_iso={n_iso}")
    pk = many_components_packets(n_iso)
    ref, _ = orc.run(pk)
    assert ref.size > 1024
    for k in range(-1, tpx.kernel_count()):
        h, _ = tpx.process_stream(pk, kernel=k, persistent=False)
        assert_hits_match(h, ref)
    h, _ = tpx.process_stream(pk, persistent=True)
    assert_hits_match(h, ref)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_stream_shuffled_shapes(tpx, orc, seed):
    """Connected shapes whose pixels arrive in a random order (a serpentine
    path of 819 pixels, a 20 x 20 square, a ring of 88): the
    smallest-neighbour forest has many local minima, so the clustering joins
    chain and displace parents concurrently; each shape must stay one hit,
    for every clustering kernel and the persistent launch."""
    _say(f"shuffled shapes seed={seed}")
    pk = shuffled_shapes_packets(seed)
    ref, _ = orc.run(pk)
    assert sorted(ref["npix"])[-3:] == [88, 400, 819]
    for k in range(-1, tpx.kernel_count()):
        h, _ = tpx.process_stream(pk, kernel=k, persistent=False)
        assert_hits_match(h, ref)
    h, _ = tpx.process_stream(pk, persistent=True)
    assert_hits_match(h, ref)


def test_stream_component_beyond_32bit_moments(tpx, orc):
    """One component of 36,992 pixels (a 136 x 136 square at ToT 1023, fired
    twice 50 ticks apart, x and y up to 255): its sum of ToT * x is about
    7e9, beyond 32 bits, so the moments must be accumulated in 64 bits."""
    _say("component beyond 32-bit moments")
    pk = big_component_packets()
    ref, _ = orc.run(pk)
    assert ref.size == 1 and ref["npix"][0] == 36992
    for k in range(-1, tpx.kernel_count()):
        h, _ = tpx.process_stream(pk, kernel=k, persistent=False)
        assert_hits_match(h, ref)
    h, _ = tpx.process_stream(pk, persistent=True)
    assert_hits_match(h, ref)


def test_streams_concurrent_on_two_hip_streams(tpx, orc):
    """Two tpx_stream objects driven at once from two host threads, each on its
    own HIP stream, chunk by chunk: each gives the hits it gives alone (and the
    oracle's)."""
    import threading

    import torch
    work = []
    for name, shots, seed in (("c5", 120, 3), ("c1", 600, 4)):
        w = synth.make_config(name, n_shots=shots)
        kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
        ref, _ = orc.run(w.packets, **kw)
        rng = np.random.default_rng(seed)
        cuts = np.sort(rng.choice(np.arange(1, w.n_packets), 12, replace=False))
        parts = np.split(w.packets, cuts)
        work.append((kw, ref, parts))
    alone = []
    for kw, ref, parts in work:
        s = tpx.Stream(max(len(p) for p in parts), **kw)
        h = np.concatenate([s.process(p, flush=(i == len(parts) - 1))[0]
                            for i, p in enumerate(parts)])
        assert_hits_match(h, ref)
        alone.append(h)
        s.close()
    # device inputs and outputs prepared up front; each thread only launches
    streams = [torch.cuda.Stream() for _ in work]
    objs, dev, outs = [], [], []
    for kw, ref, parts in work:
        objs.append(tpx.Stream(max(len(p) for p in parts), **kw))
        dev.append([torch.from_numpy(p.view(np.int64)).cuda() for p in parts])
        outs.append([torch.empty((max(len(p), 1024), 48), dtype=torch.uint8, device="cuda")
                     for p in parts])
    torch.cuda.synchronize()
    counts = [[None] * len(d) for d in dev]
    errors = []

    def drive(k):
        try:
            with torch.cuda.stream(streams[k]):
                for i, (pk, hb) in enumerate(zip(dev[k], outs[k])):
                    rc, n, _ = objs[k].process_raw(pk, i == len(dev[k]) - 1, hb, hb.shape[0])
                    if rc != 0:
                        raise RuntimeError(f"stream {k} chunk {i}: status {rc}")
                    counts[k][i] = n
        except Exception as e:  # reported by the main thread
            errors.append(e)

    th = [threading.Thread(target=drive, args=(k,)) for k in range(len(work))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for k in range(len(work)):
        h = np.concatenate([tpx.hits_to_numpy(hb, n) for hb, n in zip(outs[k], counts[k])])
        assert h.tobytes() == alone[k].tobytes()
        objs[k].close()


def test_stream_out_of_order_takes_general_path(tpx, orc):
    """A kept pixel of one shot reported after pixels of the next shot: the
    events are not in shot order and the general sorting path must give the
    oracle's result."""
    w = synth.make_config("c1", n_shots=60)
    pk = w.packets.copy()
    kept = np.nonzero(w.kept_mask())[0]
    i = kept[np.argmax(w.shot[kept] == 10)]          # first kept pixel of shot 10
    j = kept[np.argmax(w.shot[kept] == 12)]          # after trigger 12 in the stream
    moved = np.concatenate([pk[:i], pk[i + 1:j + 1], pk[i:i + 1], pk[j + 1:]])
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(moved, **kw)
    s = tpx.Stream(moved.size, **kw)
    h, _ = s.process(moved, flush=True)
    assert s.fallback_count == 1
    assert_hits_match(h, ref)


def test_stream_out_of_order_at_scale(tpx, orc):
    """Out-of-order pixels in a 300-shot c2 stream (about 190,000 events):
    the general path sorts every event by shot with the 4-bit radix sort
    (several 4,096-pair blocks and five passes) and must give the oracle's
    hits."""
    w = synth.make_config("c2", n_shots=300)
    pk = w.packets.copy()
    kept = np.nonzero(w.kept_mask())[0]
    moves = []
    for a_shot, b_shot in ((10, 12), (100, 101), (250, 254)):
        moves.append((int(kept[np.argmax(w.shot[kept] == a_shot)]),
                      int(kept[np.argmax(w.shot[kept] == b_shot)])))
    for i, j in sorted(moves, reverse=True):      # later moves first: indices stay valid
        pk = np.concatenate([pk[:i], pk[i + 1:j + 1], pk[i:i + 1], pk[j + 1:]])
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(pk, **kw)
    s = tpx.Stream(pk.size, **kw)
    h, _ = s.process(pk, flush=True)
    assert s.fallback_count == 1
    assert_hits_match(h, ref)


def test_stream_resume_from_checkpoint(tpx, orc):
    w = synth.make_config("c5", n_shots=80)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    half = w.n_packets // 2
    a = tpx.Stream(w.n_packets, **kw)
    h1, _ = a.process(w.packets[:half])
    blob = a.get_state()
    a.close()
    b = tpx.Stream(w.n_packets, **kw)
    b.set_state(blob)
    h2, _ = b.process(w.packets[half:], flush=True)
    assert_hits_match(np.concatenate([h1, h2]), ref)


def test_deterministic(tpx):
    w = synth.make_config("c2", n_shots=200)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    outs = [tpx.process_stream(w.packets, **kw)[0].tobytes() for _ in range(5)]
    assert all(o == outs[0] for o in outs)


# ---------------------------------------------------------------- centroid
def test_centroid_given_labels(tpx, orc):
    w = synth.make_config("c1", n_shots=500)
    r = orc.process(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    e = r["events"]
    d = tpx.to_device_events(e)
    import torch
    lab = torch.from_numpy(r["labels"].astype(np.uint32).view(np.int32)).cuda()
    h = tpx.centroid(d, lab, r["trig"])
    assert_hits_match(h, r["hits"])
    # the same with events out of shot order
    rng = np.random.default_rng(3)
    perm = rng.permutation(e["x"].size)
    inv = np.argsort(perm)
    ep = {k: v[perm] for k, v in e.items()}
    lp = inv[r["labels"][perm].astype(np.int64)]
    # relabel so that every label is the smallest member index after the permutation
    mins = {}
    for i, l in enumerate(lp.tolist()):
        mins[l] = min(mins.get(l, i), i)
    lp2 = np.array([mins[l] for l in lp.tolist()], np.uint32)
    href = orc.centroid(ep["x"], ep["y"], ep["tot"], ep["shot"], ep["toa"], lp2.astype(np.uint64),
                        r["trig"])
    h2 = tpx.centroid(tpx.to_device_events(ep), torch.from_numpy(lp2.view(np.int32)).cuda(),
                      r["trig"])
    assert_hits_match(h2, href)


def test_walk_table(tpx, orc):
    import torch
    w = synth.make_config("c1", n_shots=300)
    tot = np.arange(1024)
    walk32 = (180.0 / (tot + 9.0) - 0.4).astype(np.float32)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, walk_ns=walk32.astype(np.float64), **kw)
    lut = torch.from_numpy(walk32).cuda()
    h, _ = tpx.process_stream(w.packets, walk_lut_ns=lut, **kw)
    assert_hits_match(h, ref)


# ---------------------------------------------------------------- ABI errors
def test_abi_errors(tpx):
    import torch
    w = synth.make_config("c1", n_shots=50)
    s = tpx.Stream(w.n_packets)
    with pytest.raises(tpx.TpxError) as e:
        s.process(w.packets, flush=True, hit_cap=10)
    assert e.value.rc == tpx.ECAPACITY
    h, _ = s.process(w.packets, flush=True)          # state unchanged: retry works
    assert h.size > 10
    # triggers going back in time
    bad = synth.encode_tdc(np.array([5000, 1000]), np.array([0, 1]))
    s2 = tpx.Stream(16)
    with pytest.raises(tpx.TpxError) as e:
        s2.process(bad, flush=True)
    assert e.value.rc == tpx.ESTREAM
    with pytest.raises(tpx.TpxError) as e:
        s2.process(np.zeros(17, np.uint64))
    assert e.value.rc == tpx.EINVAL
    ev = tpx.to_device_events(dict(x=np.array([300], np.uint16), y=np.array([0], np.uint16),
                                   tot=np.array([1], np.uint16), shot=np.array([0], np.uint32),
                                   toa=np.array([0], np.uint64)))
    with pytest.raises(tpx.TpxError) as e:
        tpx.cluster(ev)
    assert e.value.rc == tpx.EINVAL
    torch.cuda.synchronize()
