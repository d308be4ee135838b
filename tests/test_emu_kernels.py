"""The library's kernels run on the CPU under the host emulation
(tests/emu): workgroup barriers are counting barriers that must be reached by
every thread at the same call, cross-lane operations complete per wave, the
scheduler interleaves threads at atomics (seeded), and every global and LDS
access is checked by AddressSanitizer.  Results must equal the oracle's and
the emulator must report nothing."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from cases import tiny_cluster_case

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def emu():
    from tests import emu as e
    e._build.build()
    return e


def test_selftest_reports_planted_mistakes(emu):
    """Each planted synchronisation mistake (a barrier skipped by `continue`
    in a ticket loop, threads that return before a barrier, a wait on a later
    workgroup, a barrier inside a thread-dependent branch) is reported."""
    exe = emu._build.build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe, "selftest"], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if ": reported" in l or "NOT REPORTED" in l]
    assert len(lines) == 4, r.stdout
    assert all(l.endswith(": reported") for l in lines), r.stdout


@pytest.mark.parametrize("preempt", [0, 50, 300])
def test_cluster_seed0_input(emu, orc, preempt):
    """The tiny event-mode input that once hung an earlier cluster kernel
    (61 events, 3 unsorted shots, radius 2, time window 1 tick) on the
    current kernels: exact labels, no barrier divergence, no deadlock, no
    out-of-bounds access, for several thread interleavings."""
    ev, dxy, dt = tiny_cluster_case(0)
    ref, nref = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"], dxy=dxy, dt_ticks=dt)
    st, nc, lab, errs = emu.run_cluster(ev, dxy, dt, preempt=preempt, seed=7 + preempt)
    assert errs == ""
    assert st == 0
    assert nc == nref
    assert np.array_equal(lab.astype(np.uint64), ref)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6, 9, 12])
def test_cluster_tiny(emu, orc, seed):
    ev, dxy, dt = tiny_cluster_case(seed)
    ref, nref = orc.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"], dxy=dxy, dt_ticks=dt)
    st, nc, lab, errs = emu.run_cluster(ev, dxy, dt, preempt=100, seed=seed)
    assert errs == ""
    assert st == 0 and nc == nref
    assert np.array_equal(lab.astype(np.uint64), ref)


@pytest.mark.parametrize("chunk", [1 << 20, 1500])
def test_stream_c1(emu, orc, chunk):
    """The stream path (decode -> cluster -> centroid with the carry) on 40
    shots of the small workload, whole and in chunks of 1,500 packets."""
    w = synth.make_config("c1", n_shots=40)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    st, hits, errs = emu.run_stream(w.packets, chunk, preempt=100, **kw)
    assert errs == ""
    assert st == 0
    assert hits.size == ref.size
    for f in ("shot", "label", "npix", "tot_sum", "toa_first", "flags"):
        assert np.array_equal(hits[f].astype(np.uint64), ref[f].astype(np.uint64)), f
    assert np.abs(hits["x"] - ref["x"]).max() <= 1e-4
    assert np.abs(hits["y"] - ref["y"]).max() <= 1e-4
    assert np.abs(hits["tof_ns"] - ref["tof_ns"]).max() <= 0.1


def _assert_hits(hits, ref):
    assert hits.size == ref.size
    for f in ("shot", "label", "npix", "tot_sum", "toa_first", "flags"):
        assert np.array_equal(hits[f].astype(np.uint64), ref[f].astype(np.uint64)), f
    assert np.abs(hits["x"] - ref["x"]).max(initial=0) <= 1e-4
    assert np.abs(hits["y"] - ref["y"]).max(initial=0) <= 1e-4
    assert np.abs(hits["tof_ns"] - ref["tof_ns"]).max(initial=0) <= 0.1


@pytest.mark.parametrize("kernel", [-1, 0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("name,shots,chunk", [("c1", 30, 1500), ("c3", 25, 30000)])
def test_stream_kernels(emu, orc, kernel, name, shots, chunk):
    """Every clustering kernel of the stream path (the staged pair and each
    fused variant: slot lists, forest and atomic-minimum joins, moments, staged hits
    and their compaction; the routed variant's deferred segments and its
    persistent launch) on the small and the uneven-shot workloads, whole and
    in chunks."""
    w = synth.make_config(name, n_shots=shots)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    for ch in (1 << 22, chunk):
        st, hits, errs = emu.run_stream(w.packets, ch, kernel=kernel, persistent=0, preempt=100,
                                        seed=11 + kernel, **kw)
        assert errs == ""
        assert st == 0
        _assert_hits(hits, ref)


def test_stream_out_of_order_sort(emu, orc):
    """Kept pixels reported after pixels of later shots: the stream takes the
    general path, whose stable 4-bit radix sort by shot (count, prefix,
    scatter per 4,096 pairs) must reproduce the oracle's shot order."""
    w = synth.make_config("c1", n_shots=60)
    pk = w.packets.copy()
    kept = np.nonzero(w.kept_mask())[0]
    moves = [(int(kept[np.argmax(w.shot[kept] == a)]), int(kept[np.argmax(w.shot[kept] == b)]))
             for a, b in ((10, 12), (30, 33), (45, 46))]
    for i, j in sorted(moves, reverse=True):      # later moves first: indices stay valid
        pk = np.concatenate([pk[:i], pk[i + 1:j + 1], pk[i:i + 1], pk[j + 1:]])
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(pk, **kw)
    st, hits, errs = emu.run_stream(pk, 1 << 22, kernel=1, persistent=0, preempt=100, seed=9, **kw)
    assert errs == ""
    assert st == 0
    _assert_hits(hits, ref)


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("name,shots,chunks", [("c1", 60, (1500, 40000)), ("c5", 8, (8192, 3000)),
                                               ("c3", 12, (30000, 1 << 22))])
def test_stream_persistent_launch(emu, orc, persistent, name, shots, chunks):
    """The fast path of small chunks in one persistent launch (work items by
    ticket in dependency order: tile summaries, the prefix over tiles,
    assignment, placement, grouping, segments, carry, compaction) against the
    separate launches' results and the oracle, in chunks that split shots,
    with and without it."""
    w = synth.make_config(name, n_shots=shots)
    kw = dict(pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    ref, _ = orc.run(w.packets, **kw)
    # fixed sizes, then uneven sizes that end with an empty flushing chunk
    rng = np.random.default_rng(7)
    uneven = list(rng.integers(500, 20000, w.n_packets // 5000 + 2)) + [w.n_packets, 0]
    for ch in list(chunks) + [uneven]:
        st, hits, errs = emu.run_stream(w.packets, ch, kernel=1, persistent=persistent,
                                        preempt=100, seed=3 + persistent, **kw)
        assert errs == ""
        assert st == 0
        _assert_hits(hits, ref)


@pytest.mark.parametrize("kernel,case", [(k, c) for k in (0, 4, 5)
                                         for c in ("iso1500", "iso3000", "square")]
                         + [(5, "iso9000")])
def test_stream_fused_capacity_paths(emu, orc, kernel, case):
    """The fused kernel's fallbacks: more components than the LDS
    accumulators hold (1,500 isolated pixels), a segment beyond the LDS event
    capacity (3,000; global-memory lists and unions, or the routed variant's
    persistent launch), one component of 7,200 pixels at ToT 1023 (moments
    of a large segment), and for the routed variant a segment beyond its
    persistent launch's 8,192 events (9,000 isolated pixels)."""
    from cases import big_component_packets, many_components_packets
    pk = {"iso1500": lambda: many_components_packets(1500),
          "iso3000": lambda: many_components_packets(3000),
          "iso9000": lambda: many_components_packets(9000),
          "square": lambda: big_component_packets(side=60, layers=2)}[case]()
    ref, _ = orc.run(pk)
    st, hits, errs = emu.run_stream(pk, 1 << 22, kernel=kernel, persistent=0, preempt=100, seed=5)
    assert errs == ""
    assert st == 0
    _assert_hits(hits, ref)


@pytest.mark.parametrize("kernel,seed", [(1, 0), (1, 1), (0, 2), (4, 3), (5, 4)])
def test_stream_shuffled_shapes(emu, orc, kernel, seed):
    """Connected shapes whose pixels arrive in a random order (a serpentine
    path of 819 pixels, a 20 x 20 square, a ring): the smallest-neighbour
    forest has many local minima, so the fused kernel's joins chain and
    displace parents; every shape stays one hit under seeded interleavings
    of the LDS atomics."""
    from cases import shuffled_shapes_packets
    pk = shuffled_shapes_packets(seed)
    ref, _ = orc.run(pk)
    assert sorted(ref["npix"])[-3:] == [88, 400, 819]
    st, hits, errs = emu.run_stream(pk, 1 << 22, kernel=kernel, persistent=0, preempt=100,
                                    seed=11 + seed)
    assert errs == ""
    assert st == 0
    _assert_hits(hits, ref)
