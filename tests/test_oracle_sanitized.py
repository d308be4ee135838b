"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(tests/sanitize/oracle_main.c, a test-side driver that compiles the oracle's
C source into an executable): on decoded workloads, a walk table and edge
streams it must run clean and return exactly the hits of the ordinary build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sanitize", "oracle_main.c")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asan") / "oracle_sanitized")
    r = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        SRC, "-o", out, "-lm"], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("gcc without sanitizer runtimes")
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _run(exe, tmp_path, packets, walk=None):
    pk = tmp_path / "pk.bin"
    pk.write_bytes(np.ascontiguousarray(packets, np.uint64).tobytes())
    args = [exe, str(pk), str(tmp_path / "hits.bin"), str(tmp_path / "max.bin")]
    if walk is not None:
        wf = tmp_path / "walk.bin"
        wf.write_bytes(np.ascontiguousarray(walk, np.float64).tobytes())
        args.append(str(wf))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run(args, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    hits = np.frombuffer((tmp_path / "hits.bin").read_bytes(), oracle.HIT_DTYPE)
    maxima = np.frombuffer((tmp_path / "max.bin").read_bytes(), oracle.HIT_DTYPE)
    return hits, maxima


def _reference(orc, packets, walk=None):
    hits, _ = orc.run(packets, walk_ns=walk)
    d = orc.decode(packets)
    e = d["events"]
    mx = orc.local_maxima(e["x"], e["y"], e["tot"], e["shot"], e["toa"], d["trig"],
                          walk_ns=walk)
    return hits, mx


@pytest.mark.parametrize("name,shots", [("c1", 300), ("c3", 40)])
def test_sanitized_oracle_matches(exe, orc, tmp_path, name, shots):
    w = synth.make_config(name, n_shots=shots)
    assert w.pix_epoch0 == 0 and w.tdc_epoch0 == 0
    hits, mx = _run(exe, tmp_path, w.packets)
    rh, rm = _reference(orc, w.packets)
    assert hits.tobytes() == rh.tobytes()
    assert mx.tobytes() == rm.tobytes()


def test_sanitized_oracle_walk_and_edges(exe, orc, tmp_path):
    """A walk table; then the degenerate streams: empty, triggers only,
    pixels before any trigger, a single pixel."""
    w = synth.make_config("c1", n_shots=120)
    tot = np.arange(1024)
    walk = 180.0 / (tot + 9.0) - 0.4
    hits, mx = _run(exe, tmp_path, w.packets, walk)
    rh, rm = _reference(orc, w.packets, walk)
    assert hits.tobytes() == rh.tobytes()
    assert mx.tobytes() == rm.tobytes()
    trig = np.array([100_000, 100_000 + synth.SHOT_PERIOD_TICKS])
    cases = [np.zeros(0, np.uint64),
             synth.encode_tdc(trig, [0, 1]),
             synth.encode_pixels([3], [4], [10], [50_000]),
             np.concatenate([synth.encode_tdc(trig[:1], [0]),
                             synth.encode_pixels([255], [255], [0], [trig[0] + 5])])]
    for pk in cases:
        hits, mx = _run(exe, tmp_path, pk)
        rh, rm = _reference(orc, pk)
        assert hits.tobytes() == rh.tobytes()
        assert mx.tobytes() == rm.tobytes()
