"""Host emulation of libtpx's kernels (test infrastructure): build.py
compiles the library's HIP sources for the CPU against hip_emu.h with the
address and undefined-behaviour sanitizers; run_cluster / run_stream call the
resulting executable through files."""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

from . import build as _build

HIT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("tof_ns", "<f4"), ("npix", "<u4"),
                      ("shot", "<u8"), ("label", "<u8"), ("toa_first", "<u8"),
                      ("tot_sum", "<u4"), ("flags", "<u4")])


def _env(preempt, seed):
    env = dict(os.environ)
    env["EMU_PREEMPT"] = str(int(preempt))
    env["EMU_SEED"] = str(int(seed))
    env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def _run(mode, blob, preempt, seed, timeout):
    exe = _build.build()
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as f:
            f.write(blob)
        r = subprocess.run([exe, mode, fin, fout], env=_env(preempt, seed), capture_output=True,
                           text=True, timeout=timeout)
        if r.returncode != 0:
            raise RuntimeError(f"emulation run failed (rc {r.returncode}):\n{r.stderr[-4000:]}")
        with open(fout, "rb") as f:
            return f.read(), r.stderr


def _errors(buf, off):
    n = int(np.frombuffer(buf, np.uint64, 1, off)[0])
    return buf[off + 8: off + 8 + n].decode()


def run_cluster(ev, dxy=1, dt_ticks=128, preempt=0, seed=1, timeout=600):
    """tpx_cluster on event arrays; returns (status, n_clusters, labels,
    emulator findings)."""
    n = len(ev["x"])
    blob = b"".join([np.array([n], np.uint64).tobytes(), np.array([dxy, dt_ticks], np.uint32).tobytes(),
                     np.asarray(ev["x"], np.uint16).tobytes(), np.asarray(ev["y"], np.uint16).tobytes(),
                     np.asarray(ev["tot"], np.uint16).tobytes(),
                     np.asarray(ev["shot"], np.uint32).tobytes(),
                     np.asarray(ev["toa"], np.uint64).tobytes()])
    out, _ = _run("cluster", blob, preempt, seed, timeout)
    st = int(np.frombuffer(out, np.int32, 1, 0)[0])
    nc = int(np.frombuffer(out, np.uint64, 1, 4)[0])
    lab = np.frombuffer(out, np.uint32, n, 12).copy()
    return st, nc, lab, _errors(out, 12 + 4 * n)


def run_stream(packets, chunk, pix_epoch0=0, tdc_epoch0=0, q=0, kernel=0, persistent=1,
               preempt=0, seed=1, timeout=600):
    """tpx_process_stream over the packets in chunks of `chunk` words, or of
    the sizes in a list (flush on the last),
    with the given clustering kernel (-1 staged, >= 0 a fused variant) and
    the persistent launch of small chunks on or off; returns (status, hits,
    emulator findings)."""
    pk = np.ascontiguousarray(packets, dtype=np.uint64)
    sizes = b""
    if not np.isscalar(chunk):  # a list of chunk sizes
        sizes = np.array([len(chunk)] + list(chunk), np.uint64).tobytes()
        chunk = 0
    blob = b"".join([np.array([pk.size, chunk], np.uint64).tobytes(),
                     np.array([pix_epoch0, tdc_epoch0], np.int64).tobytes(),
                     np.array([q], np.uint32).tobytes(),
                     np.array([kernel, persistent], np.int32).tobytes(),
                     sizes, pk.tobytes()])
    out, _ = _run("stream", blob, preempt, seed, timeout)
    st = int(np.frombuffer(out, np.int32, 1, 0)[0])
    nh = int(np.frombuffer(out, np.uint64, 1, 4)[0])
    hits = np.frombuffer(out, HIT_DTYPE, nh, 12).copy()
    return st, hits, _errors(out, 12 + HIT_DTYPE.itemsize * nh)
