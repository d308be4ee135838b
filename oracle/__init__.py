"""Oracle for the TimePix3 VMI hot path (decode, unwrap, shot assignment with
ToF cut, connected-component clustering, ToT-weighted centroids).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports or
loads anything from here.  The arithmetic lives in ``tpx_oracle.c`` (plain,
single-threaded C); this module only builds it with gcc and marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ECAPACITY, ESTREAM, ENOMEM = 0, -1, -2, -3, -5

DEFAULTS = dict(dxy=1, dt_ticks=128, tof_max_ticks=64_000, trig_subtype=0xF,
                jump_ticks=12_800_000_000, pix_epoch0=0, tdc_epoch0=0)


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"oracle {what} failed with status {rc}")
        self.rc = rc


class Params(ctypes.Structure):
    _fields_ = [("dxy", ctypes.c_uint32), ("dt_ticks", ctypes.c_uint32),
                ("tof_max_ticks", ctypes.c_uint32), ("trig_subtype", ctypes.c_uint32),
                ("jump_ticks", ctypes.c_uint64), ("pix_epoch0", ctypes.c_int64),
                ("tdc_epoch0", ctypes.c_int64), ("walk_ns", ctypes.c_void_p)]


STAT_FIELDS = ("n_packets", "n_pixels", "n_tdc", "n_other", "n_pre_trigger", "n_tof_cut",
               "n_events", "n_hits", "n_pix_wraps", "n_pix_backjumps", "n_tdc_wraps",
               "n_tdc_backjumps")


class Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STAT_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in STAT_FIELDS}


HIT_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("tof_ns", "<f8"), ("shot", "<u8"),
                      ("label", "<u8"), ("toa_first", "<u8"), ("npix", "<u8"),
                      ("tot_sum", "<u8"), ("flags", "<u4"), ("pad", "<u4")])


def build(force=False, extra_flags=()):
    """Compile tpx_oracle.c into liboracle.so with gcc (single-threaded -O2)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC) \
            and not extra_flags:
        return _LIB
    out = _LIB if not extra_flags else os.path.join(
        _HERE, "liboracle_%d.so" % (abs(hash(tuple(extra_flags))) % 10**8))
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                           *extra_flags, _SRC, "-o", tmp])
    os.replace(tmp, out)
    return out


_lib = None


def _load(path=None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        _lib = _bind(ctypes.CDLL(build()))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    S = ctypes.c_size_t
    lib.orc_decode_word.argtypes = [ctypes.c_uint64, ctypes.c_uint32] + [P] * 5
    lib.orc_decode.argtypes = [P, S, P, P, P, P, P, P, S, P, P, S, P, P, P]
    lib.orc_cluster.argtypes = [S, P, P, P, P, ctypes.c_uint32, ctypes.c_uint32, P, P]
    lib.orc_centroid.argtypes = [S, P, P, P, P, P, P, P, S, P, P, S, P]
    lib.orc_local_maxima.argtypes = [S, P, P, P, P, P, ctypes.c_uint32, ctypes.c_uint32, P, S,
                                     P, P, S, P]
    lib.orc_run.argtypes = [P, S, P, P, S, P, P]
    for f in ("orc_decode_word", "orc_decode", "orc_cluster", "orc_centroid", "orc_run"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def make_params(**kw):
    d = dict(DEFAULTS)
    walk = kw.pop("walk_ns", None)
    d.update(kw)
    p = Params(**d)
    keep = None
    if walk is not None:
        keep = np.ascontiguousarray(walk, dtype=np.float64)
        assert keep.size == 1024
        p.walk_ns = keep.ctypes.data
    return p, keep


class Oracle:
    """Thin marshalling layer over one loaded copy of liboracle.so."""

    def __init__(self, lib_path=None):
        self.lib = _load(lib_path)

    def decode_word(self, w, trig_subtype=0xF):
        k, x, y, tot = (ctypes.c_uint32() for _ in range(4))
        raw = ctypes.c_uint64()
        self.lib.orc_decode_word(ctypes.c_uint64(int(w)), trig_subtype, ctypes.byref(k),
                                 ctypes.byref(x), ctypes.byref(y), ctypes.byref(tot),
                                 ctypes.byref(raw))
        return int(k.value), int(x.value), int(y.value), int(tot.value), int(raw.value)

    def decode(self, packets, want_times=False, **kw):
        pk = np.ascontiguousarray(packets, dtype=np.uint64)
        n = pk.size
        p, keep = make_params(**kw)
        cap = max(n, 1)
        ev = dict(x=np.empty(cap, np.uint16), y=np.empty(cap, np.uint16),
                  tot=np.empty(cap, np.uint16), shot=np.empty(cap, np.uint32),
                  toa=np.empty(cap, np.uint64))
        trig = np.empty(cap, np.uint64)
        t_out = np.empty(cap, np.int64) if want_times else None
        ne, nt = ctypes.c_size_t(), ctypes.c_size_t()
        st = Stats()
        rc = self.lib.orc_decode(_ptr(pk), n, ctypes.byref(p), _ptr(ev["x"]), _ptr(ev["y"]),
                                 _ptr(ev["tot"]), _ptr(ev["shot"]), _ptr(ev["toa"]), cap,
                                 ctypes.byref(ne), _ptr(trig), cap, ctypes.byref(nt),
                                 _ptr(t_out), ctypes.byref(st))
        del keep
        if rc != OK:
            raise OracleError(rc, "decode")
        ev = {k: v[:ne.value].copy() for k, v in ev.items()}
        out = dict(events=ev, trig=trig[:nt.value].copy(), stats=st.as_dict())
        if want_times:
            out["t"] = t_out[:n].copy()
        return out

    def cluster(self, x, y, shot, toa, dxy=1, dt_ticks=128):
        x = np.ascontiguousarray(x, np.uint16)
        y = np.ascontiguousarray(y, np.uint16)
        shot = np.ascontiguousarray(shot, np.uint32)
        toa = np.ascontiguousarray(toa, np.uint64)
        n = x.size
        lab = np.empty(max(n, 1), np.uint64)
        nc = ctypes.c_size_t()
        rc = self.lib.orc_cluster(n, _ptr(x), _ptr(y), _ptr(shot), _ptr(toa), dxy, dt_ticks,
                                  _ptr(lab), ctypes.byref(nc))
        if rc != OK:
            raise OracleError(rc, "cluster")
        return lab[:n].copy(), int(nc.value)

    def centroid(self, x, y, tot, shot, toa, labels, trig, walk_ns=None):
        x = np.ascontiguousarray(x, np.uint16)
        y = np.ascontiguousarray(y, np.uint16)
        tot = np.ascontiguousarray(tot, np.uint16)
        shot = np.ascontiguousarray(shot, np.uint32)
        toa = np.ascontiguousarray(toa, np.uint64)
        labels = np.ascontiguousarray(labels, np.uint64)
        trig = np.ascontiguousarray(trig, np.uint64)
        walk = None if walk_ns is None else np.ascontiguousarray(walk_ns, np.float64)
        n = x.size
        hits = np.empty(max(n, 1), HIT_DTYPE)
        nh = ctypes.c_size_t()
        rc = self.lib.orc_centroid(n, _ptr(x), _ptr(y), _ptr(tot), _ptr(shot), _ptr(toa),
                                   _ptr(labels), _ptr(trig), trig.size, _ptr(walk),
                                   _ptr(hits), max(n, 1), ctypes.byref(nh))
        if rc != OK:
            raise OracleError(rc, "centroid")
        return hits[:nh.value].copy()

    def local_maxima(self, x, y, tot, shot, toa, trig, dxy=1, dt_ticks=128, walk_ns=None):
        """The paper's hits: local maxima of ToT over the neighbourhood and
        Eq. (9) over each one's row of A (see orc_local_maxima)."""
        x = np.ascontiguousarray(x, np.uint16)
        y = np.ascontiguousarray(y, np.uint16)
        tot = np.ascontiguousarray(tot, np.uint16)
        shot = np.ascontiguousarray(shot, np.uint32)
        toa = np.ascontiguousarray(toa, np.uint64)
        trig = np.ascontiguousarray(trig, np.uint64)
        walk = None if walk_ns is None else np.ascontiguousarray(walk_ns, np.float64)
        n = x.size
        hits = np.empty(max(n, 1), HIT_DTYPE)
        nh = ctypes.c_size_t()
        rc = self.lib.orc_local_maxima(n, _ptr(x), _ptr(y), _ptr(tot), _ptr(shot), _ptr(toa),
                                       int(dxy), int(dt_ticks), _ptr(trig), trig.size, _ptr(walk),
                                       _ptr(hits), max(n, 1), ctypes.byref(nh))
        if rc != OK:
            raise OracleError(rc, "local_maxima")
        return hits[:nh.value].copy()

    def run(self, packets, **kw):
        """Whole path over one stream; returns (hits, stats)."""
        pk = np.ascontiguousarray(packets, dtype=np.uint64)
        p, keep = make_params(**kw)
        cap = max(pk.size // 2, 16)
        while True:
            hits = np.empty(cap, HIT_DTYPE)
            nh = ctypes.c_size_t()
            st = Stats()
            rc = self.lib.orc_run(_ptr(pk), pk.size, ctypes.byref(p), _ptr(hits), cap,
                                  ctypes.byref(nh), ctypes.byref(st))
            if rc == ECAPACITY and nh.value > cap:
                cap = nh.value
                continue
            break
        del keep
        if rc != OK:
            raise OracleError(rc, "run")
        return hits[:nh.value].copy(), st.as_dict()

    def process(self, packets, **kw):
        """Step by step (decode, cluster, centroid) with every intermediate."""
        dec = self.decode(packets, **kw)
        ev = dec["events"]
        labels, nc = self.cluster(ev["x"], ev["y"], ev["shot"], ev["toa"],
                                  kw.get("dxy", 1), kw.get("dt_ticks", 128))
        hits = self.centroid(ev["x"], ev["y"], ev["tot"], ev["shot"], ev["toa"], labels,
                             dec["trig"], kw.get("walk_ns"))
        dec["labels"] = labels
        dec["hits"] = hits
        dec["stats"]["n_hits"] = int(hits.size)
        return dec


_default = None


def get():
    global _default
    if _default is None:
        _default = Oracle()
    return _default
