"""Python binding of libtpx, the MI355X (gfx950) TimePix3 VMI hot path.

Argument marshalling only: every step of the method (decode, unwrap, shot
assignment, clustering, centroids) runs in the library's HIP kernels, reached
through the C ABI declared in include/tpx.h.  PyTorch supplies device memory
and the current HIP stream.  There is no CPU fallback: if libtpx.so is missing
or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpx.so")

OK, EINVAL, ECAPACITY, ESTREAM, EHIP, ENOMEM, EINTERNAL = 0, -1, -2, -3, -4, -5, -6


class TpxError(RuntimeError):
    def __init__(self, rc, what, detail=""):
        super().__init__(f"{what}: status {rc} ({detail})")
        self.rc = rc


class Params(ctypes.Structure):
    _fields_ = [("dxy", ctypes.c_uint32), ("dt_ticks", ctypes.c_uint32),
                ("tof_max_ticks", ctypes.c_uint32), ("trig_subtype", ctypes.c_uint32),
                ("jump_ticks", ctypes.c_uint64), ("pix_epoch0", ctypes.c_int64),
                ("tdc_epoch0", ctypes.c_int64), ("close_slack_ticks", ctypes.c_uint64),
                ("walk_lut_ns", ctypes.c_void_p)]


class Events(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("tot", ctypes.c_void_p),
                ("shot", ctypes.c_void_p), ("toa", ctypes.c_void_p)]


STAT_FIELDS = ("n_packets", "n_pixels", "n_tdc", "n_other", "n_pre_trigger", "n_tof_cut",
               "n_events", "n_hits", "n_pix_wraps", "n_pix_backjumps", "n_tdc_wraps",
               "n_tdc_backjumps", "n_late_drop")


class Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STAT_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in STAT_FIELDS}


class UnwrapState(ctypes.Structure):
    _fields_ = [("pix_epoch", ctypes.c_int64), ("tdc_epoch", ctypes.c_int64),
                ("pix_last_raw", ctypes.c_uint64), ("tdc_last_raw", ctypes.c_uint64),
                ("pix_has_last", ctypes.c_uint32), ("tdc_has_last", ctypes.c_uint32),
                ("trig_base", ctypes.c_uint64), ("last_trig_toa", ctypes.c_uint64),
                ("has_last_trig", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


HIT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("tof_ns", "<f4"), ("npix", "<u4"),
                      ("shot", "<u8"), ("label", "<u8"), ("toa_first", "<u8"),
                      ("tot_sum", "<u4"), ("flags", "<u4")])
assert HIT_DTYPE.itemsize == 48

EXPORTS = ("tpx_params_default", "tpx_unwrap_state_init", "tpx_workspace_bytes", "tpx_decode",
           "tpx_cluster", "tpx_centroid", "tpx_local_maxima", "tpx_stream_create",
           "tpx_process_stream",
           "tpx_stream_get_state", "tpx_stream_set_state", "tpx_stream_destroy",
           "tpx_status_str", "tpx_last_error", "tpx_stream_fallback_count",
           "tpx_stream_set_timing", "tpx_stream_get_timing", "tpx_stream_stage_name",
           "tpx_service_create", "tpx_service_submit", "tpx_service_run", "tpx_service_destroy",
           "tpx_patch_workspace_bytes", "tpx_patches", "tpx_mlp_workspace_bytes",
           "tpx_mlp_forward", "tpx_mlp_grad", "tpx_mlp_adam", "tpx_mlp_refine",
           "tpx_stream_set_segment", "tpx_stream_get_segment", "tpx_stream_autotune",
           "tpx_stream_patch_workspace_bytes", "tpx_stream_patches", "tpx_stream_set_patches",
           "tpx_stream_kernel_count", "tpx_stream_kernel_name", "tpx_stream_set_kernel",
           "tpx_stream_get_kernel", "tpx_stream_set_persistent", "tpx_stream_get_persistent",
           "tpx_service_set_segment",
           "tpx_cluster_static", "tpx_cluster_static_max_events",
           "tpx_walk_fit", "tpx_walk_fit_workspace_bytes", "tpx_stream_device_bytes",
           "tpx_service_device_bytes", "tpx_service_replay", "tpx_server_create", "tpx_server_open",
           "tpx_server_submit", "tpx_server_run", "tpx_server_close", "tpx_server_free_bytes",
           "tpx_server_destroy")

_lib = None


def load(path=LIB_PATH):
    """Load libtpx.so and declare its signatures (no GPU needed for this)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2603_04942_amd/build.py")
    lib = ctypes.CDLL(path)
    P, S, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    lib.tpx_params_default.argtypes = [P]
    lib.tpx_params_default.restype = None
    lib.tpx_unwrap_state_init.argtypes = [P, P]
    lib.tpx_unwrap_state_init.restype = None
    lib.tpx_workspace_bytes.argtypes = [S, S]
    lib.tpx_workspace_bytes.restype = S
    lib.tpx_decode.argtypes = [P, S, P, P, Events, S, P, S, P, P, P, P, S, P]
    lib.tpx_cluster.argtypes = [Events, S, P, P, P, P, S, P]
    lib.tpx_cluster_static.argtypes = [Events, S, P, P, P, P]
    lib.tpx_cluster_static.restype = I
    lib.tpx_stream_device_bytes.argtypes = [P]
    lib.tpx_stream_device_bytes.restype = S
    lib.tpx_service_device_bytes.argtypes = [P]
    lib.tpx_service_device_bytes.restype = S
    lib.tpx_service_replay.argtypes = [P, P, S, S, ctypes.c_double, P, S, P, S, P, P, P]
    lib.tpx_service_replay.restype = I
    lib.tpx_server_create.argtypes = [P, S, ctypes.c_int, P]
    lib.tpx_server_create.restype = I
    lib.tpx_server_open.argtypes = [P, P, S, S, P, P]
    lib.tpx_server_open.restype = I
    lib.tpx_server_submit.argtypes = [P, ctypes.c_uint32, P, S, ctypes.c_int, P, P]
    lib.tpx_server_submit.restype = I
    lib.tpx_server_run.argtypes = [P, ctypes.c_uint32, ctypes.c_int, P, S, P, P, P]
    lib.tpx_server_run.restype = I
    lib.tpx_server_close.argtypes = [P, ctypes.c_uint32]
    lib.tpx_server_close.restype = I
    lib.tpx_server_free_bytes.argtypes = [P]
    lib.tpx_server_free_bytes.restype = S
    lib.tpx_server_destroy.argtypes = [P]
    lib.tpx_server_destroy.restype = None
    lib.tpx_walk_fit_workspace_bytes.argtypes = []
    lib.tpx_walk_fit_workspace_bytes.restype = S
    lib.tpx_walk_fit.argtypes = [Events, S, P, S, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                 P, P, P, P, P, S, P]
    lib.tpx_walk_fit.restype = I
    lib.tpx_cluster_static_max_events.argtypes = []
    lib.tpx_cluster_static_max_events.restype = S
    lib.tpx_centroid.argtypes = [Events, P, S, P, S, P, P, S, P, P, S, P]
    lib.tpx_local_maxima.argtypes = [Events, S, P, S, P, P, S, P, P, S, P]
    lib.tpx_stream_create.argtypes = [P, S, P]
    lib.tpx_service_create.argtypes = [P, S, S, P]
    lib.tpx_service_submit.argtypes = [P, P, S, ctypes.c_int, P, P]
    lib.tpx_service_run.argtypes = [P, ctypes.c_int, P, S, P, P, P, P]
    lib.tpx_service_destroy.argtypes = [P]
    lib.tpx_service_destroy.restype = None
    lib.tpx_process_stream.argtypes = [P, P, S, ctypes.c_int, P, S, P, P, P]
    lib.tpx_stream_get_state.argtypes = [P, P, P]
    lib.tpx_stream_set_state.argtypes = [P, P, S]
    lib.tpx_stream_destroy.argtypes = [P]
    lib.tpx_stream_destroy.restype = None
    lib.tpx_patch_workspace_bytes.argtypes = [S]
    lib.tpx_patch_workspace_bytes.restype = S
    lib.tpx_patches.argtypes = [Events, P, S, P, S, P, P, S, P]
    lib.tpx_mlp_workspace_bytes.argtypes = [S]
    lib.tpx_mlp_workspace_bytes.restype = S
    lib.tpx_mlp_forward.argtypes = [P, P, S, P, P, S, P]
    lib.tpx_mlp_grad.argtypes = [P, P, P, P, P, S, P, P, P, S, P]
    lib.tpx_mlp_adam.argtypes = [P, P, P, P, S, ctypes.c_uint64, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, P]
    lib.tpx_mlp_refine.argtypes = [P, P, S, P, P]
    for f in ("tpx_patches", "tpx_mlp_forward", "tpx_mlp_grad", "tpx_mlp_adam", "tpx_mlp_refine"):
        getattr(lib, f).restype = I
    lib.tpx_stream_set_segment.argtypes = [P, ctypes.c_uint32]
    lib.tpx_stream_set_segment.restype = I
    lib.tpx_stream_get_segment.argtypes = [P]
    lib.tpx_stream_get_segment.restype = ctypes.c_uint32
    lib.tpx_stream_autotune.argtypes = [P, P, S, ctypes.c_int, P, S, P, S, P, S, ctypes.c_int, P,
                                        P, P, P]
    lib.tpx_stream_autotune.restype = I
    lib.tpx_stream_kernel_count.argtypes = []
    lib.tpx_stream_kernel_count.restype = ctypes.c_int
    lib.tpx_stream_kernel_name.argtypes = [ctypes.c_int]
    lib.tpx_stream_kernel_name.restype = ctypes.c_char_p
    lib.tpx_stream_set_kernel.argtypes = [P, ctypes.c_int]
    lib.tpx_stream_set_kernel.restype = I
    lib.tpx_stream_get_kernel.argtypes = [P]
    lib.tpx_stream_get_kernel.restype = ctypes.c_int
    lib.tpx_service_set_segment.argtypes = [P, ctypes.c_uint32]
    lib.tpx_service_set_segment.restype = I
    lib.tpx_stream_set_persistent.argtypes = [P, ctypes.c_int]
    lib.tpx_stream_set_persistent.restype = I
    lib.tpx_stream_get_persistent.argtypes = [P]
    lib.tpx_stream_get_persistent.restype = ctypes.c_int
    lib.tpx_stream_set_patches.argtypes = [P, ctypes.c_int]
    lib.tpx_stream_set_patches.restype = I
    lib.tpx_stream_patch_workspace_bytes.argtypes = [S]
    lib.tpx_stream_patch_workspace_bytes.restype = S
    lib.tpx_stream_patches.argtypes = [P, P, S, P, P, S, P]
    lib.tpx_stream_patches.restype = I
    lib.tpx_status_str.argtypes = [I]
    lib.tpx_status_str.restype = ctypes.c_char_p
    lib.tpx_last_error.argtypes = []
    lib.tpx_last_error.restype = ctypes.c_char_p
    lib.tpx_stream_fallback_count.argtypes = [P]
    lib.tpx_stream_fallback_count.restype = ctypes.c_uint64
    lib.tpx_stream_set_timing.argtypes = [P, ctypes.c_int]
    lib.tpx_stream_set_timing.restype = I
    lib.tpx_stream_get_timing.argtypes = [P, P, S, P]
    lib.tpx_stream_get_timing.restype = I
    lib.tpx_stream_stage_name.argtypes = [S]
    lib.tpx_stream_stage_name.restype = ctypes.c_char_p
    for f in ("tpx_decode", "tpx_cluster", "tpx_centroid", "tpx_stream_create",
              "tpx_process_stream", "tpx_stream_get_state", "tpx_stream_set_state"):
        getattr(lib, f).restype = I
    _lib = lib
    return lib


def _check(rc, what):
    if rc != OK:
        lib = load()
        raise TpxError(rc, what, lib.tpx_last_error().decode())


def make_params(**kw):
    """tpx_params with the library defaults, overridden by keyword."""
    lib = load()
    p = Params()
    lib.tpx_params_default(ctypes.byref(p))
    walk = kw.pop("walk_lut_ns", None)
    for k, v in kw.items():
        setattr(p, k, v)
    if walk is not None:
        p.walk_lut_ns = walk.data_ptr()
    return p


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libtpx needs a visible GPU (no CPU fallback)")
    return torch


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(torch, a, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).view(dtype).to("cuda")


def _u64(torch, a):
    if isinstance(a, torch.Tensor):
        return a.to("cuda").contiguous().view(torch.int64)
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda")


def events_struct(ev):
    return Events(ev["x"].data_ptr(), ev["y"].data_ptr(), ev["tot"].data_ptr(),
                  ev["shot"].data_ptr(), ev["toa"].data_ptr())


def to_device_events(ev):
    """numpy/torch dict (x, y, tot u16; shot u32; toa u64) -> device tensors."""
    torch = _torch()
    return dict(x=_dev(torch, np.asarray(ev["x"], np.uint16).view(np.int16), torch.int16),
                y=_dev(torch, np.asarray(ev["y"], np.uint16).view(np.int16), torch.int16),
                tot=_dev(torch, np.asarray(ev["tot"], np.uint16).view(np.int16), torch.int16),
                shot=_dev(torch, np.asarray(ev["shot"], np.uint32).view(np.int32), torch.int32),
                toa=_u64(torch, np.asarray(ev["toa"], np.uint64)))


def hits_to_numpy(h, n):
    return h[:n].cpu().numpy().view(HIT_DTYPE).reshape(-1)


def workspace(n_packets, n_events):
    torch = _torch()
    nbytes = load().tpx_workspace_bytes(n_packets, n_events)
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def decode(packets, state=None, params=None, ev_cap=None, trig_cap=None, ws=None):
    """tpx_decode over one buffer of packets (device tensor or numpy uint64).
    Returns (events dict of device tensors, triggers, stats dict, state)."""
    torch = _torch()
    lib = load()
    pk = _u64(torch, packets)
    n = pk.numel()
    p = params or make_params()
    st = state or UnwrapState()
    if state is None:
        lib.tpx_unwrap_state_init(ctypes.byref(st), ctypes.byref(p))
    ev_cap = n if ev_cap is None else ev_cap
    trig_cap = n if trig_cap is None else trig_cap
    ev = dict(x=torch.empty(ev_cap, dtype=torch.int16, device="cuda"),
              y=torch.empty(ev_cap, dtype=torch.int16, device="cuda"),
              tot=torch.empty(ev_cap, dtype=torch.int16, device="cuda"),
              shot=torch.empty(ev_cap, dtype=torch.int32, device="cuda"),
              toa=torch.empty(ev_cap, dtype=torch.int64, device="cuda"))
    trig = torch.empty(max(trig_cap, 1), dtype=torch.int64, device="cuda")
    ws = workspace(n, 0) if ws is None else ws
    ne, nt = ctypes.c_size_t(), ctypes.c_size_t()
    stats = Stats()
    rc = lib.tpx_decode(_ptr(pk), n, ctypes.byref(p), ctypes.byref(st), events_struct(ev), ev_cap,
                        _ptr(trig), trig_cap, ctypes.byref(ne), ctypes.byref(nt),
                        ctypes.byref(stats), _ptr(ws), ws.numel(), _stream(torch))
    if rc == ECAPACITY:
        raise TpxError(rc, "tpx_decode", f"need {ne.value} events / {nt.value} triggers")
    _check(rc, "tpx_decode")
    ev = {k: v[:ne.value] for k, v in ev.items()}
    return ev, trig[:nt.value], stats.as_dict(), st


def cluster(ev, params=None, ws=None):
    """tpx_cluster: labels (int32 tensor; values are uint32 event indices)."""
    torch = _torch()
    lib = load()
    n = ev["x"].numel()
    p = params or make_params()
    labels = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    ws = workspace(0, n) if ws is None else ws
    nc = ctypes.c_size_t()
    rc = lib.tpx_cluster(events_struct(ev), n, ctypes.byref(p), _ptr(labels), ctypes.byref(nc),
                         _ptr(ws), ws.numel(), _stream(torch))
    _check(rc, "tpx_cluster")
    return labels[:n], int(nc.value)


def centroid(ev, labels, trig, params=None, hit_cap=None, ws=None):
    """tpx_centroid: numpy structured array of hits (HIT_DTYPE)."""
    torch = _torch()
    lib = load()
    n = ev["x"].numel()
    p = params or make_params()
    trig = _u64(torch, trig)
    hit_cap = n if hit_cap is None else hit_cap
    hits = torch.empty((max(hit_cap, 1), 48), dtype=torch.uint8, device="cuda")
    ws = workspace(0, n) if ws is None else ws
    nh = ctypes.c_size_t()
    rc = lib.tpx_centroid(events_struct(ev), _ptr(labels), n, _ptr(trig), trig.numel(),
                          ctypes.byref(p), _ptr(hits), hit_cap, ctypes.byref(nh), _ptr(ws),
                          ws.numel(), _stream(torch))
    if rc == ECAPACITY:
        raise TpxError(rc, "tpx_centroid", f"need {nh.value} hits")
    _check(rc, "tpx_centroid")
    return hits_to_numpy(hits, nh.value)


def local_maxima(ev, trig, params=None, hit_cap=None, ws=None):
    """tpx_local_maxima (the paper's local-maximum hits): numpy structured
    array of hits (HIT_DTYPE)."""
    torch = _torch()
    lib = load()
    n = ev["x"].numel()
    p = params or make_params()
    trig = _u64(torch, trig)
    hit_cap = n if hit_cap is None else hit_cap
    hits = torch.empty((max(hit_cap, 1), 48), dtype=torch.uint8, device="cuda")
    ws = workspace(0, n) if ws is None else ws
    nh = ctypes.c_size_t()
    rc = lib.tpx_local_maxima(events_struct(ev), n, _ptr(trig), trig.numel(), ctypes.byref(p),
                              _ptr(hits), hit_cap, ctypes.byref(nh), _ptr(ws), ws.numel(),
                              _stream(torch))
    if rc == ECAPACITY:
        raise TpxError(rc, "tpx_local_maxima", f"need {nh.value} hits or smaller shot groups")
    _check(rc, "tpx_local_maxima")
    return hits_to_numpy(hits, nh.value)


def local_maxima_raw(ev, trig, hits, hit_cap, ws, params=None):
    """Device-only tpx_local_maxima into a caller's hit buffer; returns
    (status, n_hits) without copying anything back."""
    torch = _torch()
    lib = load()
    p = params or make_params()
    nh = ctypes.c_size_t()
    rc = lib.tpx_local_maxima(events_struct(ev), ev["x"].numel(), _ptr(trig), trig.numel(),
                              ctypes.byref(p), _ptr(hits), hit_cap, ctypes.byref(nh), _ptr(ws),
                              ws.numel(), _stream(torch))
    return rc, int(nh.value)


def kernel_count():
    """Fused clustering-kernel variants (kernel -1 = the staged kernels)."""
    return int(load().tpx_stream_kernel_count())


def kernel_name(k):
    return load().tpx_stream_kernel_name(int(k)).decode()


class Stream:
    """tpx_stream: decode -> cluster -> centroid over consecutive chunks.
    kernel: clustering kernel (None = the library's default); patches: record
    the hit of every event so that patches() can follow each call."""

    def __init__(self, max_chunk_pkts, params=None, kernel=None, patches=False, persistent=None,
                 **kw):
        self.torch = _torch()
        self.lib = load()
        self.params = params or make_params(**kw)
        self._walk = kw.get("walk_lut_ns")
        h = ctypes.c_void_p()
        _check(self.lib.tpx_stream_create(ctypes.byref(self.params), max_chunk_pkts,
                                          ctypes.byref(h)), "tpx_stream_create")
        self.h = h
        self.max_chunk = max_chunk_pkts
        if kernel is not None:
            self.set_kernel(kernel)
        if persistent is not None:
            self.set_persistent(persistent)
        if patches:
            self.set_patches(True)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpx_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def process_raw(self, chunk, flush, hits, hit_cap):
        """Device-only call: chunk and hits are device tensors; returns
        (status, n_hits, stats) without copying anything back."""
        nh = ctypes.c_size_t()
        st = Stats()
        rc = self.lib.tpx_process_stream(self.h, _ptr(chunk), chunk.numel(), int(flush),
                                         _ptr(hits), hit_cap, ctypes.byref(nh), ctypes.byref(st),
                                         _stream(self.torch))
        return rc, int(nh.value), st

    def process(self, chunk, flush=False, hit_cap=None, hits=None):
        torch = self.torch
        pk = _u64(torch, chunk)
        if hits is None:
            hit_cap = max(pk.numel(), 1024) if hit_cap is None else hit_cap
            hits = torch.empty((hit_cap, 48), dtype=torch.uint8, device="cuda")
        else:
            hit_cap = hits.shape[0]
        rc, n, st = self.process_raw(pk, flush, hits, hit_cap)
        if rc == ECAPACITY:
            raise TpxError(rc, "tpx_process_stream", f"need {n} hits")
        _check(rc, "tpx_process_stream")
        return hits_to_numpy(hits, n), st.as_dict()

    def set_segment(self, q):
        _check(self.lib.tpx_stream_set_segment(self.h, int(q)), "tpx_stream_set_segment")

    def segment(self):
        return int(self.lib.tpx_stream_get_segment(self.h))

    def set_patches(self, enable=True):
        """Record the hit of every event in the following calls (needed by
        patches() after the fused kernel)."""
        _check(self.lib.tpx_stream_set_patches(self.h, int(enable)), "tpx_stream_set_patches")

    def set_kernel(self, k):
        _check(self.lib.tpx_stream_set_kernel(self.h, int(k)), "tpx_stream_set_kernel")

    def kernel(self):
        return int(self.lib.tpx_stream_get_kernel(self.h))

    def set_persistent(self, max_tiles=512):
        """Chunks of at most max_tiles tiles (4,096 words each) in one
        persistent launch; True = every chunk the launch can take (512
        tiles), False = none."""
        if max_tiles is True:
            max_tiles = 512
        _check(self.lib.tpx_stream_set_persistent(self.h, int(max_tiles)),
               "tpx_stream_set_persistent")

    def persistent(self):
        return int(self.lib.tpx_stream_get_persistent(self.h))

    def autotune(self, chunk, flush, candidates, hits, hit_cap, reps=3, kernels=None):
        """tpx_stream_autotune over strides x kernels (None: the current
        kernel only): (best stride, best kernel, {(kernel, stride): ms})."""
        torch = self.torch
        pk = _u64(torch, chunk)
        cand = (ctypes.c_uint32 * len(candidates))(*candidates)
        ks = list(kernels) if kernels is not None else [self.kernel()]
        kern = (ctypes.c_int * len(ks))(*ks) if kernels is not None else None
        ms = (ctypes.c_float * (len(candidates) * len(ks)))()
        best, best_k = ctypes.c_uint32(), ctypes.c_int()
        rc = self.lib.tpx_stream_autotune(self.h, _ptr(pk), pk.numel(), int(flush), _ptr(hits),
                                          hit_cap, cand, len(candidates), kern, len(ks), reps, ms,
                                          ctypes.byref(best), ctypes.byref(best_k), _stream(torch))
        _check(rc, "tpx_stream_autotune")
        times = {(int(k), int(c)): float(ms[j * len(candidates) + i])
                 for j, k in enumerate(ks) for i, c in enumerate(candidates)}
        return int(best.value), int(best_k.value), times

    def patches(self, hits, n_hits):
        """tpx_stream_patches: bfloat16 patches (int16 tensor [n_hits, 98]) of
        the hits (device uint8 [>= n_hits, 48]) of the last process call."""
        torch = self.torch
        feat = torch.empty((max(n_hits, 1), MLP_IN), dtype=torch.int16, device="cuda")
        ws = torch.empty(self.lib.tpx_stream_patch_workspace_bytes(n_hits), dtype=torch.uint8,
                         device="cuda")
        _check(self.lib.tpx_stream_patches(self.h, _ptr(hits), n_hits, _ptr(feat), _ptr(ws),
                                           ws.numel(), _stream(torch)), "tpx_stream_patches")
        return feat[:n_hits]

    def get_state(self):
        n = ctypes.c_size_t()
        _check(self.lib.tpx_stream_get_state(self.h, None, ctypes.byref(n)), "get_state")
        buf = ctypes.create_string_buffer(n.value)
        _check(self.lib.tpx_stream_get_state(self.h, buf, ctypes.byref(n)), "get_state")
        return bytes(buf.raw[:n.value])

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.lib.tpx_stream_set_state(self.h, buf, len(blob)), "set_state")

    def set_timing(self, enable=True):
        _check(self.lib.tpx_stream_set_timing(self.h, int(enable)), "set_timing")

    def stage_times_ms(self):
        """{stage: ms} of the last process call (timing must be enabled)."""
        buf = (ctypes.c_float * 8)()
        n = ctypes.c_size_t()
        _check(self.lib.tpx_stream_get_timing(self.h, buf, 8, ctypes.byref(n)), "get_timing")
        return {self.lib.tpx_stream_stage_name(i).decode(): float(buf[i]) for i in range(n.value)}

    @property
    def fallback_count(self):
        return int(self.lib.tpx_stream_fallback_count(self.h))


class Service:
    """tpx_service: continuous batching of chunks over one stream."""

    def __init__(self, max_batch_pkts, ring_pkts=None, params=None, **kw):
        self.torch = _torch()
        self.lib = load()
        self.p = params or make_params(**kw)
        self.h = ctypes.c_void_p()
        ring = 4 * max_batch_pkts if ring_pkts is None else ring_pkts
        _check(self.lib.tpx_service_create(ctypes.byref(self.p), max_batch_pkts, ring,
                                           ctypes.byref(self.h)), "tpx_service_create")

    def set_segment(self, q):
        """Segment stride of the service's stream."""
        _check(self.lib.tpx_service_set_segment(self.h, int(q)), "tpx_service_set_segment")

    def submit(self, chunk):
        """Admit a chunk (device tensor or numpy uint64); returns its number."""
        torch = self.torch
        if isinstance(chunk, np.ndarray):
            arr = np.ascontiguousarray(chunk.view(np.uint64))
            ptr, n, dev = arr.ctypes.data, arr.size, 0
        else:
            arr = chunk
            ptr, n, dev = arr.data_ptr(), arr.numel(), 1
        seq = ctypes.c_uint64()
        rc = self.lib.tpx_service_submit(self.h, ctypes.c_void_p(ptr), n, dev, ctypes.byref(seq),
                                         _stream(torch))
        _check(rc, "tpx_service_submit")
        return int(seq.value)

    def run_raw(self, flush, hits, hit_cap):
        """One batch into a device hit buffer: (status, n_hits, n_done, stats)."""
        nh, nd = ctypes.c_size_t(), ctypes.c_uint64()
        st = Stats()
        rc = self.lib.tpx_service_run(self.h, int(flush), _ptr(hits), hit_cap, ctypes.byref(nh),
                                      ctypes.byref(nd), ctypes.byref(st), _stream(self.torch))
        return rc, int(nh.value), int(nd.value), st

    def run(self, flush=False, hit_cap=1 << 20):
        hits = self.torch.empty((max(hit_cap, 1), 48), dtype=self.torch.uint8, device="cuda")
        rc, n, nd, st = self.run_raw(flush, hits, hit_cap)
        if rc == ECAPACITY:
            raise TpxError(rc, "tpx_service_run", f"need {n} hits")
        _check(rc, "tpx_service_run")
        return hits_to_numpy(hits, n), nd, st.as_dict()

    def replay(self, pk, chunk, pkts_per_s, hit_cap=1 << 20):
        """tpx_service_replay of a device-resident stream: (latencies in ms
        per chunk, runs)."""
        torch = self.torch
        n_chunks = (pk.numel() + chunk - 1) // chunk
        lat = np.zeros(max(n_chunks, 1), np.float32)
        hits = torch.empty((max(hit_cap, 1), 48), dtype=torch.uint8, device="cuda")
        nc, nr = ctypes.c_size_t(), ctypes.c_uint64()
        _check(self.lib.tpx_service_replay(self.h, _ptr(pk), pk.numel(), chunk, float(pkts_per_s),
                                           _ptr(hits), hit_cap, lat.ctypes.data, lat.size,
                                           ctypes.byref(nc), ctypes.byref(nr), _stream(torch)),
               "tpx_service_replay")
        return lat[:nc.value], int(nr.value)

    @property
    def device_bytes(self):
        return int(self.lib.tpx_service_device_bytes(self.h))

    def close(self):
        if self.h:
            self.lib.tpx_service_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """tpx_server: independent request streams in slots admitted against an
    HBM budget, their runs spread over several HIP streams."""

    def __init__(self, budget_bytes, n_streams=4, params=None, **kw):
        self.torch = _torch()
        self.lib = load()
        self.p = params or make_params(**kw)
        self.h = ctypes.c_void_p()
        _check(self.lib.tpx_server_create(ctypes.byref(self.p), int(budget_bytes), int(n_streams),
                                          ctypes.byref(self.h)), "tpx_server_create")

    def open(self, max_batch_pkts, ring_pkts=None, params=None, **kw):
        """A new slot (its own parameters, e.g. initial epochs, or the
        server's): (slot number, its device bytes)."""
        slot, nb = ctypes.c_uint32(), ctypes.c_size_t()
        ring = 4 * max_batch_pkts if ring_pkts is None else ring_pkts
        p = params or (make_params(**kw) if kw else None)
        _check(self.lib.tpx_server_open(self.h, ctypes.byref(p) if p is not None else None,
                                        max_batch_pkts, ring, ctypes.byref(slot),
                                        ctypes.byref(nb)), "tpx_server_open")
        return int(slot.value), int(nb.value)

    def submit(self, slot, chunk):
        """Admit a host chunk (numpy uint64) into the slot."""
        arr = np.ascontiguousarray(np.asarray(chunk).view(np.uint64))
        seq = ctypes.c_uint64()
        _check(self.lib.tpx_server_submit(self.h, slot, ctypes.c_void_p(arr.ctypes.data), arr.size,
                                          0, ctypes.byref(seq), None), "tpx_server_submit")
        return int(seq.value)

    def run(self, slot, flush=False, hit_cap=1 << 20):
        """One batch of the slot on its HIP stream: (hits, chunks done)."""
        torch = self.torch
        hits = torch.empty((max(hit_cap, 1), 48), dtype=torch.uint8, device="cuda")
        nh, nd = ctypes.c_size_t(), ctypes.c_uint64()
        rc = self.lib.tpx_server_run(self.h, slot, int(flush), _ptr(hits), hit_cap,
                                     ctypes.byref(nh), ctypes.byref(nd), None)
        if rc == ECAPACITY:
            raise TpxError(rc, "tpx_server_run", f"need {nh.value} hits")
        _check(rc, "tpx_server_run")
        # the run synchronised its own stream: the hits are complete
        return hits[:nh.value].cpu().numpy().view(HIT_DTYPE).reshape(-1), int(nd.value)

    def close_slot(self, slot):
        _check(self.lib.tpx_server_close(self.h, slot), "tpx_server_close")

    @property
    def free_bytes(self):
        return int(self.lib.tpx_server_free_bytes(self.h))

    def close(self):
        if self.h:
            self.lib.tpx_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def process_stream(packets, flush=True, kernel=None, persistent=None, **kw):
    """One-shot helper: the whole packet buffer as a single flushed chunk."""
    s = Stream(max(int(len(packets)), 1), kernel=kernel, persistent=persistent, **kw)
    try:
        return s.process(packets, flush=flush)
    finally:
        s.close()


def walk_fit(ev, trig, tof_lo, tof_hi, min_count=20):
    """tpx_walk_fit on device events: dict(params=(a, b, c, d), count, mean,
    lut=device float tensor [1024])."""
    torch = _torch()
    lib = load()
    t = trig if isinstance(trig, torch.Tensor) else _u64(torch, np.asarray(trig, np.uint64))
    params = (ctypes.c_double * 4)()
    count = np.zeros(1024, np.uint32)
    mean = np.zeros(1024, np.float64)
    lut = torch.empty(1024, dtype=torch.float32, device="cuda")
    ws = torch.empty(lib.tpx_walk_fit_workspace_bytes(), dtype=torch.uint8, device="cuda")
    n = ev["x"].numel()
    _check(lib.tpx_walk_fit(events_struct(ev), n, _ptr(t), t.numel(), int(tof_lo), int(tof_hi),
                            int(min_count), params, count.ctypes.data, mean.ctypes.data, _ptr(lut),
                            _ptr(ws), ws.numel(), _stream(torch)), "tpx_walk_fit")
    return dict(params=tuple(params), count=count, mean=mean, lut=lut)


# ------------------------------------------------------- learned centroider
MLP_IN, MLP_HID, MLP_OUT, MLP_NPARAM = 98, 256, 8, 93192


def centroid_dev(ev, labels, trig, params=None, ws=None):
    """tpx_centroid into device memory: uint8 tensor [n_hits, 48]."""
    torch = _torch()
    lib = load()
    n = ev["x"].numel()
    p = params or make_params()
    trig = _u64(torch, trig)
    hits = torch.empty((max(n, 1), 48), dtype=torch.uint8, device="cuda")
    ws = workspace(0, n) if ws is None else ws
    nh = ctypes.c_size_t()
    rc = lib.tpx_centroid(events_struct(ev), _ptr(labels), n, _ptr(trig), trig.numel(),
                          ctypes.byref(p), _ptr(hits), n, ctypes.byref(nh), _ptr(ws),
                          ws.numel(), _stream(torch))
    _check(rc, "tpx_centroid")
    return hits[:nh.value]


def patches(ev, labels, hits):
    """tpx_patches: bfloat16 bit patterns as an int16 tensor [n_hits, 98]."""
    torch = _torch()
    lib = load()
    n_h = hits.shape[0]
    feat = torch.empty((max(n_h, 1), MLP_IN), dtype=torch.int16, device="cuda")
    ws = torch.empty(lib.tpx_patch_workspace_bytes(n_h), dtype=torch.uint8, device="cuda")
    rc = lib.tpx_patches(events_struct(ev), _ptr(labels), ev["x"].numel(), _ptr(hits), n_h,
                         _ptr(feat), _ptr(ws), ws.numel(), _stream(torch))
    _check(rc, "tpx_patches")
    return feat[:n_h]


def refine(hits, out):
    """tpx_mlp_refine: fp32 tensor [n, 8] (x, y, t_ns of hits A and B,
    probability of two hits, 0)."""
    torch = _torch()
    n = out.shape[0]
    r = torch.empty((max(n, 1), 8), dtype=torch.float32, device="cuda")
    _check(load().tpx_mlp_refine(_ptr(hits), _ptr(out), n, _ptr(r), _stream(torch)),
           "tpx_mlp_refine")
    return r[:n]


class Mlp:
    """Parameters, Adam moments and workspaces of the 98-256-256-8 network;
    every call runs the library's kernels."""

    def __init__(self, params, batch=4096):
        torch = _torch()
        self.torch = torch
        self.lib = load()
        p = params if isinstance(params, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(params, np.float32))
        assert p.numel() == MLP_NPARAM
        self.p = p.to(device="cuda", dtype=torch.float32).contiguous().clone()
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.step = 0
        self.batch = batch
        self.ws = torch.empty(self.lib.tpx_mlp_workspace_bytes(batch), dtype=torch.uint8,
                              device="cuda")
        self.fws = None

    def forward(self, feat):
        torch = self.torch
        n = feat.shape[0]
        out = torch.empty((max(n, 1), MLP_OUT), dtype=torch.float32, device="cuda")
        need = self.lib.tpx_mlp_workspace_bytes(min(n, 65536))
        if self.fws is None or self.fws.numel() < need:
            self.fws = torch.empty(need, dtype=torch.uint8, device="cuda")
        _check(self.lib.tpx_mlp_forward(_ptr(self.p), _ptr(feat), n, _ptr(out), _ptr(self.fws),
                                        self.fws.numel(), _stream(torch)), "tpx_mlp_forward")
        return out[:n]

    def grad(self, feat, hits, truth, mult, want_loss=True):
        """Gradient of the mean loss into self.g; returns the loss (or None)."""
        n = feat.shape[0]
        assert n <= self.batch
        loss = ctypes.c_float()
        rc = self.lib.tpx_mlp_grad(_ptr(self.p), _ptr(feat), _ptr(hits), _ptr(truth), _ptr(mult),
                                   n, _ptr(self.g), ctypes.byref(loss) if want_loss else None,
                                   _ptr(self.ws), self.ws.numel(), _stream(self.torch))
        _check(rc, "tpx_mlp_grad")
        return float(loss.value) if want_loss else None

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(self.lib.tpx_mlp_adam(_ptr(self.p), _ptr(self.m), _ptr(self.v), _ptr(self.g),
                                     MLP_NPARAM, self.step, lr, beta1, beta2, eps,
                                     _stream(self.torch)), "tpx_mlp_adam")

    def train_step(self, feat, hits, truth, mult, lr, want_loss=False):
        loss = self.grad(feat, hits, truth, mult, want_loss)
        self.adam(lr)
        return loss

