"""tpx_cluster_static (the allocation-free clustering entry point, workspace in
the library's own static device array) through the C ABI against tpx_cluster
with a caller workspace: identical labels and counts on two calls in a row, the
second smaller (the array keeps the first call's contents), on inputs that take
the sorting path and the global-memory path; sizes beyond the array are
refused before any launch."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from cases import tiny_cluster_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tpx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_04942_amd as t
    lib = t.load()
    lib.tpx_cluster_static.argtypes = [t.Events, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]
    lib.tpx_cluster_static.restype = ctypes.c_int32
    lib.tpx_cluster_static_max_events.argtypes = []
    lib.tpx_cluster_static_max_events.restype = ctypes.c_size_t
    return t


def _static(tpx, d, n, params):
    import torch
    lab = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    nc = ctypes.c_size_t()
    ev = tpx.events_struct(d)
    rc = tpx.load().tpx_cluster_static(ev, n, ctypes.byref(params), lab.data_ptr(),
                                       ctypes.byref(nc), torch.cuda.current_stream().cuda_stream)
    return rc, lab[:n].cpu().numpy().view(np.uint32), int(nc.value)


def _inputs():
    w = synth.make_config("c1", n_shots=400)
    import oracle
    dec = oracle.get().decode(w.packets, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    big = dec["events"]
    ev, dxy, dt = tiny_cluster_case(3)          # unsorted shots, another radius
    return [(big, 1, 128), (ev, dxy, dt)]


def test_static_matches_workspace_entry_twice(tpx, orc):
    for k, (e, dxy, dt) in enumerate(_inputs()):
        n = len(e["x"])
        print(f"call {k}: {n} events, radius {dxy}, window {dt}", flush=True)
        sys.stdout.flush()
        params = tpx.make_params(dxy=dxy, dt_ticks=dt)
        d = tpx.to_device_events(e)
        ref_lab, ref_nc = tpx.cluster(d, params=params)
        rc, lab, nc = _static(tpx, d, n, params)
        assert rc == 0, tpx.load().tpx_last_error()
        assert np.array_equal(lab, ref_lab.cpu().numpy().view(np.uint32))
        assert nc == ref_nc
        o_lab, o_nc = orc.cluster(e["x"], e["y"], e["shot"], e["toa"], dxy=dxy, dt_ticks=dt)
        assert np.array_equal(lab.astype(np.uint64), o_lab) and nc == o_nc


def test_static_refuses_beyond_its_array(tpx):
    import torch
    m = tpx.load().tpx_cluster_static_max_events()
    assert m > 100_000
    n = m + 1
    one = lambda dt: torch.zeros(n, dtype=dt, device="cuda")  # noqa: E731
    d = dict(x=one(torch.int16), y=one(torch.int16), tot=one(torch.int16),
             shot=one(torch.int32), toa=one(torch.int64))
    rc, _, _ = _static(tpx, d, n, tpx.make_params())
    assert rc == tpx.EINVAL
    assert b"static workspace" in tpx.load().tpx_last_error()
