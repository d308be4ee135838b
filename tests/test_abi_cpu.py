"""The C-ABI library loads without a GPU and exports every entry point that
include/tpx.h declares; host-only helpers behave as documented."""
import ctypes
import os
import re

import paper_2603_04942_amd as tpx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tpx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpx_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = tpx.load()
    names = _declared()
    assert "tpx_process_stream" in names and "tpx_decode" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(tpx.EXPORTS)


def test_struct_sizes_match_header():
    assert ctypes.sizeof(tpx.Params) == 56
    assert ctypes.sizeof(tpx.Stats) == 13 * 8
    assert ctypes.sizeof(tpx.UnwrapState) == 64
    assert tpx.HIT_DTYPE.itemsize == 48


def test_defaults_and_strings():
    p = tpx.make_params()
    assert (p.dxy, p.dt_ticks, p.tof_max_ticks, p.trig_subtype) == (1, 128, 64000, 0xF)
    assert p.jump_ticks == 12_800_000_000 and p.close_slack_ticks == 64000
    assert p.walk_lut_ns is None
    lib = tpx.load()
    assert lib.tpx_status_str(0) == b"ok"
    assert lib.tpx_status_str(-3) == b"inconsistent stream"
    st = tpx.UnwrapState()
    p.pix_epoch0 = 2
    lib.tpx_unwrap_state_init(ctypes.byref(st), ctypes.byref(p))
    assert st.pix_epoch == 2 and st.tdc_epoch == 0 and st.trig_base == 0


def test_workspace_grows_with_size():
    lib = tpx.load()
    a = lib.tpx_workspace_bytes(1000, 1000)
    b = lib.tpx_workspace_bytes(10**6, 10**6)
    assert 0 < a < b
    # decode needs about 8 bytes per packet for the trigger staging area
    assert lib.tpx_workspace_bytes(10**6, 0) > 8 * 10**6


def test_argument_errors_need_no_gpu():
    lib = tpx.load()
    p = tpx.make_params(dxy=9)
    h = ctypes.c_void_p()
    assert lib.tpx_stream_create(ctypes.byref(p), 1000, ctypes.byref(h)) == tpx.EINVAL
    assert b"dxy" in lib.tpx_last_error()
    p = tpx.make_params(tof_max_ticks=0)
    assert lib.tpx_stream_create(ctypes.byref(p), 1000, ctypes.byref(h)) == tpx.EINVAL
    p = tpx.make_params()
    assert lib.tpx_stream_create(ctypes.byref(p), 0, ctypes.byref(h)) == tpx.EINVAL


def test_learned_and_tuning_argument_errors_need_no_gpu():
    """Calls that return before any GPU work: empty inputs, bad sizes, NULLs."""
    lib = tpx.load()
    fake = ctypes.c_void_p(0x1000)          # never dereferenced on these paths
    big = 1 << 40
    assert lib.tpx_mlp_workspace_bytes(0) > 0
    assert lib.tpx_mlp_workspace_bytes(4096) > lib.tpx_mlp_workspace_bytes(1024)
    assert lib.tpx_patch_workspace_bytes(10) == 10 * 98 * 4 + 256
    # forward of nothing is fine; without a workspace it is an error
    assert lib.tpx_mlp_forward(fake, fake, 0, fake, fake, big, None) == tpx.OK
    assert lib.tpx_mlp_forward(fake, fake, 5, fake, None, 0, None) == tpx.EINVAL
    # gradient of an empty batch, Adam step 0, NULL parameters
    loss = ctypes.c_float()
    assert lib.tpx_mlp_grad(fake, fake, fake, fake, fake, 0, fake, ctypes.byref(loss), fake, big,
                            None) == tpx.EINVAL
    assert lib.tpx_mlp_grad(None, fake, fake, fake, fake, 4, fake, None, fake, big,
                            None) == tpx.EINVAL
    assert lib.tpx_mlp_adam(fake, fake, fake, fake, 10, 0, 1e-3, 0.9, 0.999, 1e-8,
                            None) == tpx.EINVAL
    assert lib.tpx_mlp_refine(fake, fake, 0, fake, None) == tpx.OK
    # patches: nothing to do; events without hits; a workspace too small
    ev = tpx.Events()
    assert lib.tpx_patches(ev, None, 0, None, 0, None, fake, big, None) == tpx.OK
    ev = tpx.Events(fake, fake, fake, fake, fake)
    assert lib.tpx_patches(ev, fake, 3, fake, 0, fake, fake, big, None) == tpx.EINVAL
    assert lib.tpx_patches(ev, fake, 3, fake, 2, fake, fake, 10, None) == tpx.EINVAL
    # segment stride of a NULL stream and the autotuner's argument checks
    assert lib.tpx_stream_set_segment(None, 512) == tpx.EINVAL
    assert lib.tpx_stream_get_segment(None) == 0
    cand = (ctypes.c_uint32 * 2)(64, 4096)
    best = ctypes.c_uint32()
    assert lib.tpx_stream_autotune(None, fake, 0, 1, fake, 0, cand, 2, None, 0, 1, None,
                                   ctypes.byref(best), None, None) == tpx.EINVAL
    # clustering kernels: names, and the calls on a NULL stream
    assert lib.tpx_stream_kernel_count() >= 1
    assert lib.tpx_stream_kernel_name(-1) and lib.tpx_stream_kernel_name(0)
    assert lib.tpx_stream_set_kernel(None, 0) == tpx.EINVAL
    assert lib.tpx_stream_get_kernel(None) == -2
    assert lib.tpx_stream_set_persistent(None, 4) == tpx.EINVAL
    assert lib.tpx_stream_get_persistent(None) == -1
    assert lib.tpx_service_set_segment(None, 256) == tpx.EINVAL
    assert lib.tpx_stream_set_patches(None, 1) == tpx.EINVAL
