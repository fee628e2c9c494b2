"""The C ABI on the CPU: the library loads, exports every function declared in
include/tgs.h, and rejects bad arguments on the host before any HIP call (so
no GPU is needed here)."""
import ctypes as C
import os
import re

import pytest

from paper_2412_13547_amd import api, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "tgs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tgs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = api.lib()
    names = _declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(api.EXPORTED) == set(names)


def test_status_strings_and_version():
    lib = api.lib()
    assert lib.tgs_status_str(0) == b"ok"
    assert lib.tgs_status_str(2) == b"pair capacity exceeded"
    assert lib.tgs_version().startswith(b"tgs")


def _cam(w=128, h=96):
    return api.camera_struct(scenes.identity_camera(w, h, float(w)))


def test_query_sizes_host_only():
    cam = _cam(3840, 2160)
    s = api.query_sizes(3_000_000, cam, api.dilation_struct(2, 1, 0), api.options_struct(16), 10_000)
    assert (s.w_ds, s.h_ds, s.grid_x, s.grid_y) == (1920, 1080, 120, 68)
    assert s.num_tiles == 8160 and s.pixels == 1920 * 1080
    s2 = api.query_sizes(3_000_000, cam, api.dilation_struct(2, 1, 0), api.options_struct(16), 10_000_000)
    assert s2.workspace_bytes >= s.workspace_bytes + 10 * 9_990_000   # >= 10 B per pair
    s3 = api.query_sizes(5, _cam(101, 37), api.dilation_struct(3, 2, 1), api.options_struct(8), 0)
    assert (s3.w_ds, s3.h_ds, s3.grid_x, s3.grid_y) == (33, 12, 5, 2)


def test_default_launch_host_only():
    for tile in (8, 16, 32):
        lds, ppt = api.default_launch(tile)
        assert lds in (64, 128, 256) and ppt in (1, 2, 4)
        assert tile != 8 or ppt == 1
        assert tile != 32 or ppt in (2, 4)
    lds, ppt = C.c_int32(), C.c_int32()
    assert api.lib().tgs_default_launch(12, C.byref(lds), C.byref(ppt)) == api.TGS_ERR_INVALID_ARG
    assert api.lib().tgs_default_launch(16, None, C.byref(ppt)) == api.TGS_ERR_INVALID_ARG


@pytest.mark.parametrize("field,value", [("stride", 0), ("off_x", 2), ("off_y", -1)])
def test_bad_dilation_rejected(field, value):
    dil = api.dilation_struct(2, 0, 0)
    setattr(dil, field, value)
    out = api.tgs_sizes()
    st = api.lib().tgs_query_sizes(10, C.byref(_cam()), C.byref(dil), C.byref(api.options_struct(16)),
                                   0, C.byref(out))
    assert st == api.TGS_ERR_INVALID_ARG
    assert b"" != api.lib().tgs_last_error()


@pytest.mark.parametrize("tile", [0, 4, 12, 64])
def test_bad_tile_rejected(tile):
    out = api.tgs_sizes()
    st = api.lib().tgs_query_sizes(10, C.byref(_cam()), C.byref(api.dilation_struct()),
                                   C.byref(api.options_struct(tile)), 0, C.byref(out))
    assert st == api.TGS_ERR_INVALID_ARG


def test_bad_camera_rejected():
    out = api.tgs_sizes()
    # near_z <= 0 would let Gaussians at depth <= 0 through: their float-bit
    # depth keys would sort after every positive depth, and depth 0 divides
    for mutate in (lambda c: setattr(c, "width", 0), lambda c: setattr(c, "fx", -1.0),
                   lambda c: setattr(c, "fy", float("nan")), lambda c: setattr(c, "near_z", 0.0),
                   lambda c: setattr(c, "near_z", -0.2), lambda c: setattr(c, "near_z", float("inf"))):
        cam = _cam()
        mutate(cam)
        st = api.lib().tgs_query_sizes(10, C.byref(cam), C.byref(api.dilation_struct()),
                                       C.byref(api.options_struct()), 0, C.byref(out))
        assert st == api.TGS_ERR_INVALID_ARG
    cam = _cam()
    cam.near_z = 1e-3
    assert api.lib().tgs_query_sizes(10, C.byref(cam), C.byref(api.dilation_struct()),
                                     C.byref(api.options_struct()), 0, C.byref(out)) == api.TGS_OK


def _gauss(n=10, deg=0, coeffs=1, ptr=1 << 20):
    return api.tgs_gaussians(n, deg, coeffs, ptr, ptr, ptr, ptr, ptr)


@pytest.mark.parametrize("g,status", [
    (_gauss(deg=4, coeffs=25), api.TGS_ERR_INVALID_ARG),
    (_gauss(deg=2, coeffs=4), api.TGS_ERR_INVALID_ARG),
    (_gauss(n=-1), api.TGS_ERR_INVALID_ARG),
    (api.tgs_gaussians(10, 0, 1, None, None, None, None, None), api.TGS_ERR_INVALID_ARG),
])
def test_bad_gaussians_rejected_before_any_device_call(g, status):
    st = api.tgs_state()
    r = api.lib().tgs_forward(None, C.byref(g), C.byref(_cam()), C.byref(api.dilation_struct()),
                              C.byref(api.options_struct()), C.byref(st), 1 << 20, None)
    assert r == status


def test_workspace_checks_before_device():
    g = _gauss()
    st = api.tgs_state()
    lib = api.lib()
    r = lib.tgs_preprocess_fwd(None, C.byref(g), C.byref(_cam()), C.byref(api.dilation_struct()),
                               C.byref(api.options_struct()), C.byref(st), None)
    assert r == api.TGS_ERR_INVALID_ARG and b"workspace" in lib.tgs_last_error()
    st.workspace = 4096 + 8            # misaligned
    st.workspace_bytes = 1 << 30
    r = lib.tgs_preprocess_fwd(None, C.byref(g), C.byref(_cam()), C.byref(api.dilation_struct()),
                               C.byref(api.options_struct()), C.byref(st), None)
    assert r == api.TGS_ERR_INVALID_ARG and b"aligned" in lib.tgs_last_error()
    st.workspace = 4096
    st.workspace_bytes = 16
    r = lib.tgs_preprocess_fwd(None, C.byref(g), C.byref(_cam()), C.byref(api.dilation_struct()),
                               C.byref(api.options_struct()), C.byref(st), None)
    assert r == api.TGS_ERR_INVALID_ARG and b"required" in lib.tgs_last_error()
    st.workspace_bytes = 1 << 30
    r = lib.tgs_preprocess_fwd(None, C.byref(g), C.byref(_cam()), C.byref(api.dilation_struct()),
                               C.byref(api.options_struct()), C.byref(st), None)
    assert r == api.TGS_ERR_INVALID_ARG and b"context" in lib.tgs_last_error()


def test_raster_refuses_unbinned_state():
    st = api.tgs_state()
    st.workspace = 4096
    st.workspace_bytes = 1 << 30
    lib = api.lib()
    r = lib.tgs_raster_fwd(None, C.byref(_cam()), C.byref(api.dilation_struct()),
                           C.byref(api.options_struct()), C.byref(st), 10, 1 << 20, None, None, None,
                           None, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"binned" in lib.tgs_last_error()
    r = lib.tgs_raster_bwd(None, C.byref(_cam()), C.byref(api.dilation_struct()),
                           C.byref(api.options_struct()), C.byref(st), 10, 1 << 20, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"binned" in lib.tgs_last_error()


def test_create_reports_missing_device():
    h = C.c_void_p()
    assert api.lib().tgs_create(10_000, C.byref(h)) == api.TGS_ERR_NO_DEVICE
    assert not h.value


def test_bad_lds_batch_and_flags_rejected():
    out = api.tgs_sizes()
    for lb in (32, 100, 512, -1):
        st = api.lib().tgs_query_sizes(10, C.byref(_cam()), C.byref(api.dilation_struct()),
                                       C.byref(api.options_struct(16, lds_batch=lb)), 0, C.byref(out))
        assert st == api.TGS_ERR_INVALID_ARG and b"lds_batch" in api.lib().tgs_last_error()
    for lb in (0, 64, 128, 256):
        st = api.lib().tgs_query_sizes(10, C.byref(_cam()), C.byref(api.dilation_struct()),
                                       C.byref(api.options_struct(16, lds_batch=lb)), 0, C.byref(out))
        assert st == api.TGS_OK
    # TGS_SYNC_CHECK is the only defined flag
    opt = api.options_struct(16)
    for flags, want in ((api.SYNC_CHECK, api.TGS_OK), (2, api.TGS_ERR_INVALID_ARG),
                        (api.SYNC_CHECK | 4, api.TGS_ERR_INVALID_ARG), (1 << 31, api.TGS_ERR_INVALID_ARG)):
        opt.flags = flags
        st = api.lib().tgs_query_sizes(10, C.byref(_cam()), C.byref(api.dilation_struct()),
                                       C.byref(opt), 0, C.byref(out))
        assert st == want, flags


def test_pair_capacity_limit():
    """The device pair count saturates at 2^32 - 1, so the largest capacity
    is 2^32 - 2 (a saturated count then always reads as an overflow)."""
    out = api.tgs_sizes()
    lib = api.lib()
    args = lambda cap: (10, C.byref(_cam()), C.byref(api.dilation_struct()),
                        C.byref(api.options_struct(16)), cap, C.byref(out))
    assert lib.tgs_query_sizes(*args(api.MAX_PAIR_CAPACITY)) == api.TGS_OK
    assert out.workspace_bytes > 16 * api.MAX_PAIR_CAPACITY
    assert lib.tgs_query_sizes(*args(api.MAX_PAIR_CAPACITY + 1)) == api.TGS_ERR_UNSUPPORTED
    assert lib.tgs_query_sizes(*args((1 << 40))) == api.TGS_ERR_UNSUPPORTED
    # the same limit on a state handed to a stage, before any device call
    st = api.tgs_state()
    st.workspace = 4096
    st.workspace_bytes = 1 << 62
    st.pair_capacity = api.MAX_PAIR_CAPACITY + 1
    r = lib.tgs_bin_sort(None, C.byref(_gauss()), C.byref(_cam()), C.byref(api.dilation_struct()),
                         C.byref(api.options_struct(16)), C.byref(st), None)
    assert r == api.TGS_ERR_UNSUPPORTED and b"2^32 - 2" in lib.tgs_last_error()


def _batch_args(nv, ws_bytes=1 << 30, stride=1 << 31):
    cams = (api.tgs_camera * nv)(*[_cam() for _ in range(nv)])
    dils = (api.tgs_dilation * nv)(*[api.dilation_struct(2, k % 2, 0) for k in range(nv)])
    states = (api.tgs_state * nv)()
    io = (api.tgs_view_io * nv)()
    for k in range(nv):
        states[k].workspace = (1 << 40) + k * stride
        states[k].workspace_bytes = ws_bytes
        states[k].pair_capacity = 1000
        io[k].image = 1 << 20
        io[k].dL_dimage = 1 << 20
        io[k].target = 1 << 20
    return cams, dils, states, io


def test_batch_view_count_and_overlap_rejected_before_device():
    lib = api.lib()
    g = _gauss()
    opt = api.options_struct(16)
    for nv in (0, 17):
        cams, dils, states, io = _batch_args(max(nv, 1))
        r = lib.tgs_batch_forward(None, C.byref(g), nv, cams, dils, C.byref(opt), states, io, None)
        assert r == api.TGS_ERR_INVALID_ARG and b"views" in lib.tgs_last_error()
    cams, dils, states, io = _batch_args(3, stride=4096)       # workspaces overlap
    r = lib.tgs_batch_forward(None, C.byref(g), 3, cams, dils, C.byref(opt), states, io, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"overlap" in lib.tgs_last_error()
    cams, dils, states, io = _batch_args(3)
    io[1].image = None
    r = lib.tgs_batch_forward(None, C.byref(g), 3, cams, dils, C.byref(opt), states, io, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"view 1" in lib.tgs_last_error()
    cams, dils, states, io = _batch_args(3)
    dils[2].off_x = 5
    r = lib.tgs_batch_forward(None, C.byref(g), 3, cams, dils, C.byref(opt), states, io, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"view 2" in lib.tgs_last_error()
    cams, dils, states, io = _batch_args(3)                  # valid up to the missing context
    r = lib.tgs_batch_forward(None, C.byref(g), 3, cams, dils, C.byref(opt), states, io, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"context" in lib.tgs_last_error()


def test_batch_backward_and_counts_refuse_unbinned_states():
    lib = api.lib()
    g = _gauss()
    cams, dils, states, io = _batch_args(2)
    grads = api.tgs_grads(1 << 20, 1 << 20, 1 << 20, 1 << 20, 1 << 20)
    r = lib.tgs_batch_backward(None, C.byref(g), 2, cams, dils, C.byref(api.options_struct(16)),
                               states, io, C.byref(grads), None, None, None, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"binned" in lib.tgs_last_error()
    r = lib.tgs_pair_counts(None, 2, states, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"binned" in lib.tgs_last_error()
    io[0].target = None
    r = lib.tgs_batch_l1_grad(None, 2, cams, dils, io, None, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"view 0" in lib.tgs_last_error()


def test_forward_static_rejects_what_exceeds_the_scratch_on_the_host():
    """The no-allocation forward checks its request against the static
    scratch before any device call: the same workspace tgs_query_sizes
    reports must fit TGS_STATIC_SCRATCH_BYTES, else TGS_ERR_UNSUPPORTED."""
    lib = api.lib()
    cam, dil, opt = _cam(), api.dilation_struct(), api.options_struct(16)
    out = api.tgs_sizes()
    n_fit, cap_fit = 1000, 100_000
    assert lib.tgs_query_sizes(n_fit, C.byref(cam), C.byref(dil), C.byref(opt), cap_fit,
                               C.byref(out)) == api.TGS_OK
    assert out.workspace_bytes <= api.STATIC_SCRATCH_BYTES
    # fits: the first failure is the missing context
    r = lib.tgs_forward_static(None, C.byref(_gauss(n_fit)), C.byref(cam), C.byref(dil),
                               C.byref(opt), cap_fit, 1 << 20, None)
    assert r == api.TGS_ERR_INVALID_ARG and b"context" in lib.tgs_last_error()
    # too many pairs, and too many Gaussians
    for n, cap in ((n_fit, 8_000_000), (2_000_000, cap_fit)):
        assert lib.tgs_query_sizes(n, C.byref(cam), C.byref(dil), C.byref(opt), cap,
                                   C.byref(out)) == api.TGS_OK
        assert out.workspace_bytes > api.STATIC_SCRATCH_BYTES
        r = lib.tgs_forward_static(None, C.byref(_gauss(n)), C.byref(cam), C.byref(dil),
                                   C.byref(opt), cap, 1 << 20, None)
        assert r == api.TGS_ERR_UNSUPPORTED and b"static scratch" in lib.tgs_last_error()
    r = lib.tgs_forward_static(None, C.byref(_gauss(n_fit)), C.byref(cam), C.byref(dil),
                               C.byref(opt), 0, 1 << 20, None)
    assert r == api.TGS_ERR_UNSUPPORTED
    r = lib.tgs_forward_static(None, C.byref(_gauss(n_fit)), C.byref(cam), C.byref(dil),
                               C.byref(opt), cap_fit, None, None)
    assert r == api.TGS_ERR_INVALID_ARG
