"""Thin Python binding of libtgs (ctypes).  Argument marshalling only: every
step of the path runs in the HIP library; torch supplies device memory and the
stream.  The names follow the C ABI in include/tgs.h.

A missing or unloadable library raises; nothing here computes a fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtgs.so")

TGS_OK, TGS_ERR_INVALID_ARG, TGS_ERR_CAPACITY, TGS_ERR_HIP, TGS_ERR_NO_DEVICE, TGS_ERR_UNSUPPORTED = range(6)

EXPORTED = (
    "tgs_status_str", "tgs_last_error", "tgs_version", "tgs_create", "tgs_destroy",
    "tgs_query_sizes", "tgs_preprocess_fwd", "tgs_bin_sort", "tgs_raster_fwd", "tgs_forward",
    "tgs_l1_grad", "tgs_raster_bwd", "tgs_preprocess_bwd", "tgs_backward",
)


class tgs_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("world_to_cam", C.c_float * 12),
                ("near_z", C.c_float)]


class tgs_dilation(C.Structure):
    _fields_ = [("stride", C.c_int32), ("off_x", C.c_int32), ("off_y", C.c_int32)]


class tgs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("sh_coeffs", C.c_int32),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class tgs_options(C.Structure):
    _fields_ = [("tile", C.c_int32), ("reserved", C.c_int32), ("bg", C.c_float * 3),
                ("flags", C.c_uint32)]


class tgs_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class tgs_sizes(C.Structure):
    _fields_ = [("w_ds", C.c_int32), ("h_ds", C.c_int32), ("grid_x", C.c_int32),
                ("grid_y", C.c_int32), ("num_tiles", C.c_int64), ("pixels", C.c_int64),
                ("pair_capacity", C.c_uint64), ("workspace_bytes", C.c_uint64)]


class tgs_state(C.Structure):
    _fields_ = [("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64),
                ("pair_capacity", C.c_uint64), ("pair_count", C.c_uint64),
                ("key_bits", C.c_uint32), ("reserved", C.c_uint32),
                ("off_records", C.c_uint64), ("off_tiles_touched", C.c_uint64),
                ("off_depth_order", C.c_uint64),
                ("off_pair_vals", C.c_uint64), ("off_ranges", C.c_uint64),
                ("off_grad2d", C.c_uint64)]


_P = C.POINTER
_LIB = None


def _declare(lib):
    vp = C.c_void_p
    sig = {
        "tgs_status_str": (C.c_char_p, [C.c_int]),
        "tgs_last_error": (C.c_char_p, []),
        "tgs_version": (C.c_char_p, []),
        "tgs_create": (C.c_int, [C.c_int, _P(vp)]),
        "tgs_destroy": (None, [vp]),
        "tgs_query_sizes": (C.c_int, [C.c_int64, _P(tgs_camera), _P(tgs_dilation), _P(tgs_options),
                                      C.c_uint64, _P(tgs_sizes)]),
        "tgs_preprocess_fwd": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                         _P(tgs_options), _P(tgs_state), vp]),
        "tgs_bin_sort": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                   _P(tgs_options), _P(tgs_state), vp]),
        "tgs_raster_fwd": (C.c_int, [vp, _P(tgs_camera), _P(tgs_dilation), _P(tgs_options),
                                     _P(tgs_state), C.c_int64, vp, vp, vp, vp, vp, vp]),
        "tgs_forward": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                  _P(tgs_options), _P(tgs_state), vp, vp]),
        "tgs_l1_grad": (C.c_int, [vp, _P(tgs_camera), _P(tgs_dilation), vp, vp, vp, vp, vp]),
        "tgs_raster_bwd": (C.c_int, [vp, _P(tgs_camera), _P(tgs_dilation), _P(tgs_options),
                                     _P(tgs_state), C.c_int64, vp, vp, vp]),
        "tgs_preprocess_bwd": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                         _P(tgs_options), _P(tgs_state), _P(tgs_grads), vp, vp, vp,
                                         vp]),
        "tgs_backward": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                   _P(tgs_options), _P(tgs_state), vp, vp, _P(tgs_grads), vp, vp,
                                   vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def lib():
    """Load libtgs.so (built by ``paper_2412_13547_amd.build``); raise if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2412_13547_amd.build` (no CPU fallback exists)")
        handle = C.CDLL(LIB_PATH)
        _declare(handle)
        _LIB = handle
    return _LIB


class TgsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"tgs status {status}: {message}")
        self.status = status


def check(status: int):
    if status != TGS_OK:
        raise TgsError(status, lib().tgs_last_error().decode())


# ---------------------------------------------------------------------------
# argument builders


def camera_struct(cam) -> tgs_camera:
    c = tgs_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w = np.asarray(cam.w2c, dtype=np.float32).reshape(12)
    for k in range(12):
        c.world_to_cam[k] = float(w[k])
    c.near_z = float(getattr(cam, "near", 0.2))
    return c


def dilation_struct(stride=1, off_x=0, off_y=0) -> tgs_dilation:
    return tgs_dilation(int(stride), int(off_x), int(off_y))


def options_struct(tile=16, bg=(0.0, 0.0, 0.0)) -> tgs_options:
    o = tgs_options()
    o.tile = int(tile)
    o.reserved = 0
    for k in range(3):
        o.bg[k] = float(bg[k])
    o.flags = 0
    return o


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


@dataclasses.dataclass
class DeviceScene:
    """Parameters resident on the GPU, structure-of-arrays float32 torch tensors."""
    means: "object"
    scales: "object"
    quats: "object"
    opacities: "object"
    sh: "object"
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        import torch
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return cls(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities), f(scene.sh),
                   int(scene.sh_degree))

    def struct(self) -> tgs_gaussians:
        for t in (self.means, self.scales, self.quats, self.opacities, self.sh):
            assert t.is_contiguous() and str(t.dtype) == "torch.float32"
        return tgs_gaussians(self.n, self.sh_degree, int(self.sh.shape[0]), _ptr(self.means),
                             _ptr(self.scales), _ptr(self.quats), _ptr(self.opacities),
                             _ptr(self.sh))

    def zeros_like(self) -> "DeviceScene":
        import torch
        return DeviceScene(*(torch.zeros_like(t) for t in (self.means, self.scales, self.quats,
                                                            self.opacities, self.sh)),
                           self.sh_degree)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Context:
    """A libtgs context on one device."""

    def __init__(self, device: int = 0):
        self._lib = lib()
        h = C.c_void_p()
        check(self._lib.tgs_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self._lib.tgs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_sizes(n, cam, dil: tgs_dilation, opt: tgs_options, pair_capacity: int) -> tgs_sizes:
    out = tgs_sizes()
    check(lib().tgs_query_sizes(int(n), C.byref(camera_struct(cam) if not isinstance(cam, tgs_camera) else cam),
                                C.byref(dil), C.byref(opt), int(pair_capacity), C.byref(out)))
    return out


class View:
    """One camera + dilation pattern with its workspace (device memory owned by torch).

    ``pair_capacity`` grows on demand (a forward that needs more pairs than
    the workspace holds is re-run once with a larger workspace).
    """

    def __init__(self, ctx: Context, n: int, cam, stride=1, off_x=0, off_y=0, tile=16,
                 bg=(0.0, 0.0, 0.0), pair_capacity: int | None = None):
        import torch
        self.ctx = ctx
        self.n = int(n)
        self.cam = cam
        self.cam_s = camera_struct(cam)
        self.dil = dilation_struct(stride, off_x, off_y)
        self.opt = options_struct(tile, bg)
        self.state = tgs_state()
        self.workspace = None
        self.sizes = query_sizes(self.n, self.cam_s, self.dil, self.opt, 0)
        self._torch = torch
        self.reserve(pair_capacity if pair_capacity is not None else max(1024, 16 * self.n))

    def set_offsets(self, off_x: int, off_y: int):
        self.dil = dilation_struct(self.dil.stride, off_x, off_y)
        self.sizes = query_sizes(self.n, self.cam_s, self.dil, self.opt, self.state.pair_capacity)

    def reserve(self, pair_capacity: int):
        sz = query_sizes(self.n, self.cam_s, self.dil, self.opt, int(pair_capacity))
        if self.workspace is None or self.workspace.numel() < sz.workspace_bytes:
            self.workspace = self._torch.empty(int(sz.workspace_bytes) + 256, dtype=self._torch.uint8,
                                               device="cuda")
        base = int(self.workspace.data_ptr())
        aligned = (base + 255) // 256 * 256
        self.state.workspace = aligned
        self.state.workspace_bytes = int(sz.workspace_bytes)
        self.state.pair_capacity = int(pair_capacity)
        self.state.key_bits = 0
        self.sizes = sz

    @property
    def image_shape(self):
        return (3, int(self.sizes.h_ds), int(self.sizes.w_ds))

    # -- stages ------------------------------------------------------------
    def preprocess_fwd(self, scene: DeviceScene, stream=None):
        g = scene.struct()
        check(lib().tgs_preprocess_fwd(self.ctx.handle, C.byref(g), C.byref(self.cam_s),
                                       C.byref(self.dil), C.byref(self.opt), C.byref(self.state),
                                       _stream(stream)))

    def bin_sort(self, scene: DeviceScene, stream=None, grow: bool = True):
        g = scene.struct()
        st = lib().tgs_bin_sort(self.ctx.handle, C.byref(g), C.byref(self.cam_s), C.byref(self.dil),
                                C.byref(self.opt), C.byref(self.state), _stream(stream))
        if st == TGS_ERR_CAPACITY and grow:
            need = int(self.state.pair_count)
            self.reserve(int(need * 1.25) + 1024)
            self.preprocess_fwd(scene, stream)
            st = lib().tgs_bin_sort(self.ctx.handle, C.byref(g), C.byref(self.cam_s),
                                    C.byref(self.dil), C.byref(self.opt), C.byref(self.state),
                                    _stream(stream))
        check(st)

    def raster_fwd(self, image, t_final=None, last_contrib=None, n_eval=None, n_blend=None,
                   stream=None):
        check(lib().tgs_raster_fwd(self.ctx.handle, C.byref(self.cam_s), C.byref(self.dil),
                                   C.byref(self.opt), C.byref(self.state), self.n, _ptr(image),
                                   _ptr(t_final), _ptr(last_contrib), _ptr(n_eval), _ptr(n_blend),
                                   _stream(stream)))

    def forward(self, scene: DeviceScene, image=None, stream=None, t_final=None, last_contrib=None,
                n_eval=None, n_blend=None):
        torch = self._torch
        if image is None:
            image = torch.empty(self.image_shape, dtype=torch.float32, device="cuda")
        self.preprocess_fwd(scene, stream)
        self.bin_sort(scene, stream)
        self.raster_fwd(image, t_final, last_contrib, n_eval, n_blend, stream)
        return image

    def l1_grad(self, image, target, dL_dimage=None, loss=None, stream=None):
        torch = self._torch
        if dL_dimage is None:
            dL_dimage = torch.empty_like(image)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device="cuda")
        check(lib().tgs_l1_grad(self.ctx.handle, C.byref(self.cam_s), C.byref(self.dil),
                                _ptr(image), _ptr(target), _ptr(dL_dimage), _ptr(loss),
                                _stream(stream)))
        return dL_dimage, loss

    def raster_bwd(self, image, dL_dimage, stream=None):
        check(lib().tgs_raster_bwd(self.ctx.handle, C.byref(self.cam_s), C.byref(self.dil),
                                   C.byref(self.opt), C.byref(self.state), self.n, _ptr(image),
                                   _ptr(dL_dimage), _stream(stream)))

    def preprocess_bwd(self, scene: DeviceScene, grads: DeviceScene, pos_stat=None, col_stat=None,
                       visible=None, stream=None):
        g = scene.struct()
        out = tgs_grads(_ptr(grads.means), _ptr(grads.scales), _ptr(grads.quats),
                        _ptr(grads.opacities), _ptr(grads.sh))
        check(lib().tgs_preprocess_bwd(self.ctx.handle, C.byref(g), C.byref(self.cam_s),
                                       C.byref(self.dil), C.byref(self.opt), C.byref(self.state),
                                       C.byref(out), _ptr(pos_stat), _ptr(col_stat), _ptr(visible),
                                       _stream(stream)))

    def backward(self, scene: DeviceScene, image, dL_dimage, grads: DeviceScene | None = None,
                 pos_stat=None, col_stat=None, visible=None, stream=None):
        if grads is None:
            grads = scene.zeros_like()
        g = scene.struct()
        out = tgs_grads(_ptr(grads.means), _ptr(grads.scales), _ptr(grads.quats),
                        _ptr(grads.opacities), _ptr(grads.sh))
        check(lib().tgs_backward(self.ctx.handle, C.byref(g), C.byref(self.cam_s), C.byref(self.dil),
                                 C.byref(self.opt), C.byref(self.state), _ptr(image),
                                 _ptr(dL_dimage), C.byref(out), _ptr(pos_stat), _ptr(col_stat),
                                 _ptr(visible), _stream(stream)))
        return grads

    # -- views into the workspace (inspection and tests) --------------------
    def _view(self, off: int, count: int, dtype):
        torch = self._torch
        base = int(self.state.workspace) - int(self.workspace.data_ptr())
        itemsize = torch.empty(0, dtype=dtype).element_size()
        raw = self.workspace[base + int(off): base + int(off) + count * itemsize]
        return raw.view(dtype)

    def records(self):
        """(n, 12) float32 view: u v A B C o r g b z radius(int bits) flags(bits)."""
        return self._view(self.state.off_records, self.n * 12, self._torch.float32).view(self.n, 12)

    def tiles_touched(self):
        return self._view(self.state.off_tiles_touched, self.n, self._torch.int32)

    def depth_order(self):
        return self._view(self.state.off_depth_order, self.n, self._torch.int32)

    def pair_vals(self):
        return self._view(self.state.off_pair_vals, int(self.state.pair_count), self._torch.int32)

    def ranges(self):
        nt = int(self.sizes.num_tiles)
        return self._view(self.state.off_ranges, 2 * nt, self._torch.int32).view(nt, 2)

    def grad2d(self):
        return self._view(self.state.off_grad2d, self.n * 9, self._torch.float32).view(self.n, 9)
