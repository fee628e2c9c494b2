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
    "tgs_query_sizes", "tgs_default_launch", "tgs_preprocess_fwd", "tgs_bin_sort", "tgs_raster_fwd", "tgs_forward",
    "tgs_forward_static",
    "tgs_l1_grad", "tgs_raster_bwd", "tgs_preprocess_bwd", "tgs_backward",
    "tgs_batch_preprocess_fwd", "tgs_batch_bin_sort", "tgs_batch_raster_fwd",
    "tgs_batch_forward", "tgs_batch_l1_grad", "tgs_batch_raster_bwd", "tgs_batch_preprocess_bwd",
    "tgs_batch_backward", "tgs_pair_counts", "tgs_adam_step", "tgs_densify_query",
    "tgs_densify_select",
)
STATIC_SCRATCH_BYTES = 64 << 20
ADAM_STATE_BYTES = 16
MAX_ADAM_GROUPS = 8

MAX_VIEWS = 16
PAIR_COUNT_PENDING = (1 << 64) - 1
SYNC_CHECK = 1                      # tgs_options.flags: synchronous capacity check
MAX_PAIR_CAPACITY = (1 << 32) - 2


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
    _fields_ = [("tile", C.c_int32), ("lds_batch", C.c_int32), ("pixels_per_thread", C.c_int32),
                ("bg", C.c_float * 3), ("flags", C.c_uint32)]


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
                ("off_grad2d", C.c_uint64), ("off_pair_count", C.c_uint64),
                ("off_depth_count", C.c_uint64), ("off_tile_work", C.c_uint64),
                ("off_t_final", C.c_uint64), ("off_last_contrib", C.c_uint64),
                ("off_nonfinite_count", C.c_uint64)]


class tgs_adam_group(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("exp_avg", C.c_void_p),
                ("exp_avg_sq", C.c_void_p), ("count", C.c_int64), ("lr", C.c_float)]


class tgs_view_io(C.Structure):
    _fields_ = [("image", C.c_void_p), ("t_final", C.c_void_p), ("last_contrib", C.c_void_p),
                ("n_eval", C.c_void_p), ("n_blend", C.c_void_p), ("target", C.c_void_p),
                ("dL_dimage", C.c_void_p), ("n_tested", C.c_void_p), ("pos_stat", C.c_void_p),
                ("col_stat", C.c_void_p), ("visible", C.c_void_p)]


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
        "tgs_default_launch": (C.c_int, [C.c_int32, _P(C.c_int32), _P(C.c_int32)]),
        "tgs_preprocess_fwd": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                         _P(tgs_options), _P(tgs_state), vp]),
        "tgs_bin_sort": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                   _P(tgs_options), _P(tgs_state), vp]),
        "tgs_raster_fwd": (C.c_int, [vp, _P(tgs_camera), _P(tgs_dilation), _P(tgs_options),
                                     _P(tgs_state), C.c_int64, vp, vp, vp, vp, vp, vp]),
        "tgs_forward": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                  _P(tgs_options), _P(tgs_state), vp, vp]),
        "tgs_forward_static": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                         _P(tgs_options), C.c_uint64, vp, vp]),
        "tgs_l1_grad": (C.c_int, [vp, _P(tgs_camera), _P(tgs_dilation), vp, vp, vp, vp, vp]),
        "tgs_raster_bwd": (C.c_int, [vp, _P(tgs_camera), _P(tgs_dilation), _P(tgs_options),
                                     _P(tgs_state), C.c_int64, vp, vp]),
        "tgs_preprocess_bwd": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                         _P(tgs_options), _P(tgs_state), _P(tgs_grads), vp, vp, vp,
                                         vp]),
        "tgs_backward": (C.c_int, [vp, _P(tgs_gaussians), _P(tgs_camera), _P(tgs_dilation),
                                   _P(tgs_options), _P(tgs_state), vp, _P(tgs_grads), vp, vp,
                                   vp, vp]),
        "tgs_batch_forward": (C.c_int, [vp, _P(tgs_gaussians), C.c_int32, _P(tgs_camera),
                                        _P(tgs_dilation), _P(tgs_options), _P(tgs_state),
                                        _P(tgs_view_io), vp]),
        "tgs_batch_l1_grad": (C.c_int, [vp, C.c_int32, _P(tgs_camera), _P(tgs_dilation),
                                        _P(tgs_view_io), vp, vp]),
        "tgs_batch_backward": (C.c_int, [vp, _P(tgs_gaussians), C.c_int32, _P(tgs_camera),
                                         _P(tgs_dilation), _P(tgs_options), _P(tgs_state),
                                         _P(tgs_view_io), _P(tgs_grads), vp, vp, vp, vp]),
        "tgs_pair_counts": (C.c_int, [vp, C.c_int32, _P(tgs_state), vp]),
        "tgs_adam_step": (C.c_int, [vp, _P(tgs_adam_group), C.c_int32, C.c_float, C.c_float,
                                    C.c_float, vp, vp]),
        "tgs_densify_query": (C.c_int, [C.c_int64, _P(C.c_uint64)]),
        "tgs_densify_select": (C.c_int, [vp, C.c_int64, vp, vp, vp, C.c_float, C.c_float,
                                         C.c_int32, C.c_int64, vp, vp, vp, C.c_uint64, vp]),
        "tgs_batch_preprocess_fwd": (C.c_int, [vp, _P(tgs_gaussians), C.c_int32, _P(tgs_camera),
                                               _P(tgs_dilation), _P(tgs_options), _P(tgs_state),
                                               vp]),
        "tgs_batch_bin_sort": (C.c_int, [vp, _P(tgs_gaussians), C.c_int32, _P(tgs_camera),
                                         _P(tgs_dilation), _P(tgs_options), _P(tgs_state), vp]),
        "tgs_batch_raster_fwd": (C.c_int, [vp, C.c_int64, C.c_int32, _P(tgs_camera),
                                           _P(tgs_dilation), _P(tgs_options), _P(tgs_state),
                                           _P(tgs_view_io), vp]),
        "tgs_batch_raster_bwd": (C.c_int, [vp, C.c_int64, C.c_int32, _P(tgs_camera),
                                           _P(tgs_dilation), _P(tgs_options), _P(tgs_state),
                                           _P(tgs_view_io), vp]),
        "tgs_batch_preprocess_bwd": (C.c_int, [vp, _P(tgs_gaussians), C.c_int32, _P(tgs_camera),
                                               _P(tgs_dilation), _P(tgs_options), _P(tgs_state),
                                               _P(tgs_view_io), _P(tgs_grads), vp, vp, vp, vp]),
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


def options_struct(tile=16, bg=(0.0, 0.0, 0.0), lds_batch=0, pixels_per_thread=0,
                   flags=0) -> tgs_options:
    o = tgs_options()
    o.tile = int(tile)
    o.lds_batch = int(lds_batch)
    o.pixels_per_thread = int(pixels_per_thread)
    for k in range(3):
        o.bg[k] = float(bg[k])
    o.flags = int(flags)
    return o


def _ptr(t) -> int | None:
    """Device address of a dense device tensor (None passes NULL).  The C ABI
    reads plain arrays, so strided views and host tensors are refused."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError(f"tensor of shape {tuple(t.shape)} is not contiguous; "
                         "libtgs reads dense arrays (call .contiguous())")
    if not t.is_cuda:
        raise ValueError("libtgs reads device memory: move the tensor to the GPU")
    return int(t.data_ptr())


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


def default_launch(tile: int) -> tuple[int, int]:
    """(lds_batch, pixels_per_thread) the rasterizers use for `tile` when the
    options leave them at 0."""
    lds, ppt = C.c_int32(), C.c_int32()
    check(lib().tgs_default_launch(int(tile), C.byref(lds), C.byref(ppt)))
    return int(lds.value), int(ppt.value)


class View:
    """One camera + dilation pattern with its workspace (device memory owned by torch).

    With ``sync_check`` (the default here) the binning reads the pair count
    back and ``pair_capacity`` grows on demand: a forward that needs more
    pairs than the workspace holds is re-run once with a larger workspace.
    Without it every call stays asynchronous (the library's default; the
    step can be captured in a graph): size the workspace first with
    ``fit_capacity``, and read the count with ``pair_count()``.
    """

    def __init__(self, ctx: Context, n: int, cam, stride=1, off_x=0, off_y=0, tile=16,
                 bg=(0.0, 0.0, 0.0), pair_capacity: int | None = None, lds_batch: int = 0,
                 state: tgs_state | None = None, pixels_per_thread: int = 0,
                 sync_check: bool = True):
        import torch
        self.ctx = ctx
        self.n = int(n)
        self.cam = cam
        self.cam_s = camera_struct(cam)
        self.dil = dilation_struct(stride, off_x, off_y)
        self.opt = options_struct(tile, bg, lds_batch, pixels_per_thread)
        self.opt_sync = options_struct(tile, bg, lds_batch, pixels_per_thread, SYNC_CHECK)
        self.sync_check = bool(sync_check)
        self.state = state if state is not None else tgs_state()
        self.workspace = None
        self.sizes = query_sizes(self.n, self.cam_s, self.dil, self.opt, 0)
        self._torch = torch
        # bumped by every call that rewrites the workspace's forward results
        self.generation = 0
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
        self.generation += 1
        check(lib().tgs_preprocess_fwd(self.ctx.handle, C.byref(g), C.byref(self.cam_s),
                                       C.byref(self.dil), C.byref(self.opt), C.byref(self.state),
                                       _stream(stream)))

    def bin_sort(self, scene: DeviceScene, stream=None, grow: bool = True, sync: bool | None = None):
        """Pairs, sort and ranges.  sync (default: the view's sync_check) reads
        the count back and, with grow, enlarges the workspace and repeats."""
        g = scene.struct()
        self.generation += 1
        sync = self.sync_check if sync is None else bool(sync)
        opt = self.opt_sync if sync else self.opt
        st = lib().tgs_bin_sort(self.ctx.handle, C.byref(g), C.byref(self.cam_s), C.byref(self.dil),
                                C.byref(opt), C.byref(self.state), _stream(stream))
        if sync and st == TGS_ERR_CAPACITY and grow:
            need = int(self.state.pair_count)
            self.reserve(int(need * 1.25) + 1024)
            self.preprocess_fwd(scene, stream)
            st = lib().tgs_bin_sort(self.ctx.handle, C.byref(g), C.byref(self.cam_s),
                                    C.byref(self.dil), C.byref(opt), C.byref(self.state),
                                    _stream(stream))
        check(st)

    def pair_count(self, stream=None) -> int:
        """The pair count of the last bin/sort; reads the device count back
        (synchronises) when it is pending.  Raises TgsError when the pairs did
        not fit the workspace (the count is then in state.pair_count)."""
        if int(self.state.pair_count) == PAIR_COUNT_PENDING:
            check(lib().tgs_pair_counts(self.ctx.handle, 1, C.byref(self.state), _stream(stream)))
        elif int(self.state.pair_count) > int(self.state.pair_capacity):
            raise TgsError(TGS_ERR_CAPACITY, "pairs exceed the workspace capacity")
        return int(self.state.pair_count)

    def fit_capacity(self, scene: DeviceScene, slack: float = 1.1, tries: int = 4) -> int:
        """Run asynchronous forwards until the pairs fit the workspace; returns
        the count.  The workspace may be re-allocated, so capture graphs only
        after this."""
        for _ in range(tries):
            self.preprocess_fwd(scene)
            self.bin_sort(scene, sync=False)
            lib().tgs_pair_counts(self.ctx.handle, 1, C.byref(self.state), _stream(None))
            need = int(self.state.pair_count)
            if need >= (1 << 32) - 1:
                raise TgsError(TGS_ERR_UNSUPPORTED, "2^32 - 1 or more pairs in one view")
            if need <= int(self.state.pair_capacity):
                return need
            self.reserve(min(int(need * slack) + 4096, MAX_PAIR_CAPACITY))
        raise TgsError(TGS_ERR_CAPACITY, "pair capacity did not converge")

    def raster_fwd(self, image=None, t_final=None, last_contrib=None, n_eval=None, n_blend=None,
                   stream=None):
        """Blend forward; image None writes only the per-pixel state the
        backward reads (final transmittance, last blended entry)."""
        self.generation += 1
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

    def raster_bwd(self, dL_dimage, stream=None):
        """Blend backward of the last forward on this view's workspace."""
        check(lib().tgs_raster_bwd(self.ctx.handle, C.byref(self.cam_s), C.byref(self.dil),
                                   C.byref(self.opt), C.byref(self.state), self.n,
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

    def backward(self, scene: DeviceScene, dL_dimage, grads: DeviceScene | None = None,
                 pos_stat=None, col_stat=None, visible=None, stream=None):
        """Blend and preprocess backward of the last forward on this view's
        workspace."""
        if grads is None:
            grads = scene.zeros_like()
        g = scene.struct()
        out = tgs_grads(_ptr(grads.means), _ptr(grads.scales), _ptr(grads.quats),
                        _ptr(grads.opacities), _ptr(grads.sh))
        check(lib().tgs_backward(self.ctx.handle, C.byref(g), C.byref(self.cam_s), C.byref(self.dil),
                                 C.byref(self.opt), C.byref(self.state),
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
        """Ids of the Gaussians with tiles, sorted by depth key (equal keys by id);
        valid after a bin/sort of this state."""
        m = int(self._view(self.state.off_depth_count, 1, self._torch.int32).item())
        return self._view(self.state.off_depth_order, min(max(m, 0), self.n), self._torch.int32)

    def pair_vals(self):
        return self._view(self.state.off_pair_vals, self.pair_count(), self._torch.int32)

    def ranges(self):
        nt = int(self.sizes.num_tiles)
        return self._view(self.state.off_ranges, 2 * nt, self._torch.int32).view(nt, 2)

    def grad2d(self):
        return self._view(self.state.off_grad2d, self.n * 9, self._torch.float32).view(self.n, 9)

    def t_final(self):
        """Every pixel's transmittance after the last forward's walk."""
        h, w = int(self.sizes.h_ds), int(self.sizes.w_ds)
        return self._view(self.state.off_t_final, h * w, self._torch.float32).view(h, w)

    def last_contrib(self):
        """Every pixel's 1-based index of its last blended entry (0: none),
        from the last forward."""
        h, w = int(self.sizes.h_ds), int(self.sizes.w_ds)
        return self._view(self.state.off_last_contrib, h * w, self._torch.int32).view(h, w)

    def nonfinite_count(self) -> int:
        """Gaussians the last preprocess culled for a non-finite parameter
        (reads the device counter back)."""
        return int(self._view(self.state.off_nonfinite_count, 1, self._torch.int32).item())

    def tile_work(self):
        """Entries the last forward walked per tile (the backward's tile order
        weights; any values give the same results)."""
        return self._view(self.state.off_tile_work, int(self.sizes.num_tiles), self._torch.int32)


def forward_static(ctx: Context, scene: DeviceScene, cam, image, pair_capacity: int, stride=1,
                   off_x=0, off_y=0, tile=16, bg=(0.0, 0.0, 0.0), lds_batch=0,
                   pixels_per_thread=0, sync_check=False, stream=None):
    """tgs_forward_static: the forward of one view into ``image`` with the
    library's static per-GPU scratch as workspace (no allocation).  Raises
    TgsError(TGS_ERR_UNSUPPORTED) when the request needs more workspace than
    STATIC_SCRATCH_BYTES."""
    g = scene.struct()
    opt = options_struct(tile, bg, lds_batch, pixels_per_thread, SYNC_CHECK if sync_check else 0)
    check(lib().tgs_forward_static(ctx.handle if ctx is not None else None, C.byref(g),
                                   C.byref(camera_struct(cam)),
                                   C.byref(dilation_struct(stride, off_x, off_y)), C.byref(opt),
                                   int(pair_capacity), _ptr(image), _stream(stream)))
    return image


def _grads_struct(grads: DeviceScene) -> tgs_grads:
    return tgs_grads(_ptr(grads.means), _ptr(grads.scales), _ptr(grads.quats),
                     _ptr(grads.opacities), _ptr(grads.sh))


class Batch:
    """Up to MAX_VIEWS views (camera + dilation pattern) of one Gaussian set,
    processed by the batched calls: one preprocess launch, per-view binning,
    one rasterizer launch per direction, one summed preprocess backward.
    None of its step methods synchronises, so ``step`` can be captured in a
    HIP graph (``torch.cuda.CUDAGraph``) once the capacities fit.

    views: sequence of (camera, stride, off_x, off_y).  Images and upstream
    gradients are allocated here; targets are full-resolution [3][H][W]
    float32 device tensors set with ``set_targets``."""

    def __init__(self, ctx: Context, n: int, views, tile=16, bg=(0.0, 0.0, 0.0), lds_batch=0,
                 pair_capacity=None, counts: bool = False, pixels_per_thread: int = 0,
                 view_stats: bool = False):
        import torch
        self._torch = torch
        nv = len(views)
        if not 1 <= nv <= MAX_VIEWS:
            raise ValueError(f"a batch holds 1..{MAX_VIEWS} views, got {nv}")
        self.ctx, self.n, self.nv = ctx, int(n), nv
        self.generation = 0          # bumped by every forward stage
        self.states = (tgs_state * nv)()
        caps = pair_capacity if isinstance(pair_capacity, (list, tuple)) else [pair_capacity] * nv
        self.views = [View(ctx, n, cam, stride, ox, oy, tile, bg, pair_capacity=caps[k],
                           lds_batch=lds_batch, state=self.states[k],
                           pixels_per_thread=pixels_per_thread)
                      for k, (cam, stride, ox, oy) in enumerate(views)]
        self.cams = (tgs_camera * nv)(*[v.cam_s for v in self.views])
        self.dils = (tgs_dilation * nv)(*[v.dil for v in self.views])
        self.opt = options_struct(tile, bg, lds_batch, pixels_per_thread)
        self.io = (tgs_view_io * nv)()
        f32, i32 = torch.float32, torch.int32
        self.images = [torch.zeros(v.image_shape, dtype=f32, device="cuda") for v in self.views]
        self.dL = [torch.zeros(v.image_shape, dtype=f32, device="cuda") for v in self.views]
        self.targets = [None] * nv
        self.loss = torch.zeros(nv, dtype=torch.float64, device="cuda")
        self.t_final = self.last_contrib = self.n_eval = self.n_blend = self.n_tested = None
        if counts:
            px = lambda v, dt: torch.zeros(v.image_shape[1:], dtype=dt, device="cuda")
            self.t_final = [px(v, f32) for v in self.views]
            self.last_contrib = [px(v, i32) for v in self.views]
            self.n_eval = [px(v, i32) for v in self.views]
            self.n_blend = [px(v, i32) for v in self.views]
            self.n_tested = [px(v, i32) for v in self.views]
        # each view's own densification statistics (besides the summed ones)
        self.view_pos = self.view_col = self.view_vis = None
        if view_stats:
            self.view_pos = [torch.zeros(n, dtype=f32, device="cuda") for _ in range(nv)]
            self.view_col = [torch.zeros(n, dtype=f32, device="cuda") for _ in range(nv)]
            self.view_vis = [torch.zeros(n, dtype=torch.uint8, device="cuda") for _ in range(nv)]
        for k in range(nv):
            io = self.io[k]
            io.image = _ptr(self.images[k])
            io.dL_dimage = _ptr(self.dL[k])
            if view_stats:
                io.pos_stat = _ptr(self.view_pos[k])
                io.col_stat = _ptr(self.view_col[k])
                io.visible = _ptr(self.view_vis[k])
            if counts:
                io.t_final = _ptr(self.t_final[k])
                io.last_contrib = _ptr(self.last_contrib[k])
                io.n_eval = _ptr(self.n_eval[k])
                io.n_blend = _ptr(self.n_blend[k])
                io.n_tested = _ptr(self.n_tested[k])

    def set_targets(self, targets):
        for k, t in enumerate(targets):
            v = self.views[k]
            assert tuple(t.shape) == (3, v.cam_s.height, v.cam_s.width) and t.is_contiguous()
            self.targets[k] = t
            self.io[k].target = _ptr(t)

    def forward(self, scene: DeviceScene, stream=None):
        g = scene.struct()
        self.generation += 1
        check(lib().tgs_batch_forward(self.ctx.handle, C.byref(g), self.nv, self.cams, self.dils,
                                      C.byref(self.opt), self.states, self.io, _stream(stream)))
        return self.images

    # -- stages (each one batched call) --------------------------------------
    def preprocess_fwd(self, scene: DeviceScene, stream=None):
        g = scene.struct()
        self.generation += 1
        check(lib().tgs_batch_preprocess_fwd(self.ctx.handle, C.byref(g), self.nv, self.cams,
                                             self.dils, C.byref(self.opt), self.states,
                                             _stream(stream)))

    def bin_sort(self, scene: DeviceScene, stream=None):
        g = scene.struct()
        self.generation += 1
        check(lib().tgs_batch_bin_sort(self.ctx.handle, C.byref(g), self.nv, self.cams, self.dils,
                                       C.byref(self.opt), self.states, _stream(stream)))

    def raster_fwd(self, stream=None):
        self.generation += 1
        check(lib().tgs_batch_raster_fwd(self.ctx.handle, self.n, self.nv, self.cams, self.dils,
                                         C.byref(self.opt), self.states, self.io, _stream(stream)))

    def raster_bwd(self, stream=None):
        check(lib().tgs_batch_raster_bwd(self.ctx.handle, self.n, self.nv, self.cams, self.dils,
                                         C.byref(self.opt), self.states, self.io, _stream(stream)))

    def preprocess_bwd(self, scene: DeviceScene, grads: DeviceScene, pos_stat=None, col_stat=None,
                       visible=None, stream=None):
        g = scene.struct()
        out = _grads_struct(grads)
        check(lib().tgs_batch_preprocess_bwd(self.ctx.handle, C.byref(g), self.nv, self.cams,
                                             self.dils, C.byref(self.opt), self.states, self.io,
                                             C.byref(out), _ptr(pos_stat), _ptr(col_stat),
                                             _ptr(visible), _stream(stream)))

    def l1_grad(self, stream=None):
        if any(t is None for t in self.targets):
            raise ValueError("set_targets first")
        check(lib().tgs_batch_l1_grad(self.ctx.handle, self.nv, self.cams, self.dils, self.io,
                                      _ptr(self.loss), _stream(stream)))
        return self.loss

    def backward(self, scene: DeviceScene, grads: DeviceScene, pos_stat=None, col_stat=None,
                 visible=None, stream=None):
        g = scene.struct()
        out = _grads_struct(grads)
        check(lib().tgs_batch_backward(self.ctx.handle, C.byref(g), self.nv, self.cams, self.dils,
                                       C.byref(self.opt), self.states, self.io, C.byref(out),
                                       _ptr(pos_stat), _ptr(col_stat), _ptr(visible),
                                       _stream(stream)))
        return grads

    def step(self, scene: DeviceScene, grads: DeviceScene, pos_stat=None, col_stat=None,
             visible=None, stream=None):
        """Forward, L1 loss gradient and backward of every view (no synchronisation)."""
        self.forward(scene, stream)
        self.l1_grad(stream)
        self.backward(scene, grads, pos_stat, col_stat, visible, stream)

    def pair_counts(self, stream=None) -> list:
        """Device pair counts read back (synchronises); raises TgsError on overflow."""
        st = lib().tgs_pair_counts(self.ctx.handle, self.nv, self.states, _stream(stream))
        counts = [int(s.pair_count) for s in self.states]
        if st != TGS_OK:
            raise TgsError(st, lib().tgs_last_error().decode())
        return counts

    def fit_capacity(self, scene: DeviceScene, slack: float = 1.1, tries: int = 4) -> list:
        """Run forwards until every view's pairs fit its workspace; returns the counts.
        Workspaces are re-allocated, so capture graphs only after this."""
        for _ in range(tries):
            self.forward(scene)
            lib().tgs_pair_counts(self.ctx.handle, self.nv, self.states, _stream(None))
            over = [k for k, s in enumerate(self.states) if s.pair_count > s.pair_capacity]
            if not over:
                return [int(s.pair_count) for s in self.states]
            for k in over:
                self.views[k].reserve(int(self.states[k].pair_count * slack) + 4096)
        raise TgsError(TGS_ERR_CAPACITY, "pair capacity did not converge")


class Adam:
    """Fused Adam over a list of float32 device tensors (one group each, with
    its own learning rate); moments and the device step counter are owned
    here.  ``step(grads)`` is one kernel pair, capturable in a graph."""

    def __init__(self, ctx: Context, params, lrs, betas=(0.9, 0.999), eps=1e-15):
        import torch
        if not 1 <= len(params) <= MAX_ADAM_GROUPS or len(lrs) != len(params):
            raise ValueError(f"1..{MAX_ADAM_GROUPS} groups with one learning rate each")
        for p in params:
            assert p.is_contiguous() and p.dtype == torch.float32 and p.is_cuda
        self.ctx, self.params = ctx, list(params)
        self.lrs = [float(x) for x in lrs]
        self.betas, self.eps = (float(betas[0]), float(betas[1])), float(eps)
        self.exp_avg = [torch.zeros_like(p) for p in self.params]
        self.exp_avg_sq = [torch.zeros_like(p) for p in self.params]
        self.state = torch.zeros(ADAM_STATE_BYTES // 4, dtype=torch.int32, device="cuda")
        self._groups = (tgs_adam_group * len(self.params))()

    @property
    def step_count(self) -> int:
        return int(self.state[0].item())

    def step(self, grads, stream=None):
        for k, (p, g, m, v) in enumerate(zip(self.params, grads, self.exp_avg, self.exp_avg_sq)):
            assert g.shape == p.shape and g.is_contiguous() and g.dtype == p.dtype
            self._groups[k] = tgs_adam_group(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(),
                                             self.lrs[k])
        check(lib().tgs_adam_step(self.ctx.handle, self._groups, len(self.params), self.betas[0],
                                  self.betas[1], self.eps, _ptr(self.state), _stream(stream)))


def densify_select(ctx: Context, pos_sum, col_sum, count, tau_pos: float, tau_col: float,
                   color_active: bool, budget: int = -1, stream=None):
    """Selection mask (uint8 [n]) and the device count of selected Gaussians."""
    import torch
    n = int(pos_sum.numel())
    need = C.c_uint64()
    check(lib().tgs_densify_query(n, C.byref(need)))
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device="cuda")
    base = (int(ws.data_ptr()) + 255) // 256 * 256
    sel = torch.empty(n, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    check(lib().tgs_densify_select(ctx.handle, n, _ptr(pos_sum), _ptr(col_sum), _ptr(count),
                                   float(tau_pos), float(tau_col), int(bool(color_active)),
                                   int(budget), _ptr(sel), _ptr(cnt), base, int(need.value),
                                   _stream(stream)))
    return sel, cnt, ws
