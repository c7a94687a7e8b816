"""Thin ctypes binding of libgsmi (include/gs.h): argument marshalling only.

Every function named ``gs_*`` here calls the C entry point of the same name;
PyTorch tensors serve only as device memory and the current HIP stream.
Tensors holding uint32/uint64 data use int32/int64 storage.  All work runs
in the library's HIP kernels; there is no fallback path: importing this
module fails if ``libgsmi.so`` is missing, and calls fail on a machine
without a GPU.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import scenes

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2409_09295_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

GS_OK = 0
GS_ERR_INVALID_ARGUMENT = 1
GS_ERR_CAPACITY = 2
GS_ERR_HIP = 3
GS_ERR_UNSUPPORTED = 4
GS_BWD_NO_POSE = 1
GS_BWD_POSE_ONLY = 2
GS_BWD_OVERWRITE = 4
GS_BWD_KEEP_CLEAR = 8
GS_KERNEL_PREPROCESS = 0
GS_KERNEL_BIN_SORT = 1
GS_KERNEL_RENDER_FWD = 2
GS_KERNEL_RENDER_BWD = 3
GS_KERNEL_PROJECT_BWD = 4
GS_TUNE_FWD_PIXELS_PER_LANE = 0
GS_TUNE_BWD_PIXELS_PER_LANE = 1
GS_TUNE_FWD_SCHEDULE = 2
GS_TUNE_BWD_SCHEDULE = 3
GS_TUNE_FWD_STAGE = 4
GS_TUNE_BWD_STAGE = 5
GS_SCHEDULE_HEAVIEST_FIRST = 1
GS_SCHEDULE_TILE_ID = 2
GS_SCHEDULE_PERSISTENT = 3
GS_SCHEDULE_PERSISTENT_HALF = 4
GS_QUEUE_COUNTERS = 8
GS_QUEUE_STRIDE = 32
GS_QUEUE_WORDS = 1024
GS_MAX_VIEWS = 64
TILE = 16

_p = ctypes.c_void_p


class GsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.gs_last_error().decode(errors="replace")
        name = _lib.gs_status_string(status).decode()
        super().__init__(f"{where}: {name}: {msg}")


class gs_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pad", ctypes.c_int32 * 2)]


class gs_gaussians(ctypes.Structure):
    _fields_ = [("means", _p), ("log_scales", _p), ("quats", _p), ("opacity_logits", _p),
                ("sh", _p), ("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32)]


class gs_views(ctypes.Structure):
    _fields_ = [("cams_host", _p), ("cams_dev", _p), ("n_views", ctypes.c_int32),
                ("tile_size", ctypes.c_int32)]


class gs_projected(ctypes.Structure):
    _fields_ = [("xy", _p), ("conic_opacity", _p), ("rgb_depth", _p), ("radius", _p),
                ("tiles", _p)]


class gs_bins(ctypes.Structure):
    _fields_ = [("keys", _p), ("values", _p), ("ranges", _p), ("n_keys", _p),
                ("capacity", ctypes.c_int64), ("order", _p), ("queue", _p)]


class gs_grads(ctypes.Structure):
    _fields_ = [("means", _p), ("log_scales", _p), ("quats", _p), ("opacity_logits", _p),
                ("sh", _p), ("xi", _p)]


assert ctypes.sizeof(gs_camera) == 80

_S = ctypes.c_void_p
_lib.gs_status_string.restype = ctypes.c_char_p
_lib.gs_status_string.argtypes = [ctypes.c_int]
_lib.gs_last_error.restype = ctypes.c_char_p
_lib.gs_version.restype = ctypes.c_char_p
_lib.gs_num_tiles.restype = ctypes.c_int64
_lib.gs_num_tiles.argtypes = [ctypes.POINTER(gs_views)]
_lib.gs_num_pixels.restype = ctypes.c_int64
_lib.gs_num_pixels.argtypes = [ctypes.POINTER(gs_views)]
_lib.gs_preprocess.argtypes = [ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_views),
                               ctypes.POINTER(gs_projected), _S]
_lib.gs_bin_sort_workspace_size.restype = ctypes.c_size_t
_lib.gs_bin_sort_workspace_size.argtypes = [ctypes.c_int64, ctypes.POINTER(gs_views), ctypes.c_int64]
_lib.gs_bin_sort.argtypes = [ctypes.POINTER(gs_projected), ctypes.c_int64, ctypes.POINTER(gs_views),
                             ctypes.POINTER(gs_bins), ctypes.POINTER(ctypes.c_uint32), _p,
                             ctypes.c_size_t, _S]
_lib.gs_render_fwd.argtypes = [ctypes.POINTER(gs_projected), ctypes.c_int64, ctypes.POINTER(gs_bins),
                               ctypes.POINTER(gs_views), ctypes.POINTER(ctypes.c_float), _p, _p, _p,
                               _p, _S]
_lib.gs_render_fwd_l1_workspace_size.restype = ctypes.c_size_t
_lib.gs_render_fwd_l1_workspace_size.argtypes = [ctypes.POINTER(gs_views)]
_lib.gs_render_fwd_l1.argtypes = [ctypes.POINTER(gs_projected), ctypes.c_int64, ctypes.POINTER(gs_bins),
                                  ctypes.POINTER(gs_views), ctypes.POINTER(ctypes.c_float), _p, _p, _p,
                                  _p, _p, _p, _p, ctypes.c_size_t, _S]
_lib.gs_render_fwd_l1_noalloc.argtypes = [ctypes.POINTER(gs_projected), ctypes.c_int64,
                                          ctypes.POINTER(gs_bins), ctypes.POINTER(gs_views),
                                          ctypes.POINTER(ctypes.c_float), _p, _p, _p, _p, _p, _p, _S]
GS_NOALLOC_MAX_TILES = 262144
_lib.gs_render_bwd_workspace_size.restype = ctypes.c_size_t
_lib.gs_render_bwd_workspace_size.argtypes = [ctypes.c_int64, ctypes.POINTER(gs_views)]
_lib.gs_render_bwd.argtypes = [ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_projected),
                               ctypes.POINTER(gs_bins), ctypes.POINTER(gs_views),
                               ctypes.POINTER(ctypes.c_float), _p, _p, _p, ctypes.POINTER(gs_grads),
                               ctypes.c_uint32, _p, ctypes.c_size_t, _S]
_lib.gs_adam_step.argtypes = [_p, _p, _p, _p, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, ctypes.c_int32, _p, _S]
_lib.gs_l1_loss_grad.argtypes = [_p, _p, ctypes.POINTER(gs_views), _p, _p, _S]
_lib.gs_set_kernel_events.argtypes = [ctypes.c_int, _p, _p]
_lib.gs_set_tuning.argtypes = [ctypes.c_int, ctypes.c_int]
_lib.gs_get_tuning.argtypes = [ctypes.c_int]
_lib.gs_adam_step_dev.argtypes = [_p, _p, _p, _p, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, _p, ctypes.c_int32, _p, _p,
                                  ctypes.c_int64, _S]


class gs_adam_group(ctypes.Structure):
    _fields_ = [("p", _p), ("g", _p), ("m", _p), ("v", _p), ("n", ctypes.c_int64),
                ("lr", ctypes.c_float)]


GS_ADAM_MAX_GROUPS = 8
_lib.gs_adam_step_groups_dev.argtypes = [ctypes.POINTER(gs_adam_group), ctypes.c_int32,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_float, _p, _p,
                                         ctypes.c_int64, _S]

_lib.gs_render_error.argtypes = [ctypes.POINTER(gs_projected), ctypes.c_int64, ctypes.POINTER(gs_bins),
                                 ctypes.POINTER(gs_views), _p, _p, _p, _p, _S]
_lib.gs_active_set.argtypes = [_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, _p, _p, _p, _p, _S]
_lib.gs_adam_step_groups_masked_dev.argtypes = [ctypes.POINTER(gs_adam_group), ctypes.c_int32,
                                                ctypes.c_float, ctypes.c_float, ctypes.c_float, _p, _p,
                                                ctypes.c_int64, _p, ctypes.c_int64, _S]


class gs_concat_array(ctypes.Structure):
    _fields_ = [("a", _p), ("b", _p), ("dst", _p), ("components", ctypes.c_int32),
                ("fill", ctypes.c_float)]


class gs_compact_array(ctypes.Structure):
    _fields_ = [("src", _p), ("dst", _p), ("components", ctypes.c_int32)]


GS_SOA_MAX_ARRAYS = 16
_lib.gs_concat.argtypes = [ctypes.POINTER(gs_concat_array), ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_int64, _S]
_lib.gs_prune_mask.argtypes = [_p, ctypes.c_int64, ctypes.c_float, _p, _S]
_lib.gs_compact_workspace_size.restype = ctypes.c_size_t
_lib.gs_compact_workspace_size.argtypes = [ctypes.c_int64]
_lib.gs_compact.argtypes = [ctypes.POINTER(gs_compact_array), ctypes.c_int32, ctypes.c_int64, _p, _p,
                            _p, ctypes.c_size_t, _S]
_lib.gs_iso_loss_grad.argtypes = [_p, ctypes.c_int64, ctypes.c_float, _p, _p, _S]
_lib.gs_pose_adam_step.argtypes = [_p, _p, _p, _p, ctypes.c_int32, _p, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, _p, _S]

GS_MEM_MAP, GS_MEM_KEYFRAMES, GS_MEM_POSES, GS_MEM_INIT = 0, 1, 2, 3
GS_MEM_RENDER_TARGETS, GS_MEM_BLEND_STATE, GS_MEM_OPTIMISER, GS_MEM_CATEGORIES = 4, 5, 6, 7
MEM_CATEGORY_NAMES = ("map", "keyframes", "poses", "init", "render_targets", "blend_state", "optimiser")
_lib.gs_mem_track.argtypes = [ctypes.c_int32, ctypes.c_int64]
_lib.gs_mem_report.argtypes = [_p, _p, _p, _p]
_lib.gs_mem_reset_peaks.argtypes = []

EXPORTED = ("gs_status_string", "gs_last_error", "gs_version", "gs_num_tiles", "gs_num_pixels",
            "gs_preprocess", "gs_bin_sort_workspace_size", "gs_bin_sort", "gs_render_fwd",
            "gs_render_bwd_workspace_size", "gs_render_bwd", "gs_adam_step", "gs_l1_loss_grad",
            "gs_set_kernel_events", "gs_adam_step_dev", "gs_adam_step_groups_dev",
            "gs_render_fwd_l1_workspace_size", "gs_render_fwd_l1", "gs_render_fwd_l1_noalloc",
            "gs_set_tuning", "gs_get_tuning", "gs_render_error", "gs_active_set",
            "gs_adam_step_groups_masked_dev", "gs_concat", "gs_prune_mask",
            "gs_compact_workspace_size", "gs_compact", "gs_iso_loss_grad", "gs_pose_adam_step",
            "gs_mem_track", "gs_mem_report", "gs_mem_reset_peaks")


def lib() -> ctypes.CDLL:
    return _lib


def version() -> str:
    return _lib.gs_version().decode()


def _check(status: int, where: str):
    if status != GS_OK:
        raise GsError(status, where)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _bg(bg) -> Optional[ctypes.Array]:
    if bg is None:
        return None
    return (ctypes.c_float * 3)(*[float(x) for x in bg])


# ---------------------------------------------------------------------------
# containers (device memory owned by torch tensors)
# ---------------------------------------------------------------------------

class Views:
    """A batch of cameras: host records (sizes, tile layout) plus a device copy
    (poses and intrinsics read by the kernels)."""

    def __init__(self, cams: Sequence[scenes.Camera], device="cuda", tile_size: int = TILE):
        recs = scenes.camera_records(list(cams))
        self._host = (gs_camera * len(recs))()
        ctypes.memmove(self._host, recs.ctypes.data, recs.nbytes)
        self.records = recs
        self.n_views = len(recs)
        self.tile_size = tile_size
        self.dev = torch.from_numpy(recs.view(np.uint8).copy()).to(device)
        self.sizes = [(int(r["width"]), int(r["height"])) for r in recs]
        self.struct = gs_views(ctypes.cast(self._host, _p), self.dev.data_ptr(), self.n_views, tile_size)

    def update_poses(self, cams: Sequence[scenes.Camera]):
        """Overwrite poses/intrinsics on the device (sizes must not change)."""
        recs = scenes.camera_records(list(cams))
        if [(int(r["width"]), int(r["height"])) for r in recs] != self.sizes:
            raise ValueError("image sizes changed")
        self.records = recs
        ctypes.memmove(self._host, recs.ctypes.data, recs.nbytes)
        self.dev.copy_(torch.from_numpy(recs.view(np.uint8).copy()))

    def download_poses(self):
        """Host records <- device records (after poses were moved on the device)."""
        recs = self.dev.cpu().numpy().view(self.records.dtype).copy()
        self.records = recs
        ctypes.memmove(self._host, recs.ctypes.data, recs.nbytes)
        return recs

    @property
    def n_tiles(self) -> int:
        v = _lib.gs_num_tiles(ctypes.byref(self.struct))
        if v < 0:
            raise GsError(GS_ERR_INVALID_ARGUMENT, "gs_num_tiles")
        return int(v)

    @property
    def n_pixels(self) -> int:
        v = _lib.gs_num_pixels(ctypes.byref(self.struct))
        if v < 0:
            raise GsError(GS_ERR_INVALID_ARGUMENT, "gs_num_pixels")
        return int(v)

    def pixel_offsets(self) -> List[int]:
        out, acc = [], 0
        for w, h in self.sizes:
            out.append(acc)
            acc += w * h
        return out

    def split_images(self, flat: torch.Tensor) -> List[torch.Tensor]:
        """Packed [V][3][H][W] buffer -> list of (3, H, W) views."""
        out = []
        for off, (w, h) in zip(self.pixel_offsets(), self.sizes):
            out.append(flat[3 * off:3 * (off + w * h)].view(3, h, w))
        return out

    def split_maps(self, flat: torch.Tensor) -> List[torch.Tensor]:
        """Packed [V][H][W] buffer -> list of (H, W) views."""
        return [flat[off:off + w * h].view(h, w) for off, (w, h) in zip(self.pixel_offsets(), self.sizes)]


@dataclasses.dataclass
class Gaussians:
    means: torch.Tensor            # (3, N) float32
    log_scales: torch.Tensor       # (3, N)
    quats: torch.Tensor            # (4, N)
    opacity_logits: torch.Tensor   # (N,)
    sh: torch.Tensor               # (3, K, N)
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @classmethod
    def from_map(cls, gmap: scenes.GaussianMap, device="cuda") -> "Gaussians":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(t(gmap.means), t(gmap.log_scales), t(gmap.quats), t(gmap.opacity_logits),
                   t(gmap.sh), gmap.sh_degree)

    def tensors(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logits, self.sh]

    def struct(self) -> gs_gaussians:
        for x in self.tensors():
            if x.dtype != torch.float32 or not x.is_contiguous():
                raise ValueError("Gaussian parameters must be contiguous float32")
        return gs_gaussians(*[_ptr(x) for x in self.tensors()], self.n, self.sh_degree)


@dataclasses.dataclass
class Projected:
    xy: torch.Tensor               # (V, N, 2) float32
    conic_opacity: torch.Tensor    # (V, N, 4)
    rgb_depth: torch.Tensor        # (V, N, 4)
    radius: torch.Tensor           # (V, N) int32
    tiles: Optional[torch.Tensor] = None   # (V, N) int32 storage of uint32, or not stored

    @classmethod
    def empty(cls, n_views: int, n: int, device="cuda") -> "Projected":
        f = lambda *s: torch.empty(*s, dtype=torch.float32, device=device)
        i = lambda: torch.empty(n_views, n, dtype=torch.int32, device=device)
        return cls(f(n_views, n, 2), f(n_views, n, 4), f(n_views, n, 4), i(), i())

    @classmethod
    def from_splats(cls, sp: scenes.SplatSet, device="cuda") -> "Projected":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(t(sp.xy), t(sp.conic_opacity), t(sp.rgb_depth), t(sp.radius.astype(np.int32)))

    def struct(self) -> gs_projected:
        return gs_projected(_ptr(self.xy), _ptr(self.conic_opacity), _ptr(self.rgb_depth),
                            _ptr(self.radius), _ptr(self.tiles) if self.tiles is not None else None)


@dataclasses.dataclass
class Bins:
    keys: Optional[torch.Tensor]   # (capacity,) int64 storage of uint64, or not written
    values: torch.Tensor   # (capacity,) int32 storage of uint32
    ranges: torch.Tensor   # (n_tiles, 2) int32 storage of uint32
    n_keys: torch.Tensor   # (1,) int32 storage of uint32
    capacity: int
    order: Optional[torch.Tensor] = None   # (n_tiles,) int32 storage of uint32, or not computed
    queue: Optional[torch.Tensor] = None   # (GS_QUEUE_WORDS,) int32 storage of uint32 tile counters

    @classmethod
    def empty(cls, capacity: int, n_tiles: int, device="cuda", order: bool = True,
              keys: bool = True) -> "Bins":
        """keys=False: no key array (gs_bin_sort then sorts 32-bit tile ids
        in its workspace; values, ranges and order are the same)."""
        cap = max(int(capacity), 1)
        return cls(torch.empty(cap, dtype=torch.int64, device=device) if keys else None,
                   torch.empty(cap, dtype=torch.int32, device=device),
                   torch.empty(n_tiles, 2, dtype=torch.int32, device=device),
                   torch.zeros(1, dtype=torch.int32, device=device), int(capacity),
                   torch.empty(max(n_tiles, 1), dtype=torch.int32, device=device) if order else None,
                   torch.zeros(GS_QUEUE_WORDS, dtype=torch.int32, device=device))

    def struct(self) -> gs_bins:
        return gs_bins(_ptr(self.keys), _ptr(self.values), _ptr(self.ranges), _ptr(self.n_keys),
                       self.capacity, _ptr(self.order) if self.order is not None else None,
                       _ptr(self.queue) if self.queue is not None else None)


@dataclasses.dataclass
class Grads:
    means: Optional[torch.Tensor]
    log_scales: Optional[torch.Tensor]
    quats: Optional[torch.Tensor]
    opacity_logits: Optional[torch.Tensor]
    sh: Optional[torch.Tensor]
    xi: Optional[torch.Tensor]     # (V, 6) float32

    @classmethod
    def zeros_like(cls, g: Gaussians, n_views: int) -> "Grads":
        z = torch.zeros_like
        return cls(z(g.means), z(g.log_scales), z(g.quats), z(g.opacity_logits), z(g.sh),
                   torch.zeros(n_views, 6, dtype=torch.float32, device=g.means.device))

    def struct(self) -> gs_grads:
        return gs_grads(_ptr(self.means), _ptr(self.log_scales), _ptr(self.quats),
                        _ptr(self.opacity_logits), _ptr(self.sh), _ptr(self.xi))


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """Caller-owned scratch (torch's allocator returns >= 256-byte aligned blocks)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def gs_preprocess(g: Gaussians, views: Views, out: Projected, stream=None) -> None:
    gs_, ps = g.struct(), out.struct()
    _check(_lib.gs_preprocess(ctypes.byref(gs_), ctypes.byref(views.struct), ctypes.byref(ps),
                              _stream(stream)), "gs_preprocess")


def _capacity_error(status: int, required: int) -> GsError:
    err = GsError(status, "gs_bin_sort")
    err.required = required
    return err


def gs_bin_sort_workspace_size(n: int, views: Views, capacity: int) -> int:
    return int(_lib.gs_bin_sort_workspace_size(n, ctypes.byref(views.struct), capacity))


def gs_bin_sort(p: Projected, n: int, views: Views, bins: Bins, ws: torch.Tensor,
                sync: bool = True, stream=None) -> Optional[int]:
    """Returns the key count when ``sync`` (raises GsError(GS_ERR_CAPACITY)
    with ``.required`` set if it exceeds the capacity); None otherwise."""
    ps, bs = p.struct(), bins.struct()
    cnt = ctypes.c_uint32(0)
    st = _lib.gs_bin_sort(ctypes.byref(ps), n, ctypes.byref(views.struct), ctypes.byref(bs),
                          ctypes.byref(cnt) if sync else None, _ptr(ws), ws.numel(), _stream(stream))
    if st != GS_OK:
        # built and raised in one expression: an exception held in a local of
        # this frame would reference itself through its traceback, keeping the
        # caller's frame (and everything it holds) alive until a cyclic GC pass
        raise _capacity_error(st, int(cnt.value))
    return int(cnt.value) if sync else None


def gs_render_fwd(p: Projected, n: int, bins: Bins, views: Views, bg, image: torch.Tensor,
                  final_T: torch.Tensor, n_contrib: torch.Tensor, depth: Optional[torch.Tensor] = None,
                  stream=None) -> None:
    ps, bs = p.struct(), bins.struct()
    _check(_lib.gs_render_fwd(ctypes.byref(ps), n, ctypes.byref(bs), ctypes.byref(views.struct),
                              _bg(bg), _ptr(image), _ptr(final_T), _ptr(n_contrib), _ptr(depth),
                              _stream(stream)), "gs_render_fwd")


def gs_render_fwd_l1_workspace_size(views: Views) -> int:
    return int(_lib.gs_render_fwd_l1_workspace_size(ctypes.byref(views.struct)))


def gs_render_fwd_l1(p: Projected, n: int, bins: Bins, views: Views, bg, image: torch.Tensor,
                     final_T: torch.Tensor, n_contrib: torch.Tensor, target: torch.Tensor,
                     dL_dimage: torch.Tensor, loss: Optional[torch.Tensor], ws: torch.Tensor,
                     stream=None) -> None:
    ps, bs = p.struct(), bins.struct()
    _check(_lib.gs_render_fwd_l1(ctypes.byref(ps), n, ctypes.byref(bs), ctypes.byref(views.struct),
                                 _bg(bg), _ptr(image), _ptr(final_T), _ptr(n_contrib), _ptr(target),
                                 _ptr(dL_dimage), _ptr(loss), _ptr(ws), ws.numel(), _stream(stream)),
           "gs_render_fwd_l1")


def gs_render_fwd_l1_noalloc(p: Projected, n: int, bins: Bins, views: Views, bg, image: torch.Tensor,
                             final_T: torch.Tensor, n_contrib: torch.Tensor, target: torch.Tensor,
                             dL_dimage: torch.Tensor, loss: Optional[torch.Tensor], stream=None) -> None:
    """gs_render_fwd_l1 with the library's static scratch (no workspace)."""
    ps, bs = p.struct(), bins.struct()
    _check(_lib.gs_render_fwd_l1_noalloc(ctypes.byref(ps), n, ctypes.byref(bs), ctypes.byref(views.struct),
                                         _bg(bg), _ptr(image), _ptr(final_T), _ptr(n_contrib), _ptr(target),
                                         _ptr(dL_dimage), _ptr(loss), _stream(stream)),
           "gs_render_fwd_l1_noalloc")


def gs_render_bwd_workspace_size(n: int, views: Views) -> int:
    return int(_lib.gs_render_bwd_workspace_size(n, ctypes.byref(views.struct)))


def gs_render_bwd(g: Gaussians, p: Projected, bins: Bins, views: Views, bg, dL_dimage: torch.Tensor,
                  final_T: torch.Tensor, n_contrib: torch.Tensor, grads: Grads, flags: int,
                  ws: torch.Tensor, stream=None) -> None:
    gs_, ps, bs, gr = g.struct(), p.struct(), bins.struct(), grads.struct()
    _check(_lib.gs_render_bwd(ctypes.byref(gs_), ctypes.byref(ps), ctypes.byref(bs),
                              ctypes.byref(views.struct), _bg(bg), _ptr(dL_dimage), _ptr(final_T),
                              _ptr(n_contrib), ctypes.byref(gr), flags, _ptr(ws), ws.numel(),
                              _stream(stream)), "gs_render_bwd")


def gs_adam_step(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, step: int = 1,
                 mask: Optional[torch.Tensor] = None, stream=None) -> None:
    n = p.numel()
    for x in (g, m, v):
        if x.numel() != n:
            raise ValueError("Adam tensors must have equal sizes")
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != n):
        raise ValueError("mask must be uint8 with one entry per parameter")
    _check(_lib.gs_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), n, lr, beta1, beta2, eps, step,
                             _ptr(mask), _stream(stream)), "gs_adam_step")


def gs_adam_step_dev(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float,
                     beta1: float, beta2: float, eps: float, step_dev: torch.Tensor, commit: bool,
                     mask: Optional[torch.Tensor] = None, guard_n_keys: Optional[torch.Tensor] = None,
                     guard_capacity: int = 0, stream=None) -> None:
    n = p.numel()
    for x in (g, m, v):
        if x.numel() != n:
            raise ValueError("Adam tensors must have equal sizes")
    if step_dev.dtype != torch.int32 or step_dev.numel() != 1:
        raise ValueError("step_dev must be one int32")
    _check(_lib.gs_adam_step_dev(_ptr(p), _ptr(g), _ptr(m), _ptr(v), n, lr, beta1, beta2, eps,
                                 _ptr(step_dev), int(bool(commit)), _ptr(mask), _ptr(guard_n_keys),
                                 guard_capacity, _stream(stream)), "gs_adam_step_dev")


def adam_groups(groups: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor, float]]):
    """Host array of gs_adam_group from (p, g, m, v, lr) tuples (kept by the caller)."""
    arr = (gs_adam_group * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        n = p.numel()
        for x in (g, m, v):
            if x.numel() != n:
                raise ValueError("Adam tensors must have equal sizes")
        arr[k] = gs_adam_group(_ptr(p), _ptr(g), _ptr(m), _ptr(v), n, lr)
    return arr


def gs_adam_step_groups_dev(groups, beta1: float, beta2: float, eps: float, step_dev: torch.Tensor,
                            guard_n_keys: Optional[torch.Tensor] = None, guard_capacity: int = 0,
                            stream=None) -> None:
    """groups: an array from adam_groups()."""
    if step_dev.dtype != torch.int32 or step_dev.numel() != 1:
        raise ValueError("step_dev must be one int32")
    _check(_lib.gs_adam_step_groups_dev(groups, len(groups), beta1, beta2, eps, _ptr(step_dev),
                                        _ptr(guard_n_keys), guard_capacity, _stream(stream)),
           "gs_adam_step_groups_dev")


def gs_render_error(p: Projected, n: int, bins: Bins, views: Views, image: torch.Tensor,
                    target: torch.Tensor, n_contrib: torch.Tensor, err: torch.Tensor,
                    stream=None) -> None:
    """err: float32 (V, n), overwritten with E_k(g)."""
    if err.dtype != torch.float32 or err.numel() != views.n_views * n:
        raise ValueError("err must be float32 with n_views * n entries")
    ps, bs = p.struct(), bins.struct()
    _check(_lib.gs_render_error(ctypes.byref(ps), n, ctypes.byref(bs), ctypes.byref(views.struct),
                                _ptr(image), _ptr(target), _ptr(n_contrib), _ptr(err), _stream(stream)),
           "gs_render_error")


def gs_active_set(err: torch.Tensor, n: int, n_views: int, eps: float, mask: torch.Tensor,
                  always: Optional[torch.Tensor] = None, err_max: Optional[torch.Tensor] = None,
                  n_active: Optional[torch.Tensor] = None, stream=None) -> None:
    if err.dtype != torch.float32 or err.numel() < n_views * n:
        raise ValueError("err must be float32 with n_views * n entries")
    if mask.dtype != torch.uint8 or mask.numel() < n:
        raise ValueError("mask must be uint8 with n entries")
    if always is not None and (always.dtype != torch.uint8 or always.numel() < n):
        raise ValueError("always must be uint8 with n entries")
    _check(_lib.gs_active_set(_ptr(err), n, n_views, eps, _ptr(always), _ptr(mask), _ptr(err_max),
                              _ptr(n_active), _stream(stream)), "gs_active_set")


def gs_adam_step_groups_masked_dev(groups, beta1: float, beta2: float, eps: float,
                                   step_dev: torch.Tensor, gauss_mask: torch.Tensor, n_gauss: int,
                                   guard_n_keys: Optional[torch.Tensor] = None,
                                   guard_capacity: int = 0, stream=None) -> None:
    """groups: an array from adam_groups(); gauss_mask: uint8 [n_gauss]."""
    if step_dev.dtype != torch.int32 or step_dev.numel() != 1:
        raise ValueError("step_dev must be one int32")
    if gauss_mask.dtype != torch.uint8 or gauss_mask.numel() != n_gauss:
        raise ValueError("gauss_mask must be uint8 with n_gauss entries")
    _check(_lib.gs_adam_step_groups_masked_dev(groups, len(groups), beta1, beta2, eps, _ptr(step_dev),
                                               _ptr(gauss_mask), n_gauss, _ptr(guard_n_keys),
                                               guard_capacity, _stream(stream)),
           "gs_adam_step_groups_masked_dev")


def gs_concat(arrays: Sequence[Tuple[torch.Tensor, Optional[torch.Tensor], torch.Tensor, int, float]],
              n_a: int, n_b: int, stream=None) -> None:
    """arrays: (a [C*n_a], b [C*n_b] or None, dst [C*(n_a+n_b)], C, fill) tuples."""
    arr = (gs_concat_array * len(arrays))()
    for k, (a, b, dst, c, fill) in enumerate(arrays):
        if a.numel() != c * n_a or dst.numel() != c * (n_a + n_b) or (b is not None and b.numel() != c * n_b):
            raise ValueError(f"array {k}: sizes do not match the component count")
        for t in (a, b, dst):
            if t is not None and t.dtype != torch.float32:
                raise ValueError("arrays are float32")
        arr[k] = gs_concat_array(_ptr(a), _ptr(b), _ptr(dst), c, fill)
    _check(_lib.gs_concat(arr, len(arrays), n_a, n_b, _stream(stream)), "gs_concat")


def gs_prune_mask(opacity_logits: torch.Tensor, min_opacity: float, keep: torch.Tensor,
                  stream=None) -> None:
    n = opacity_logits.numel()
    if keep.dtype != torch.uint8 or keep.numel() < n:
        raise ValueError("keep must be uint8 with n entries")
    _check(_lib.gs_prune_mask(_ptr(opacity_logits), n, min_opacity, _ptr(keep), _stream(stream)),
           "gs_prune_mask")


def gs_compact_workspace_size(n: int) -> int:
    return int(_lib.gs_compact_workspace_size(n))


def gs_compact(arrays: Sequence[Tuple[torch.Tensor, torch.Tensor, int]], n: int, keep: torch.Tensor,
               n_kept: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    """arrays: (src [C*n], dst [>= C*n], C) tuples; n_kept: int32 [1] (device)."""
    arr = (gs_compact_array * len(arrays))()
    for k, (src, dst, c) in enumerate(arrays):
        if src.numel() != c * n or dst.numel() < c * n:
            raise ValueError(f"array {k}: sizes do not match the component count")
        arr[k] = gs_compact_array(_ptr(src), _ptr(dst), c)
    _check(_lib.gs_compact(arr, len(arrays), n, _ptr(keep), _ptr(n_kept), _ptr(ws), ws.numel(),
                           _stream(stream)), "gs_compact")


def gs_iso_loss_grad(log_scales: torch.Tensor, weight: float, grad_log_scales: torch.Tensor,
                     loss: Optional[torch.Tensor] = None, stream=None) -> None:
    n = log_scales.shape[-1]
    if log_scales.numel() != 3 * n or grad_log_scales.numel() != 3 * n:
        raise ValueError("log-scales and their gradient are [3][n]")
    _check(_lib.gs_iso_loss_grad(_ptr(log_scales), n, weight, _ptr(grad_log_scales), _ptr(loss),
                                 _stream(stream)), "gs_iso_loss_grad")


def gs_pose_adam_step(views: Views, grad_xi: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                      step_dev: torch.Tensor, lr_trans: float, lr_rot: float, beta1: float = 0.9,
                      beta2: float = 0.999, eps: float = 1e-15,
                      view_mask: Optional[torch.Tensor] = None, stream=None) -> None:
    """Moves the device poses of ``views`` (their host records keep the old
    poses; ``Views.download_poses`` refreshes them)."""
    V = views.n_views
    for t in (grad_xi, m, v):
        if t.dtype != torch.float32 or t.numel() != 6 * V:
            raise ValueError("grad_xi, m, v must be float32 [n_views][6]")
    _check(_lib.gs_pose_adam_step(views.dev.data_ptr(), _ptr(grad_xi), _ptr(m), _ptr(v), V,
                                  _ptr(view_mask), lr_trans, lr_rot, beta1, beta2, eps, _ptr(step_dev),
                                  _stream(stream)), "gs_pose_adam_step")


def gs_mem_track(category: int, nbytes: int) -> None:
    _check(_lib.gs_mem_track(category, int(nbytes)), "gs_mem_track")


def gs_mem_report() -> dict:
    cur = (ctypes.c_int64 * GS_MEM_CATEGORIES)()
    peak = (ctypes.c_int64 * GS_MEM_CATEGORIES)()
    oc, op = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(_lib.gs_mem_report(cur, peak, ctypes.byref(oc), ctypes.byref(op)), "gs_mem_report")
    return {"current": dict(zip(MEM_CATEGORY_NAMES, list(cur))),
            "peak": dict(zip(MEM_CATEGORY_NAMES, list(peak))),
            "overhead_current": oc.value, "overhead_peak": op.value}


def gs_mem_reset_peaks() -> None:
    _check(_lib.gs_mem_reset_peaks(), "gs_mem_reset_peaks")


class Tracked:
    """Registers a buffer's bytes in the overhead-memory ledger for as long
    as this object lives (the constructor/destructor accounting the paper's
    memory profiler uses).  ``release()`` ends the registration early."""

    def __init__(self, category: int, t_or_bytes):
        self.category = category
        self.nbytes = int(t_or_bytes.numel() * t_or_bytes.element_size()
                          if isinstance(t_or_bytes, torch.Tensor) else t_or_bytes)
        gs_mem_track(category, self.nbytes)
        self._live = True

    def release(self):
        if self._live:
            self._live = False
            _lib.gs_mem_track(self.category, -self.nbytes)

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def gs_l1_loss_grad(image: torch.Tensor, target: torch.Tensor, views: Views, dL_dimage: torch.Tensor,
                    loss: Optional[torch.Tensor] = None, stream=None) -> None:
    _check(_lib.gs_l1_loss_grad(_ptr(image), _ptr(target), ctypes.byref(views.struct),
                                _ptr(dL_dimage), _ptr(loss), _stream(stream)), "gs_l1_loss_grad")


def gs_set_kernel_events(kernel: int, start: Optional["torch.cuda.Event"], stop: Optional["torch.cuda.Event"]) -> None:
    """Bracket every launch of ``kernel`` (GS_KERNEL_*) on this thread with the
    two (timing-enabled) events; None clears."""
    sp = None if start is None else start.cuda_event
    ep = None if stop is None else stop.cuda_event
    if (start is not None and not sp) or (stop is not None and not ep):
        raise ValueError("record each event once before registering it (torch creates it lazily)")
    _check(_lib.gs_set_kernel_events(kernel, sp, ep), "gs_set_kernel_events")


def gs_set_tuning(key: int, value: int) -> None:
    _check(_lib.gs_set_tuning(key, value), "gs_set_tuning")


def gs_get_tuning(key: int) -> int:
    return int(_lib.gs_get_tuning(key))


# ---------------------------------------------------------------------------
# learned / plain initialiser (include/gs_nn.h)
# ---------------------------------------------------------------------------

class gs_act(ctypes.Structure):
    _fields_ = [("data", _p), ("n", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("c", ctypes.c_int32), ("stride", ctypes.c_int32), ("offset", ctypes.c_int32)]


_PA = ctypes.POINTER(gs_act)
_lib.gs_nn_conv3x3.argtypes = [_PA, _PA, _PA, _p, ctypes.c_int32, _p, ctypes.c_int32, _PA, _p,
                               ctypes.c_int32, _S]
_lib.gs_nn_conv3x3_wgrad.argtypes = [_PA, _PA, _PA, _PA, _p, _p, _S]
_lib.gs_nn_flip_weights.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, _p, _S]
_lib.gs_nn_avgpool2.argtypes = [_PA, _PA, _S]
_lib.gs_nn_avgpool2_bwd.argtypes = [_PA, _PA, _PA, ctypes.c_int32, _S]
_lib.gs_nn_upsample2.argtypes = [_PA, _PA, _S]
_lib.gs_nn_upsample2_bwd.argtypes = [_PA, _PA, _S]
_lib.gs_nn_rgb_to_nhwc.argtypes = [_p, _PA, _S]
_lib.gs_nn_f32_to_bf16.argtypes = [_p, _p, ctypes.c_int64, _S]
_lib.gs_nn_head.argtypes = [_PA, _p, _p, _p, _S]
_lib.gs_nn_head_bwd.argtypes = [_PA, _p, _p, _PA, _p, _p, _S]
_lib.gs_nn_depth_loss.argtypes = [_p, _p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_float, _p, _p, _p, _S]
_lib.gs_cost_volume_workspace_size.restype = ctypes.c_size_t
_lib.gs_cost_volume_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
_lib.gs_cost_volume_wta.argtypes = [_p, ctypes.POINTER(gs_views), _p, _p, _p, ctypes.c_size_t, _S]
_lib.gs_bp_workspace_size.restype = ctypes.c_size_t
_lib.gs_bp_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.gs_bp_labels.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                              ctypes.c_int32, ctypes.c_float, _p, _p, _p, ctypes.c_size_t, _S]
EXPORTED = EXPORTED + ("gs_bp_workspace_size", "gs_bp_labels")
EXPORTED = EXPORTED + ("gs_nn_conv3x3", "gs_nn_conv3x3_wgrad", "gs_nn_flip_weights", "gs_nn_avgpool2",
                       "gs_nn_avgpool2_bwd", "gs_nn_upsample2", "gs_nn_upsample2_bwd",
                       "gs_nn_rgb_to_nhwc", "gs_nn_f32_to_bf16", "gs_nn_head", "gs_nn_head_bwd",
                       "gs_nn_depth_loss", "gs_cost_volume_workspace_size", "gs_cost_volume_wta")


class Act:
    """BF16 NHWC activation view over a torch.bfloat16 tensor [n, h, w, stride]."""

    def __init__(self, t: torch.Tensor, c: Optional[int] = None, offset: int = 0):
        if t.dtype != torch.bfloat16 or t.dim() != 4 or not t.is_contiguous():
            raise ValueError("activations are contiguous bfloat16 [n, h, w, stride]")
        self.t = t
        self.n, self.h, self.w, self.stride = (int(s) for s in t.shape)
        self.c = self.stride - offset if c is None else int(c)
        self.offset = int(offset)
        self.struct = gs_act(t.data_ptr(), self.n, self.h, self.w, self.c, self.stride, self.offset)

    @classmethod
    def empty(cls, n, h, w, c, device="cuda", zero=False):
        f = torch.zeros if zero else torch.empty
        return cls(f(n, h, w, c, dtype=torch.bfloat16, device=device))

    def slice(self, offset: int, c: int) -> "Act":
        return Act(self.t, c, self.offset + offset)

    def values(self) -> torch.Tensor:
        """The view's channels as float32 [n, h, w, c] (a copy)."""
        return self.t[..., self.offset:self.offset + self.c].float()


def _ap(a: Optional[Act]):
    return None if a is None else ctypes.byref(a.struct)


def gs_nn_conv3x3(x1: Act, x2: Optional[Act], mask: Optional[Act], weights: torch.Tensor, cout: int,
                  bias: Optional[torch.Tensor], relu: bool, y: Optional[Act],
                  y_f32: Optional[torch.Tensor] = None, y_f32_stride: int = 0, stream=None) -> None:
    _check(_lib.gs_nn_conv3x3(_ap(x1), _ap(x2), _ap(mask), _ptr(weights), cout, _ptr(bias), int(relu),
                              _ap(y), _ptr(y_f32), y_f32_stride, _stream(stream)), "gs_nn_conv3x3")


def gs_nn_conv3x3_wgrad(x1: Act, x2: Optional[Act], dy: Act, mask: Optional[Act], dw: torch.Tensor,
                        dbias: Optional[torch.Tensor], stream=None) -> None:
    _check(_lib.gs_nn_conv3x3_wgrad(_ap(x1), _ap(x2), _ap(dy), _ap(mask), _ptr(dw), _ptr(dbias),
                                    _stream(stream)), "gs_nn_conv3x3_wgrad")


def gs_nn_flip_weights(w: torch.Tensor, cout: int, cin: int, wt: torch.Tensor, stream=None) -> None:
    _check(_lib.gs_nn_flip_weights(_ptr(w), cout, cin, _ptr(wt), _stream(stream)), "gs_nn_flip_weights")


def gs_nn_avgpool2(x: Act, y: Act, stream=None) -> None:
    _check(_lib.gs_nn_avgpool2(_ap(x), _ap(y), _stream(stream)), "gs_nn_avgpool2")


def gs_nn_avgpool2_bwd(dy: Act, add: Optional[Act], dx: Act, accumulate: bool = False, stream=None) -> None:
    _check(_lib.gs_nn_avgpool2_bwd(_ap(dy), _ap(add), _ap(dx), int(accumulate), _stream(stream)),
           "gs_nn_avgpool2_bwd")


def gs_nn_upsample2(x: Act, y: Act, stream=None) -> None:
    _check(_lib.gs_nn_upsample2(_ap(x), _ap(y), _stream(stream)), "gs_nn_upsample2")


def gs_nn_upsample2_bwd(dy: Act, dx: Act, stream=None) -> None:
    _check(_lib.gs_nn_upsample2_bwd(_ap(dy), _ap(dx), _stream(stream)), "gs_nn_upsample2_bwd")


def gs_nn_rgb_to_nhwc(rgb: torch.Tensor, x: Act, stream=None) -> None:
    _check(_lib.gs_nn_rgb_to_nhwc(_ptr(rgb), _ap(x), _stream(stream)), "gs_nn_rgb_to_nhwc")


def gs_nn_f32_to_bf16(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    if src.numel() != dst.numel():
        raise ValueError("size mismatch")
    _check(_lib.gs_nn_f32_to_bf16(_ptr(src), _ptr(dst), src.numel(), _stream(stream)), "gs_nn_f32_to_bf16")


def gs_nn_head(f: Act, w: torch.Tensor, b: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    _check(_lib.gs_nn_head(_ap(f), _ptr(w), _ptr(b), _ptr(out), _stream(stream)), "gs_nn_head")


def gs_nn_head_bwd(f: Act, w: torch.Tensor, dout: torch.Tensor, df: Act, dw: torch.Tensor,
                   db: torch.Tensor, stream=None) -> None:
    _check(_lib.gs_nn_head_bwd(_ap(f), _ptr(w), _ptr(dout), _ap(df), _ptr(dw), _ptr(db),
                               _stream(stream)), "gs_nn_head_bwd")


def gs_nn_depth_loss(pred: torch.Tensor, depth: torch.Tensor, fx: float, dpred: torch.Tensor,
                     loss: Optional[torch.Tensor], ws: torch.Tensor, stream=None) -> None:
    n, _, h, w = pred.shape
    _check(_lib.gs_nn_depth_loss(_ptr(pred), _ptr(depth), n, h, w, fx, _ptr(dpred), _ptr(loss),
                                 _ptr(ws), _stream(stream)), "gs_nn_depth_loss")


def gs_cost_volume_wta(keyframes: torch.Tensor, views: Views, cost: Optional[torch.Tensor],
                       depth: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    _check(_lib.gs_cost_volume_wta(_ptr(keyframes), ctypes.byref(views.struct), _ptr(cost), _ptr(depth),
                                   _ptr(ws), ws.numel(), _stream(stream)), "gs_cost_volume_wta")


def gs_cost_volume_workspace_size(k: int, h: int, w: int) -> int:
    return int(_lib.gs_cost_volume_workspace_size(k, h, w))


def gs_bp_workspace_size(h: int, w: int) -> int:
    return int(_lib.gs_bp_workspace_size(h, w))


def gs_bp_labels(cost: torch.Tensor, h: int, w: int, lam: float, trunc: float, iters: int,
                 invalid: float, labels: Optional[torch.Tensor], depth: Optional[torch.Tensor],
                 ws: torch.Tensor, stream=None) -> None:
    if cost.dtype != torch.float32 or cost.numel() != 64 * h * w:
        raise ValueError("cost must be float32 [64][h][w]")
    _check(_lib.gs_bp_labels(_ptr(cost), h, w, lam, trunc, iters, invalid, _ptr(labels), _ptr(depth),
                             _ptr(ws), ws.numel(), _stream(stream)), "gs_bp_labels")
