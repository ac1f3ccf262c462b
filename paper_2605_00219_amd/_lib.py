"""ctypes binding of libgs.so (the C ABI in include/gs.h).

Argument marshalling only: every stage of the pipeline runs in the library's
HIP kernels.  Tensors must be CUDA (HIP) tensors; pointers and the current
stream are taken from them.  If the library has not been built this module
raises on import -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

MAX_VIEWS = 16
PARAM_PLANES = 15
MLP_PARAMS = 1377
MLP_GROUPS = 64
MLP_SCRATCH = (MLP_GROUPS + 1) * (MLP_PARAMS + 1)

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_HIP, GS_ERR_WORKSPACE, GS_ERR_CAPACITY = 0, -1, -2, -3, -4
STATUS_CAPACITY, STATUS_OVERFLOW, STATUS_ROWS, STATUS_SORT = 1, 2, 4, 8
CULL_RECT, CULL_ELLIPSE = 0, 1


class GsLayout(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("tile", C.c_int32), ("pixels_per_lane", C.c_int32),
                ("cull", C.c_int32), ("width", C.c_int32 * MAX_VIEWS), ("height", C.c_int32 * MAX_VIEWS),
                ("tiles_x", C.c_int32 * MAX_VIEWS), ("tiles_y", C.c_int32 * MAX_VIEWS),
                ("depth_bits", C.c_int32 * MAX_VIEWS),
                ("tile_base", C.c_int32 * (MAX_VIEWS + 1)),
                ("pixel_base", C.c_int64 * (MAX_VIEWS + 1))]

    @property
    def total_tiles(self) -> int:
        return int(self.tile_base[self.n_views])

    @property
    def total_pixels(self) -> int:
        return int(self.pixel_base[self.n_views])


class GsSplats(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("tiles", C.c_void_p)]


class GsBins(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("row_offsets", C.c_void_p), ("rows", C.c_void_p),
                ("row_capacity", C.c_int64), ("keys", C.c_void_p), ("vals", C.c_void_p),
                ("ranges", C.c_void_p), ("status", C.c_void_p), ("capacity", C.c_int64)]


class GsSideStream(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("fork", C.c_void_p), ("join", C.c_void_p)]


class GsGrads2d(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("rec_mask", C.c_void_p), ("tile_stop", C.c_void_p),
                ("sums", C.c_void_p), ("workspace", C.c_void_p)]


class GsImage(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("T", C.c_void_p), ("last", C.c_void_p),
                ("tile_stats", C.c_void_p), ("comp_mask", C.c_void_p)]


class GsSchedule(C.Structure):
    _fields_ = [("order", C.c_void_p), ("counter", C.c_void_p), ("n_groups", C.c_int32)]


class GsAdam(C.Structure):
    _fields_ = [("m", C.c_void_p), ("v", C.c_void_p), ("step", C.c_void_p), ("scratch", C.c_void_p),
                ("lr", C.c_float * 6), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


TS_MAX_ARMS = 8


class GsTsState(C.Structure):
    _fields_ = [("n_arms", C.c_int32), ("reserved", C.c_int32), ("rng", C.c_uint64),
                ("mu0", C.c_double), ("kappa0", C.c_double), ("alpha0", C.c_double), ("beta0", C.c_double),
                ("n", C.c_double * TS_MAX_ARMS), ("mean", C.c_double * TS_MAX_ARMS),
                ("m2", C.c_double * TS_MAX_ARMS)]


_P = C.c_void_p
_SIGS = {
    "gs_version": (C.c_int, []),
    "gs_last_error": (C.c_char_p, []),
    "gs_layout_init": (C.c_int, [_P, _P, C.c_int, C.c_int, C.POINTER(GsLayout)]),
    "gs_bin_sort_workspace_size": (C.c_size_t, [C.c_int64, C.POINTER(GsLayout), C.c_int64]),
    "gs_grads2d_workspace_size": (C.c_size_t, [C.c_int64]),
    "gs_project": (C.c_int, [_P, C.c_int64, _P, C.POINTER(GsLayout), C.POINTER(GsSplats), _P]),
    "gs_bin_sort": (C.c_int, [C.POINTER(GsSplats), C.c_int64, C.POINTER(GsLayout), C.POINTER(GsBins),
                              _P, C.c_size_t, C.POINTER(GsSideStream), _P]),
    "gs_rasterize_fwd": (C.c_int, [C.POINTER(GsSplats), C.c_int64, C.POINTER(GsLayout),
                                   C.POINTER(GsBins), _P, C.POINTER(GsImage), C.c_int,
                                   C.POINTER(GsSchedule), _P]),
    "gs_rasterize_bwd": (C.c_int, [C.POINTER(GsSplats), C.c_int64, C.POINTER(GsLayout),
                                   C.POINTER(GsBins), _P, C.POINTER(GsImage), _P, _P,
                                   C.POINTER(GsGrads2d), _P, C.c_int, C.POINTER(GsSchedule), _P]),
    "gs_rasterize_bwd_twophase": (C.c_int, [C.POINTER(GsSplats), C.c_int64, C.POINTER(GsLayout),
                                            C.POINTER(GsBins), _P, C.POINTER(GsImage), _P, _P,
                                            C.POINTER(GsGrads2d), _P, C.c_int, C.POINTER(GsSchedule), _P]),
    "gs_project_bwd_adam": (C.c_int, [_P, C.c_int64, _P, C.POINTER(GsLayout), C.POINTER(GsSplats),
                                      C.POINTER(GsBins), C.POINTER(GsGrads2d), C.POINTER(GsAdam),
                                      _P, _P]),
    "gs_project_bwd_adam_noalloc": (C.c_int, [_P, C.c_int64, _P, C.POINTER(GsLayout), C.POINTER(GsSplats),
                                              C.POINTER(GsBins), C.POINTER(GsGrads2d), C.POINTER(GsAdam),
                                              _P, _P]),
    "gs_tile_features": (C.c_int, [C.POINTER(GsSplats), C.c_int64, C.POINTER(GsLayout),
                                   C.POINTER(GsBins), _P, _P]),
    "gs_mlp_forward": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P]),
    "gs_mlp_train_step": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, _P, _P, _P, C.c_float, _P, _P]),
    "gs_order_by_cost_scratch_size": (C.c_size_t, [C.c_int32]),
    "gs_order_by_cost": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "gs_loss_blocks": (C.c_int64, [C.POINTER(GsLayout)]),
    "gs_loss_workspace_size": (C.c_size_t, [C.POINTER(GsLayout)]),
    "gs_loss_l1_ssim": (C.c_int, [_P, _P, C.POINTER(GsLayout), C.c_float, C.c_int, _P, _P, _P, C.c_size_t,
                                  _P]),
    "gs_ts_init": (C.c_int, [C.POINTER(GsTsState), C.c_int, C.c_uint64, C.c_double, C.c_double, C.c_double,
                             C.c_double]),
    "gs_ts_select": (C.c_int, [C.POINTER(GsTsState)]),
    "gs_ts_update": (C.c_int, [C.POINTER(GsTsState), C.c_int, C.c_double]),
    "gs_ts_posterior": (C.c_int, [C.POINTER(GsTsState), C.c_int, C.POINTER(C.c_double)]),
    "gs_ts_sample": (C.c_double, [C.POINTER(GsTsState), C.c_int]),
}
EXPORTS = tuple(_SIGS)


class GsError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2605_00219_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(rc: int, what: str) -> None:
    if rc != GS_OK:
        msg = lib.gs_last_error().decode(errors="replace")
        raise GsError(f"{what} failed ({rc}): {msg}")


def ptr(t) -> int | None:
    """Device pointer of a tensor (None for None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libgs needs device tensors")
    if not t.is_contiguous():
        raise ValueError("libgs needs contiguous tensors")
    return t.data_ptr()


def stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def layout_init(widths, heights, tile: int, pixels_per_lane: int | None = None,
                cull: int = CULL_RECT) -> GsLayout:
    n = len(widths)
    W = (C.c_int32 * n)(*[int(w) for w in widths])
    H = (C.c_int32 * n)(*[int(h) for h in heights])
    L = GsLayout()
    check(lib.gs_layout_init(W, H, n, int(tile), C.byref(L)), "gs_layout_init")
    if pixels_per_lane is not None:
        L.pixels_per_lane = int(pixels_per_lane)
    L.cull = int(cull)
    return L
