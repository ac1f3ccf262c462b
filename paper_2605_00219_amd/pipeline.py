"""Buffers and the training step on top of the C ABI.

PyTorch supplies device memory and the stream; all arithmetic of the path is in
libgs.  Names follow the five stages of the C ABI:
project -> bin_sort -> rasterize_fwd -> rasterize_bwd -> project_bwd_adam.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as G

PLANES = G.PARAM_PLANES

# canonical per-Gaussian order: mean(3), log-scale(3), quaternion(4), opacity logit(1), SH(48)
# -> parameter-block (plane, component); the unused slot is plane 1 component 3
_PLANE_INDEX = np.zeros(59, np.int64)
for _k in range(59):
    if _k < 3:
        _PLANE_INDEX[_k] = 0 * 4 + _k
    elif _k < 6:
        _PLANE_INDEX[_k] = 1 * 4 + (_k - 3)
    elif _k < 10:
        _PLANE_INDEX[_k] = 2 * 4 + (_k - 6)
    elif _k == 10:
        _PLANE_INDEX[_k] = 0 * 4 + 3
    else:
        _PLANE_INDEX[_k] = 12 + (_k - 11)


def pack_flat(flat, device="cuda") -> torch.Tensor:
    """[N,59] canonical parameters -> parameter block [15, N, 4] float32."""
    flat = torch.as_tensor(np.ascontiguousarray(flat, np.float32) if isinstance(flat, np.ndarray) else flat,
                           dtype=torch.float32)
    n = flat.shape[0]
    blk = torch.zeros(n, PLANES * 4, dtype=torch.float32, device=flat.device)
    blk[:, torch.as_tensor(_PLANE_INDEX, device=flat.device)] = flat
    return blk.view(n, PLANES, 4).permute(1, 0, 2).contiguous().to(device)


def unpack_flat(block: torch.Tensor) -> torch.Tensor:
    """parameter block [15, N, 4] -> [N, 59] canonical order."""
    n = block.shape[1]
    rows = block.permute(1, 0, 2).reshape(n, PLANES * 4)
    return rows[:, torch.as_tensor(_PLANE_INDEX, device=block.device)]


def views_to_device(views: np.ndarray, device="cuda") -> torch.Tensor:
    """VIEW_DTYPE records -> device bytes (128 per view)."""
    raw = np.ascontiguousarray(views).view(np.uint8).reshape(-1)
    return torch.from_numpy(raw.copy()).to(device)


def _i(t) -> int:
    return t.data_ptr()


class Frame:
    """Per-view-set buffers: projected splats, intersection lists, images."""

    def __init__(self, n: int, widths, heights, tile: int = 16, capacity: int = 1 << 16,
                 device="cuda", tile_stats: bool = False, pixels_per_lane: int | None = None,
                 cull: int = G.CULL_RECT, row_capacity: int | None = None, side_stream: bool = True):
        self.n = int(n)
        self.device = device
        self.cull = int(cull)
        self.layout = G.layout_init(widths, heights, tile, pixels_per_lane, cull)
        self.n_views = len(widths)
        self.tile = tile
        V, n = self.n_views, self.n
        f32 = dict(dtype=torch.float32, device=device)
        u32 = dict(dtype=torch.int32, device=device)   # torch has no uint32 arithmetic; bits only
        self.rec = torch.zeros(V * n, 16, **f32)    # 64-byte projected records
        self.tiles = torch.zeros(V * n, **u32)
        self.offsets = torch.zeros(V * n + 1, **u32)
        self.row_offsets = torch.zeros(V * n + 1, **u32)
        self.ranges = torch.zeros(self.layout.total_tiles, 2, **u32)
        self.status = torch.zeros(1, **u32)
        P = self.layout.total_pixels
        self.image = torch.zeros(P, 3, **f32)
        self.T = torch.zeros(P, **f32)
        self.last = torch.zeros(P, **u32)
        self.tile_stats = torch.zeros(self.layout.total_tiles, 4, **u32) if tile_stats else None
        self.loss_tiles = torch.zeros(self.layout.total_tiles, **f32)
        self.tile_stop = torch.zeros(self.layout.total_tiles, **u32)
        self.sums = torch.zeros(9, V * n, **f32)      # per (view, Gaussian) screen-space gradient
        self.counter = torch.zeros(1, **u32)
        self.capacity = 0
        self.row_capacity = 0
        self.resize(capacity, row_capacity)
        # the binning's side stream (default priority) and its fork/join events,
        # owned here; the events are recorded once so that they exist
        self._side = None
        if side_stream:
            st = torch.cuda.Stream(device=device)
            fork, join = torch.cuda.Event(), torch.cuda.Event()
            fork.record(st)
            join.record(st)
            self._side_objs = (st, fork, join)
            self._side = G.GsSideStream(st.cuda_stream, fork.cuda_event, join.cuda_event)

    def side_stream(self):
        """The GsSideStream gs_bin_sort may run its depth sort on (None: one stream)."""
        return self._side

    # -- buffers sized by the intersection capacity (and the tile-row capacity) --
    def resize(self, capacity: int, row_capacity: int | None = None) -> None:
        capacity = max(int(capacity), 1)
        if row_capacity is None:        # keep the row capacity; rows never outnumber tiles
            row_capacity = self.row_capacity or capacity   # for the 3-sigma rectangle
        row_capacity = max(int(row_capacity), 1)
        u32 = dict(dtype=torch.int32, device=self.device)
        self.rows = torch.zeros(row_capacity, 4, **u32)
        self.row_capacity = row_capacity
        self.keys = torch.zeros(capacity, **u32)
        self.vals = torch.zeros(capacity, **u32)
        self.grec = torch.zeros(capacity, 12, dtype=torch.float32, device=self.device)
        self.rec_mask = torch.zeros((capacity + 31) // 32, **u32)
        self.comp_mask = torch.zeros((capacity + 31) // 32, **u32)
        ws = G.lib.gs_bin_sort_workspace_size(self.n, C.byref(self.layout), capacity)
        self.workspace = torch.zeros(max(int(ws), 1), dtype=torch.uint8, device=self.device)
        self.capacity = capacity
        self._structs()

    def _structs(self) -> None:
        self.splats = G.GsSplats(_i(self.rec), _i(self.tiles))
        self.bins = G.GsBins(_i(self.offsets), _i(self.row_offsets), _i(self.rows), self.row_capacity,
                             _i(self.keys), _i(self.vals), _i(self.ranges), _i(self.status),
                             self.capacity)
        self.grads2d = G.GsGrads2d(_i(self.grec), _i(self.rec_mask), _i(self.tile_stop), _i(self.sums), None)
        self.img = G.GsImage(_i(self.image), _i(self.T), _i(self.last),
                             _i(self.tile_stats) if self.tile_stats is not None else None,
                             _i(self.comp_mask))

    def intersections(self) -> int:
        """K (synchronises)."""
        return int(self.offsets[-1].item()) & 0xFFFFFFFF

    def status_bits(self) -> int:
        return int(self.status.item())

    def schedule(self, order: torch.Tensor | None = None, n_groups: int | None = None) -> G.GsSchedule:
        """Persistent work-queue schedule (order: global tile ids, int32 tensor)."""
        if n_groups is None:
            n_groups = 256 * 8
        return G.GsSchedule(_i(order) if order is not None else None, _i(self.counter), int(n_groups))


class Model:
    """Gaussian parameters (parameter block) and Adam state."""

    def __init__(self, flat, device="cuda", lr=1e-3, betas=(0.9, 0.999), eps=1e-15):
        self.params = pack_flat(flat, device)
        self.n = self.params.shape[1]
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = torch.zeros(1, dtype=torch.int32, device=device)
        self.scratch = torch.zeros(4, dtype=torch.float32, device=device)
        lrs = [float(lr)] * 6 if np.isscalar(lr) else [float(x) for x in lr]
        self.adam = G.GsAdam(_i(self.m), _i(self.v), _i(self.step), _i(self.scratch),
                             (C.c_float * 6)(*lrs), betas[0], betas[1], eps)

    def flat(self) -> torch.Tensor:
        return unpack_flat(self.params)


# ---------------------------------------------------------------------------
# the five stages
# ---------------------------------------------------------------------------

def project(params: torch.Tensor, frame: Frame, views_dev: torch.Tensor, stream=None) -> None:
    G.check(G.lib.gs_project(_i(params), frame.n, _i(views_dev), C.byref(frame.layout),
                             C.byref(frame.splats), G.stream_ptr(stream)), "gs_project")


def bin_sort(frame: Frame, stream=None) -> None:
    side = frame.side_stream()
    G.check(G.lib.gs_bin_sort(C.byref(frame.splats), frame.n, C.byref(frame.layout),
                              C.byref(frame.bins), _i(frame.workspace), frame.workspace.numel(),
                              C.byref(side) if side is not None else None,
                              G.stream_ptr(stream)), "gs_bin_sort")


def rasterize_fwd(frame: Frame, views_dev: torch.Tensor, lds_batch: int = 64, sched=None,
                  stream=None) -> None:
    G.check(G.lib.gs_rasterize_fwd(C.byref(frame.splats), frame.n, C.byref(frame.layout),
                                   C.byref(frame.bins), _i(views_dev), C.byref(frame.img), lds_batch,
                                   C.byref(sched) if sched is not None else None,
                                   G.stream_ptr(stream)), "gs_rasterize_fwd")


def rasterize_bwd(frame: Frame, views_dev: torch.Tensor, target: torch.Tensor | None = None,
                  dLdC: torch.Tensor | None = None, lds_batch: int = 64, sched=None,
                  stream=None) -> None:
    G.check(G.lib.gs_rasterize_bwd(C.byref(frame.splats), frame.n, C.byref(frame.layout),
                                   C.byref(frame.bins), _i(views_dev), C.byref(frame.img),
                                   _i(target) if target is not None else None,
                                   _i(dLdC) if dLdC is not None else None, C.byref(frame.grads2d),
                                   _i(frame.loss_tiles) if target is not None else None, lds_batch,
                                   C.byref(sched) if sched is not None else None,
                                   G.stream_ptr(stream)), "gs_rasterize_bwd")


def rasterize_bwd_twophase(frame: Frame, views_dev: torch.Tensor, target: torch.Tensor | None = None,
                           dLdC: torch.Tensor | None = None, lds_batch: int = 32, sched=None,
                           stream=None) -> None:
    """The two-phase backward (gs_rasterize_bwd_twophase): same outputs as rasterize_bwd."""
    G.check(G.lib.gs_rasterize_bwd_twophase(C.byref(frame.splats), frame.n, C.byref(frame.layout),
                                            C.byref(frame.bins), _i(views_dev), C.byref(frame.img),
                                            _i(target) if target is not None else None,
                                            _i(dLdC) if dLdC is not None else None, C.byref(frame.grads2d),
                                            _i(frame.loss_tiles) if target is not None else None, lds_batch,
                                            C.byref(sched) if sched is not None else None,
                                            G.stream_ptr(stream)), "gs_rasterize_bwd_twophase")


def backward(frame: Frame, views_dev: torch.Tensor, variant, target=None, dLdC=None, sched=None,
             stream=None) -> None:
    """Run one backward variant: an int is rasterize_bwd's lds_batch, ("twophase", S)
    the two-phase backward with batch S."""
    if isinstance(variant, tuple) and variant[0] == "twophase":
        rasterize_bwd_twophase(frame, views_dev, target=target, dLdC=dLdC, lds_batch=variant[1], sched=sched,
                               stream=stream)
    else:
        rasterize_bwd(frame, views_dev, target=target, dLdC=dLdC, lds_batch=int(variant), sched=sched,
                      stream=stream)


class LossL1SSIM:
    """Fused L1 + D-SSIM loss gradient of a frame's render against an RGBA8
    reference (gs_loss_l1_ssim); owns its workspace and per-block sums."""

    def __init__(self, frame: Frame, lam: float = 0.2, use_mask: bool = True):
        dev = frame.image.device
        self.frame = frame
        self.lam = float(lam)
        self.use_mask = bool(use_mask)
        nb = int(G.lib.gs_loss_blocks(C.byref(frame.layout)))
        ws = int(G.lib.gs_loss_workspace_size(C.byref(frame.layout)))
        self.blocks = torch.zeros(2 * max(nb, 1), dtype=torch.float32, device=dev)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.dLdC = torch.zeros_like(frame.image)

    def __call__(self, target_rgba: torch.Tensor, stream=None) -> torch.Tensor:
        """target_rgba: uint8 [pixels, 4] on the device; returns dL/dC [pixels, 3]."""
        assert target_rgba.dtype == torch.uint8 and target_rgba.is_contiguous()
        G.check(G.lib.gs_loss_l1_ssim(_i(self.frame.image), _i(target_rgba), C.byref(self.frame.layout),
                                      self.lam, int(self.use_mask), _i(self.dLdC), _i(self.blocks),
                                      _i(self.workspace), self.workspace.numel(), G.stream_ptr(stream)),
                "gs_loss_l1_ssim")
        return self.dLdC

    def loss(self) -> float:
        """The loss of the last call (synchronises)."""
        b = self.blocks.double().view(-1, 2).sum(0)
        P = self.frame.layout.total_pixels
        return float(((1 - self.lam) * b[0] + self.lam * b[1]).item()) / (3.0 * P)


class ThompsonScheduler:
    """Latency beliefs over a set of arms (gs_ts_*); host state, no GPU."""

    def __init__(self, n_arms: int, seed: int = 0, mu0: float = 0.0, kappa0: float = 1e-3,
                 alpha0: float = 1.0, beta0: float = 1e-4):
        self.state = G.GsTsState()
        G.check(G.lib.gs_ts_init(C.byref(self.state), int(n_arms), int(seed), float(mu0), float(kappa0),
                                 float(alpha0), float(beta0)), "gs_ts_init")

    def select(self) -> int:
        a = G.lib.gs_ts_select(C.byref(self.state))
        G.check(0 if a >= 0 else a, "gs_ts_select")
        return a

    def update(self, arm: int, latency: float) -> None:
        G.check(G.lib.gs_ts_update(C.byref(self.state), int(arm), float(latency)), "gs_ts_update")

    def posterior(self, arm: int):
        out = (C.c_double * 4)()
        G.check(G.lib.gs_ts_posterior(C.byref(self.state), int(arm), out), "gs_ts_posterior")
        return tuple(out)

    def sample(self, arm: int) -> float:
        return float(G.lib.gs_ts_sample(C.byref(self.state), int(arm)))

    def counts(self):
        return [int(self.state.n[a]) for a in range(self.state.n_arms)]


class ScheduledBackward:
    """The backward whose variant -- rasterize_bwd's LDS batch (fixed, or per tile
    when negative) or ("twophase", S) -- is chosen per call by Thompson sampling
    on measured latency (Sec. 4.2).  Every time_every-th call (default: every
    call) is bracketed by two timing events on the launch stream; finished
    calls are folded into the belief at later calls without synchronising.
    Timing fewer calls slows the learning: with the two-phase arms (twice
    the first backward's time) and time_every = 4, 100 steps picked a
    two-phase arm 20 times and ran at 0.91x the fixed batch, against 0.96x
    when every call is timed."""

    def __init__(self, arms=(64, 128, 256, -128), seed: int = 0, prior_ms: float = 0.3, time_every: int = 1):
        import collections
        self.arms = tuple(arms)
        self.time_every = max(1, int(time_every))
        self.calls = 0
        # weak prior centred on prior_ms, standard deviation about 10 % of it
        self.ts = ThompsonScheduler(len(self.arms), seed, mu0=prior_ms, kappa0=1e-3, alpha0=1.0,
                                    beta0=(0.1 * prior_ms) ** 2)
        self.pending = collections.deque()
        self.history = []

    def harvest(self, block: bool = False) -> None:
        while self.pending:
            arm, e0, e1 = self.pending[0]
            if not block and not e1.query():
                break
            e1.synchronize()
            self.pending.popleft()
            self.ts.update(arm, e0.elapsed_time(e1))

    def __call__(self, frame: Frame, views_dev: torch.Tensor, target=None, dLdC=None, sched=None,
                 stream=None) -> int:
        self.harvest()
        arm = self.ts.select()
        s = stream if stream is not None else torch.cuda.current_stream()
        timed = self.calls % self.time_every == 0
        self.calls += 1
        if timed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
        backward(frame, views_dev, self.arms[arm], target=target, dLdC=dLdC, sched=sched, stream=s)
        if timed:
            e1.record(s)
            self.pending.append((arm, e0, e1))
        self.history.append(arm)
        return arm


def project_bwd_adam(model: Model, frame: Frame, views_dev: torch.Tensor, adam: bool = True,
                     grads_out: torch.Tensor | None = None, stream=None) -> None:
    G.check(G.lib.gs_project_bwd_adam(_i(model.params), frame.n, _i(views_dev), C.byref(frame.layout),
                                      C.byref(frame.splats), C.byref(frame.bins),
                                      C.byref(frame.grads2d),
                                      C.byref(model.adam) if adam else None,
                                      _i(grads_out) if grads_out is not None else None,
                                      G.stream_ptr(stream)), "gs_project_bwd_adam")


def project_bwd_adam_noalloc(model: Model, frame: Frame, views_dev: torch.Tensor, adam: bool = True,
                             grads_out: torch.Tensor | None = None, stream=None) -> None:
    """project_bwd_adam through gs_project_bwd_adam_noalloc (allocates nothing;
    the same launch as gs_project_bwd_adam, which needs no scratch either)."""
    G.check(G.lib.gs_project_bwd_adam_noalloc(_i(model.params), frame.n, _i(views_dev), C.byref(frame.layout),
                                              C.byref(frame.splats), C.byref(frame.bins),
                                              C.byref(frame.grads2d),
                                              C.byref(model.adam) if adam else None,
                                              _i(grads_out) if grads_out is not None else None,
                                              G.stream_ptr(stream)), "gs_project_bwd_adam_noalloc")


def tile_rows(frame: Frame) -> int:
    """R: tile-row slots the current projection needs (synchronises)."""
    bits = frame.rec[:, 12:14].view(torch.int32).to(torch.int64)
    h = ((bits[:, 1] >> 16) & 0xFFFF) - ((bits[:, 0] >> 16) & 0xFFFF)
    return int(torch.where(frame.tiles != 0, h, torch.zeros_like(h)).sum().item())


def fit_capacity(params: torch.Tensor, frame: Frame, views_dev: torch.Tensor, slack: float = 1.25):
    """Project once and size the intersection and tile-row buffers for the
    current K and R (synchronises).  Returns K."""
    project(params, frame, views_dev)
    K = int(frame.tiles.to(torch.int64).sum().item())
    R = tile_rows(frame)
    need_r = int(math.ceil(R * slack)) + 1024
    # grow either buffer as needed; also shrink the row slots when far larger
    # than needed (their launches are sized by the row capacity)
    if K > frame.capacity or R > frame.row_capacity or frame.row_capacity > 4 * need_r:
        cap = max(frame.capacity, int(math.ceil(K * slack)) + 1024) if K > frame.capacity \
            else frame.capacity
        rcap = max(frame.row_capacity, need_r) if R > frame.row_capacity else need_r
        frame.resize(cap, rcap)
    return K


def render(params: torch.Tensor, frame: Frame, views_dev: torch.Tensor, lds_batch: int = 64,
           sched=None, check: bool = True) -> torch.Tensor:
    """Forward only; returns the image [pixels, 3] (a view into frame.image)."""
    project(params, frame, views_dev)
    bin_sort(frame)
    if check and frame.status_bits():
        fit_capacity(params, frame, views_dev)
        bin_sort(frame)
    rasterize_fwd(frame, views_dev, lds_batch, sched)
    return frame.image


def train_step(model: Model, frame: Frame, views_dev: torch.Tensor, target: torch.Tensor | None,
               lds_batch: int = 64, sched=None, check: bool = True,
               grads_out: torch.Tensor | None = None, adam: bool = True,
               bwd_batch: int | None = None, dLdC: torch.Tensor | None = None) -> None:
    """One L1 training step over the frame's views: 5 stages, gradients summed over views.
    bwd_batch: the backward variant if not rasterize_bwd with lds_batch (see backward()).
    dLdC: an image gradient [pixels, 3] taken instead of the L1 gradient (target None)."""
    if (target is None) == (dLdC is None):
        raise ValueError("give exactly one of target and dLdC")
    project(model.params, frame, views_dev)
    bin_sort(frame)
    if check and frame.status_bits():
        fit_capacity(model.params, frame, views_dev)
        bin_sort(frame)
        if frame.status_bits():
            raise G.GsError(f"intersection status {frame.status_bits()} after resize")
    rasterize_fwd(frame, views_dev, lds_batch, sched)
    backward(frame, views_dev, bwd_batch or lds_batch, target=target, dLdC=dLdC, sched=sched)
    project_bwd_adam(model, frame, views_dev, adam=adam, grads_out=grads_out)


def loss_value(frame: Frame) -> float:
    """Mean |C - target| of the last train_step (synchronises)."""
    return float(frame.loss_tiles.double().sum().item()) / (3.0 * frame.layout.total_pixels)
