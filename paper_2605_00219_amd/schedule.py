"""Learned tile schedule for the persistent rasteriser.

The forward rasteriser logs, per tile, the number of list entries it
traversed (the cost driver of that tile).  A small fp32 MLP (8 -> 32 -> 32 ->
1, ReLU) maps 8 per-tile features (list length, mean/max opacity, mean/min
depth, mean radius, tile x, tile y) to log(1 + traversed entries).  It is
trained on the GPU by the library's own forward/backward/Adam kernels, and its
predictions order the persistent work queue longest-first.  The ordering
changes no output bit (every tile is rendered by the same code whatever order
the queue hands it out); invalid weights or non-finite predictions fall back
to the static ascending order inside gs_order_by_cost.
"""
from __future__ import annotations

import ctypes as C
import json
import math

import numpy as np
import torch

from . import _lib as G
from . import pipeline as P

N_FEATURES = 8


def _i(t):
    return t.data_ptr()


def tile_features(frame: P.Frame) -> torch.Tensor:
    """[total tiles, 8] features of the frame's current bins."""
    out = torch.empty(frame.layout.total_tiles, N_FEATURES, dtype=torch.float32, device="cuda")
    G.check(G.lib.gs_tile_features(C.byref(frame.splats), frame.n, C.byref(frame.layout),
                                   C.byref(frame.bins), _i(out), G.stream_ptr()), "gs_tile_features")
    return out


def traversal_target(frame: P.Frame) -> torch.Tensor:
    """log(1 + entries traversed) per tile, from the forward's tile statistics."""
    ts = frame.tile_stats[:, 0].to(torch.int64).to(torch.float32)
    return torch.log1p(ts)


class CostModel:
    """MLP weights, feature normalisation and Adam state, all on the device."""

    def __init__(self, seed: int = 0):
        rng = np.random.default_rng(seed)
        w = np.zeros(G.MLP_PARAMS, np.float32)
        # He-uniform init per layer
        o = 0
        for fan_in, fan_out in ((8, 32), (32, 32), (32, 1)):
            bound = math.sqrt(6.0 / fan_in)
            w[o:o + fan_in * fan_out] = rng.uniform(-bound, bound, fan_in * fan_out)
            o += fan_in * fan_out + fan_out
        self.w = torch.tensor(w, device="cuda")
        self.norm = torch.tensor(np.r_[np.zeros(8), np.ones(8), np.full(8, -3.0e38), np.full(8, 3.0e38)]
                                 .astype(np.float32), device="cuda")
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.step = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.scratch = torch.zeros(G.MLP_SCRATCH, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def set_normalisation(self, features: torch.Tensor) -> None:
        """Mean and standard deviation of the training features, and their
        range, to which features are clamped before the network."""
        mean = features.mean(0)
        std = features.std(0).clamp_min(1e-6)
        lo, hi = features.min(0).values, features.max(0).values
        self.norm = torch.cat([mean, std, lo, hi]).to(torch.float32).contiguous()

    def predict(self, features: torch.Tensor) -> torch.Tensor:
        x = features.contiguous()
        out = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        G.check(G.lib.gs_mlp_forward(_i(self.w), _i(self.norm), _i(x), x.shape[0], _i(out),
                                     G.stream_ptr()), "gs_mlp_forward")
        return out

    def train_step(self, features: torch.Tensor, targets: torch.Tensor, lr: float = 3e-3) -> None:
        x = features.contiguous()
        y = targets.contiguous().to(torch.float32)
        G.check(G.lib.gs_mlp_train_step(_i(self.w), _i(self.norm), _i(x), _i(y), x.shape[0],
                                        _i(self.scratch), _i(self.m), _i(self.v), _i(self.step),
                                        float(lr), _i(self.loss), G.stream_ptr()), "gs_mlp_train_step")

    def fit(self, features: torch.Tensor, targets: torch.Tensor, epochs: int = 500,
            lr: float = 3e-3) -> float:
        for _ in range(epochs):
            self.train_step(features, targets, lr)
        torch.cuda.synchronize()
        return float(self.loss.item())

    def state(self) -> dict:
        return {"w": self.w.cpu().tolist(), "norm": self.norm.cpu().tolist()}

    def load_state(self, st: dict) -> None:
        self.w = torch.tensor(st["w"], dtype=torch.float32, device="cuda")
        self.norm = torch.tensor(st["norm"], dtype=torch.float32, device="cuda")


def order_by_cost(pred: torch.Tensor) -> torch.Tensor:
    """Permutation of tiles by descending predicted cost (int32 tensor)."""
    n = pred.shape[0]
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    nbytes = int(G.lib.gs_order_by_cost_scratch_size(n))
    scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
    G.check(G.lib.gs_order_by_cost(_i(pred.contiguous()), n, _i(order), _i(scratch), G.stream_ptr()),
            "gs_order_by_cost")
    return order


def prediction_quality(pred: torch.Tensor, measured: torch.Tensor) -> dict:
    """MAPE on counts and Spearman rank correlation between predicted and
    measured traversal counts."""
    p = torch.expm1(pred.double()).clamp_min(0).cpu().numpy()
    m = torch.expm1(measured.double()).cpu().numpy()
    keep = m > 0
    mape = float(np.mean(np.abs(p[keep] - m[keep]) / m[keep])) if keep.any() else float("nan")
    rp = np.argsort(np.argsort(p)).astype(np.float64)
    rm = np.argsort(np.argsort(m)).astype(np.float64)
    rp -= rp.mean()
    rm -= rm.mean()
    rho = float((rp * rm).sum() / math.sqrt((rp ** 2).sum() * (rm ** 2).sum()))
    return {"mape": mape, "spearman": rho}


def save(model: CostModel, path: str) -> None:
    with open(path, "w") as f:
        json.dump(model.state(), f)


def load(path: str) -> CostModel:
    m = CostModel()
    with open(path) as f:
        m.load_state(json.load(f))
    return m
