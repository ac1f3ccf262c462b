"""Helpers for the GPU tests: run the HIP path through the C ABI and fetch
results as numpy arrays.  Nothing here computes any part of the method."""
import sys

import numpy as np


def note(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def run_gpu_step(scene, views, tile, target=None, lds_batch=64, lr=1e-3, adam=True, grads=True,
                 capacity=None, sched_order=None, persistent=False, tile_stats=False, steps=1):
    import torch
    from paper_2605_00219_amd import pipeline as P
    n = scene.n
    model = P.Model(scene.flat(), lr=lr)
    frame = P.Frame(n, [int(v["width"]) for v in views], [int(v["height"]) for v in views], tile,
                    capacity=capacity or 1024, tile_stats=tile_stats)
    vd = P.views_to_device(views)
    if capacity is None:
        P.fit_capacity(model.params, frame, vd)
    sched = None
    if persistent or sched_order is not None:
        order = None if sched_order is None else torch.as_tensor(sched_order, dtype=torch.int32,
                                                                 device="cuda")
        sched = frame.schedule(order)
        sched_keep = order  # noqa: F841 (keeps the tensor alive)
    tgt = None if target is None else torch.as_tensor(np.ascontiguousarray(target, np.float32),
                                                      device="cuda").reshape(-1, 3)
    gout = torch.zeros_like(model.params) if grads else None
    for _ in range(steps):
        if tgt is None:
            P.render(model.params, frame, vd, lds_batch, sched)
        else:
            P.train_step(model, frame, vd, tgt, lds_batch, sched, grads_out=gout, adam=adam)
    torch.cuda.synchronize()
    out = dict(frame=frame, model=model)
    out["status"] = frame.status_bits()
    out["tiles"] = u32(frame.tiles).reshape(len(views), n)
    out["rect"] = u32(frame.rect).reshape(len(views), n, 2)
    out["geo"] = frame.geo.cpu().numpy().reshape(len(views), n, 4)
    out["geo2"] = frame.geo2.cpu().numpy().reshape(len(views), n, 4)
    out["rgb"] = frame.rgb_s.cpu().numpy().reshape(len(views), n, 4)
    out["offsets"] = u32(frame.offsets)
    K = int(out["offsets"][-1])
    out["K"] = K
    out["keys"] = u32(frame.keys)[:K]
    out["vals"] = u32(frame.vals)[:K]
    out["gid"] = u32(frame.gid)[:K]
    out["ranges"] = u32(frame.ranges)
    out["image"] = frame.image.cpu().numpy()
    out["T"] = frame.T.cpu().numpy()
    out["last"] = u32(frame.last)
    if tile_stats:
        out["tile_stats"] = u32(frame.tile_stats)
    if tgt is not None:
        out["partials"] = frame.partials.cpu().numpy()[:K]
        out["loss_tiles"] = frame.loss_tiles.cpu().numpy()
        out["params"] = P.unpack_flat(model.params).cpu().numpy()
        out["m"] = P.unpack_flat(model.m).cpu().numpy()
        out["v"] = P.unpack_flat(model.v).cpu().numpy()
        if gout is not None:
            out["grads"] = P.unpack_flat(gout).cpu().numpy()
    return out


def per_gaussian_2d(partials, offsets, V, n):
    """Sum each Gaussian's intersection records: [V, N, 9]."""
    out = np.zeros((V * n, 9))
    rec = partials[:, :9].astype(np.float64)
    cs = np.concatenate([np.zeros((1, 9)), np.cumsum(rec, axis=0)])
    o = offsets.astype(np.int64)
    out[:] = cs[o[1:]] - cs[o[:-1]]
    return out.reshape(V, n, 9)


def rect_from_packed(r):
    return np.stack([r[..., 0] & 0xFFFF, r[..., 0] >> 16, r[..., 1] & 0xFFFF, r[..., 1] >> 16], -1)
