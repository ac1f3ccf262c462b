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
                 capacity=None, sched_order=None, persistent=False, tile_stats=False, steps=1,
                 pixels_per_lane=None, cull=0, bwd_batch=None, dLdC=None):
    """One or more steps through the C ABI.  target: L1 training against it;
    dLdC ([pixels, 3]): training with that image gradient instead; neither:
    forward only."""
    import torch
    from paper_2605_00219_amd import pipeline as P
    n = scene.n
    model = P.Model(scene.flat(), lr=lr)
    frame = P.Frame(n, [int(v["width"]) for v in views], [int(v["height"]) for v in views], tile,
                    capacity=capacity or 1024, tile_stats=tile_stats, pixels_per_lane=pixels_per_lane,
                    cull=cull)
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
    gimg = None if dLdC is None else torch.as_tensor(np.ascontiguousarray(dLdC, np.float32),
                                                      device="cuda").reshape(-1, 3)
    gout = torch.zeros_like(model.params) if grads else None
    for _ in range(steps):
        if tgt is None and gimg is None:
            P.render(model.params, frame, vd, lds_batch, sched)
        else:
            P.train_step(model, frame, vd, tgt, lds_batch, sched, grads_out=gout, adam=adam,
                         bwd_batch=bwd_batch, dLdC=gimg)
    torch.cuda.synchronize()
    out = dict(frame=frame, model=model)
    out["status"] = frame.status_bits()
    out["tiles"] = u32(frame.tiles).reshape(len(views), n)
    rec = frame.rec.cpu().numpy().reshape(len(views), n, 16)
    out["rec"] = rec
    out["rect"] = rec[..., 12:14].copy().view(np.uint32)
    out["offsets"] = u32(frame.offsets)
    out["row_offsets"] = u32(frame.row_offsets)
    out["rows"] = u32(frame.rows)[:int(out["row_offsets"][-1])]
    K = int(out["offsets"][-1])
    out["K"] = K
    out["keys"] = u32(frame.keys)[:K]
    out["vals"] = u32(frame.vals)[:K]
    out["ranges"] = u32(frame.ranges)
    out["tile_stop"] = u32(frame.tile_stop)
    out["comp_mask"] = u32(frame.comp_mask)
    out["rec_mask"] = u32(frame.rec_mask)
    out["image"] = frame.image.cpu().numpy()
    out["T"] = frame.T.cpu().numpy()
    out["last"] = u32(frame.last)
    if tile_stats:
        out["tile_stats"] = u32(frame.tile_stats)
    if tgt is not None or gimg is not None:
        out["grec"] = frame.grec.cpu().numpy()[:K]
        out["sums"] = frame.sums.cpu().numpy().reshape(9, len(views), n).transpose(1, 2, 0)
        out["loss_tiles"] = frame.loss_tiles.cpu().numpy()
        out["params"] = P.unpack_flat(model.params).cpu().numpy()
        out["m"] = P.unpack_flat(model.m).cpu().numpy()
        out["v"] = P.unpack_flat(model.v).cpu().numpy()
        if gout is not None:
            out["grads"] = P.unpack_flat(gout).cpu().numpy()
    return out


def per_gaussian_2d(grec, sorted_to_unsorted, vals, ranges, tile_stop, tile_base, n):
    """Sum the traversed records (stored at unsorted indices) of each
    (view, Gaussian): [V, N, 9].  tile_base: global tile base of each view
    plus the total."""
    V = len(tile_base) - 1
    out = np.zeros((V, n, 9))
    for v in range(V):
        for t in range(tile_base[v], tile_base[v + 1]):
            s, e = int(ranges[t, 0]), int(tile_stop[t])
            if e > s:
                idx = sorted_to_unsorted[s:e]
                np.add.at(out[v], vals[s:e], grec[idx, :9].astype(np.float64))
    return out


def rect_from_packed(r):
    return np.stack([r[..., 0] & 0xFFFF, r[..., 0] >> 16, r[..., 1] & 0xFFFF, r[..., 1] >> 16], -1)
