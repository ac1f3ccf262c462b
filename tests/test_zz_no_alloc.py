"""gs_project_bwd_adam_noalloc (the library's static device scratch) against
gs_project_bwd_adam (the caller's workspace), through the C ABI: two calls in
a row on one GPU, the second on a smaller input, must give the same
parameters, moments, gradients and per-(view, Gaussian) sums bit for bit;
a capacity beyond the static scratch is refused before anything runs."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_common import note

pytestmark = pytest.mark.gpu


def _backward_state(scene, target_scene, views, tile):
    import torch
    from paper_2605_00219_amd import pipeline as P
    vd = P.views_to_device(views)
    target = torch.as_tensor(np.ascontiguousarray(oracle.render(target_scene, views, tile), np.float32),
                             device="cuda").reshape(-1, 3)
    frame = P.Frame(scene.n, [int(v["width"]) for v in views], [int(v["height"]) for v in views], tile)
    params0 = P.Model(scene.flat()).params
    P.fit_capacity(params0, frame, vd)
    P.project(params0, frame, vd)
    P.bin_sort(frame)
    P.rasterize_fwd(frame, vd, 128)
    P.rasterize_bwd(frame, vd, target=target, lds_batch=128)
    torch.cuda.synchronize()
    assert frame.status_bits() == 0
    return frame, vd


def _run(fn, scene, frame, vd):
    import torch
    from paper_2605_00219_amd import pipeline as P
    model = P.Model(scene.flat())
    grads = torch.zeros_like(model.params)
    fn(model, frame, vd, grads_out=grads)
    torch.cuda.synchronize()
    return {"params": model.params.cpu().numpy(), "m": model.m.cpu().numpy(), "v": model.v.cpu().numpy(),
            "grads": grads.cpu().numpy(), "sums": frame.sums.cpu().numpy()}


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    from paper_2605_00219_amd import pipeline as P
    big = (S.scene_normal(40_000, 9100, log_scale_mean=-3.5), S.scene_normal(40_000, 9101, log_scale_mean=-3.5),
           S.views_array([S.make_view(320, 240, (0.0, 0.0, -5.0)), S.make_view(256, 192, (3.0, 1.0, -4.0))]), 16)
    w = S.workload_plain_small()
    small = (w.scene, w.target_scene, w.views, 16)
    for label, (scene, target_scene, views, tile) in (("first call, 40k Gaussians, 2 views", big),
                                                      ("second call, 2k Gaussians, 1 view", small)):
        note(f"no-alloc entry point: {label}")
        frame, vd = _backward_state(scene, target_scene, views, tile)
        noalloc = _run(P.project_bwd_adam_noalloc, scene, frame, vd)
        ref = _run(P.project_bwd_adam, scene, frame, vd)
        for k in ref:
            np.testing.assert_array_equal(noalloc[k], ref[k], err_msg=f"{label}: {k}")
        assert np.abs(ref["grads"]).max() > 0


def test_noalloc_refuses_capacity_beyond_its_scratch():
    from paper_2605_00219_amd import _lib as G
    from paper_2605_00219_amd import pipeline as P
    w = S.workload_plain_small()
    note("no-alloc entry point: capacity beyond the static scratch")
    frame, vd = _backward_state(w.scene, w.target_scene, w.views, 16)
    model = P.Model(w.scene.flat())
    bins = G.GsBins.from_buffer_copy(frame.bins)
    bins.capacity = 400_000_000          # needs more than the static scratch holds
    need = int(G.lib.gs_grads2d_workspace_size(bins.capacity))
    assert need > G.NOALLOC_SCRATCH_BYTES
    rc = G.lib.gs_project_bwd_adam_noalloc(P._i(model.params), frame.n, P._i(vd), C.byref(frame.layout),
                                           C.byref(frame.splats), C.byref(bins), C.byref(frame.grads2d),
                                           C.byref(model.adam), None, G.stream_ptr(None))
    assert rc == -3, rc        # GS_ERR_WORKSPACE
    assert b"scratch" in G.lib.gs_last_error()
    # within the limit the same call works
    frame2, vd2 = _backward_state(w.scene, w.target_scene, w.views, 16)
    P.project_bwd_adam_noalloc(P.Model(w.scene.flat()), frame2, vd2)
