"""gs_project_bwd_adam_noalloc against gs_project_bwd_adam, through the C ABI:
two calls in a row on one GPU, the second on a smaller input, must give the
same parameters, moments, gradients and per-(view, Gaussian) sums bit for
bit (neither entry point needs scratch: the gradient buffers carry no
workspace)."""
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


def test_noalloc_matches_entry_point_on_two_calls():
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
