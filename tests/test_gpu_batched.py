"""Several views of uneven resolution per step in one persistent launch,
captured into a HIP graph; the autotuner and its cache."""
import json
import os

import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_common import note
from helpers import checked_fraction, exempt_gaussians, grad_close, masked_image_gradient

pytestmark = pytest.mark.gpu

RES = [(160, 120), (200, 150), (256, 192), (320, 180)]


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2605_00219_amd import batched as B
    from paper_2605_00219_amd import pipeline as P
    scene = S.scene_normal(40_000, 4100, log_scale_mean=-3.5)
    target_scene = S.scene_normal(40_000, 4101, log_scale_mean=-3.5)
    cams = S.fibonacci_sphere(10, 5.0)
    return dict(torch=torch, B=B, P=P, scene=scene, target_scene=target_scene, cams=cams)


def _views(it, cams):
    return S.views_array([S.make_view(w, h, cams[(len(RES) * it + k) % len(cams)])
                          for k, (w, h) in enumerate(RES)])


def test_graph_persistent_batched_steps_match_eager_and_oracle(setup):
    d = setup
    torch, B, P = d["torch"], d["B"], d["P"]
    note("batched graph step vs eager vs oracle")
    iters = [0, 1, 2]
    views = {i: _views(i, d["cams"]) for i in iters}
    targets = {i: torch.as_tensor(oracle.render(d["target_scene"], views[i], 16), device="cuda")
               for i in iters}
    vrows = {i: P.views_to_device(views[i]) for i in iters}
    n = d["scene"].n
    # eager, one workgroup per tile
    m_e = P.Model(d["scene"].flat())
    f_e = P.Frame(n, [w for w, _ in RES], [h for _, h in RES], 16)
    for i in iters:
        P.fit_capacity(m_e.params, f_e, vrows[i])
    cap = f_e.capacity
    for i in iters:
        P.train_step(m_e, f_e, vrows[i], targets[i])
    # graph-captured, persistent
    m_g = P.Model(d["scene"].flat())
    step = B.BatchedStep(m_g, n, B.ViewSet(RES, 16), cap, lds_batch=64, persistent=True)
    for i in iters:
        step.load(vrows[i], targets[i])
        step.run()
    torch.cuda.synchronize()
    assert step.status() == 0
    for a, b in ((m_e.params, m_g.params), (m_e.m, m_g.m), (m_e.v, m_g.v)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert int(m_g.step.item()) == len(iters)
    # the first step against the oracle (gradients summed over the 4 views):
    # with the fused L1 gradient, every Gaussian no fragile pixel reaches ...
    ref = oracle.train_step(d["scene"], views[0], 16, targets[0].cpu().numpy())
    m1 = P.Model(d["scene"].flat())
    g = torch.zeros_like(m1.params)
    f1 = P.Frame(n, [w for w, _ in RES], [h for _, h in RES], 16, capacity=cap)
    P.train_step(m1, f1, vrows[0], targets[0], grads_out=g)
    got = P.unpack_flat(g).cpu().numpy()
    ex = exempt_gaussians(ref.proj, ref.bins, views[0], 16, ref.fragile).any(axis=0)
    touched = np.abs(ref.grads).max(axis=1) > 0
    checked_fraction(ex, touched, 0.5, "fused L1: ")
    ok = grad_close(got, ref.grads)
    assert not (~ok.all(axis=1) & ~ex).any()
    # ... and every Gaussian, gradients and Adam update, with the oracle's image
    # gradient zeroed at fragile pixels given to both sides
    dLdC = masked_image_gradient(ref.dLdC, ref.fragile)
    ref2 = oracle.train_step(d["scene"], views[0], 16, None, dLdC=dLdC)
    m2 = P.Model(d["scene"].flat())
    g2 = torch.zeros_like(m2.params)
    f2 = P.Frame(n, [w for w, _ in RES], [h for _, h in RES], 16, capacity=cap)
    P.train_step(m2, f2, vrows[0], None, grads_out=g2, dLdC=torch.as_tensor(dLdC, device="cuda"))
    got2 = P.unpack_flat(g2).cpu().numpy()
    ok2 = grad_close(got2, ref2.grads)
    checked_fraction(np.zeros(n, bool), np.abs(ref2.grads).max(axis=1) > 0, 1.0, "given gradient: ")
    assert ok2.all(), np.argwhere(~ok2)[:5]
    par = P.unpack_flat(m2.params).cpu().numpy()
    gmax = np.abs(ref2.grads).max(axis=0, keepdims=True)
    certain = np.abs(ref2.grads) >= 1e-3 * gmax
    tol = np.where(certain, 1e-3 * np.abs(ref2.params) + 1e-6, 2e-3 + 1e-6)
    assert (np.abs(par - ref2.params) <= tol).all()


def test_autotune_picks_a_candidate_and_caches(setup, tmp_path):
    d = setup
    torch, B, P = d["torch"], d["B"], d["P"]
    from paper_2605_00219_amd import autotune as AT
    note("autotune")
    iters = [0, 1]
    views = {i: _views(i, d["cams"]) for i in iters}
    vrows = {i: P.views_to_device(views[i]) for i in iters}
    tg = {}
    for i in iters:
        tg[i] = torch.as_tensor(oracle.render(d["target_scene"], views[i], 16), device="cuda")
    model = P.Model(d["scene"].flat())
    p0 = model.params.clone()
    cache = str(tmp_path / "autotune.json")
    res = AT.autotune(model, d["scene"].n, RES, lambda i: vrows[i], lambda i: tg[i], iters,
                      cache_path=cache, tiles=(8, 16), batches=(32, 64), lane_pixels=(2, 4), log=note)
    assert res["tile"] in (8, 16) and res["lds_batch"] in (32, 64) and not res["cached"]
    assert len(res["table_ms"]) == 6 and all(np.isfinite(v) for v in res["table_ms"].values())
    # optimiser state restored after tuning
    np.testing.assert_array_equal(model.params.cpu().numpy(), p0.cpu().numpy())
    assert int(model.step.item()) == 0
    again = AT.autotune(model, d["scene"].n, RES, lambda i: vrows[i], lambda i: tg[i], iters,
                        cache_path=cache, tiles=(8, 16), batches=(32, 64), lane_pixels=(2, 4), log=note)
    assert again["cached"] and again["tile"] == res["tile"]
    # a corrupt cache is ignored
    with open(cache, "w") as f:
        f.write("{not json")
    assert AT.load_cache(cache) == {}
