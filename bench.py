"""Training-step throughput of the 3DGS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10]

Default workload: 300k Gaussians (means ~N(0,1)^3, log-scales ~N(-4,0.7)),
1280x720, 50 cameras on a radius-5 sphere, one view per L1 training step,
16x16 tiles (targets rendered from a held-out 300k-Gaussian scene outside the
timed region).  A step is the whole hot path: project -> bin_sort ->
rasterize_fwd -> rasterize_bwd (fused L1 gradient) -> project_bwd_adam.

The timed steps are replayed from one HIP graph per camera, captured outside
the timed region (--no-graph: eager launches); an eager pass of the same steps
gives the per-stage times, the work counts and the rooflines, and its rate is
reported under `eager`.

Prints one JSON line.  `roofline` describes the kernel with the largest share
of the step; `cpu_baseline` times the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train iters/sec + rasterize_bwd HBM GB/s (% peak), batched/learned vs plain"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak without packed instructions (the build disables them): one
# FMA (2 flops) per lane per clock, 256 CUs x 64 lanes x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6
# VALU issue: each of the 1024 SIMDs (16 lanes) starts one wave64 instruction
# every 4 clocks at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
# the rasterisation backward's bytes in the metric's own model: 80 per
# traversed (Gaussian, tile) entry (44 read, 36 of partials written) and 32 per
# pixel (C, target, T, last)
METRIC_BWD_BYTES_TRAVERSED = 80
METRIC_BWD_BYTES_PIXEL = 32

# Algorithmic work per unit of each stage (the same figures are derived in the
# design notes): bytes that must cross HBM, or flops that must be executed.
PROJ_BYTES_G = 308           # parameters 240 read; splat record 64 + tile count 4 written
SORT_BYTES_G = 96            # per (view, Gaussian): count/offset/row-count scans 16; depth key and
                             # index 8 w; depth histogram 4 r; 3 depth passes x 16; depth-order
                             # scan 16 (index, count, offset r; shift w); emit reads the shift 4
SORT_BYTES_ROW = 32          # per tile-row slot: written 16, read by the emit 16
SORT_BYTES_K = 48            # per intersection: emit 8 w; tile histogram 4 r; 2 passes x (8 r + 8 w);
                             # ranges 4 r
# with few intersections per (view, Gaussian) all 32 key bits are sorted directly
SORT_DIRECT_BYTES_G = 16     # count/offset/row-count scans
SORT_DIRECT_BYTES_K = 80     # emit 8 w; histogram 4 r; 4 passes x (8 r + 8 w); ranges 4 r
SORT_DEPTH_FIRST_RATIO = 12  # capacity / (views x n) from which the depth order is used
FWD_FLOP_EVAL = 14           # power, G, alpha, thresholds per evaluated pixel-Gaussian pair
FWD_FLOP_COMP = 9            # colour and transmittance update per composited pair
BWD_BYTES_TRAVERSED = 40     # Gaussian id 4 + splat 36 read per traversed entry
BWD_BYTES_FLAGGED = 64       # row slot 16 read, gradient record 48 written per composited entry
BWD_BYTES_PIXEL = 28         # C 12 + target 12 + last 4
BWD_BYTES_TILE = 16          # range 8 + loss 4 + stop 4
BWD_FLOP_EVAL = 14           # recompute of power, G, alpha, thresholds per evaluated pair
BWD_FLOP_CONTRIB = 44        # gradient terms and their sums per composited pair
ADAM_BYTES_G = 1516          # params, m, v 720 r + 720 w; offsets 4; per-view sums 36 w + 36 r
ADAM_BYTES_FLAGGED = 48      # one gradient record read per composited entry (+ K/8 of mask)
LOSS_FLOP_PX = 1215          # L1 + D-SSIM gradient, per pixel (3 channels x 405): window sums of
                             # x, y, x^2, y^2, xy (5 x 2 passes x 11 FMA) 220, products 3, SSIM and
                             # its three derivatives 40, window sums of the derivative maps
                             # (3 x 2 x 11 FMA) 132, L1 sign and the gradient 10
LOSS_BYTES_PX = 28           # render 12 + RGBA8 reference 4 read, dL/dC 12 written
LOSS_KERNEL_BYTES_PX = 116   # two-kernel form: derivative maps 36 written and read back, render
                             # and reference read by both kernels


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha() -> str:
    """Hash of every HIP source and the C header (any change to the kernels
    invalidates counters taken before it)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2605_00219_amd", "csrc", "*")))
    for p in files + [os.path.join(ROOT, "include", "gs.h")]:
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def recorded_traffic(stage: str):
    """HBM bytes per launch of a stage measured by rocprofv3 counters
    (profiles/hbm_traffic.json), or None if absent or if the kernel sources
    have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(stage)
        if rec and rec.get("source_sha") == source_sha():
            return rec
    except (OSError, ValueError, KeyError):
        pass
    return None


def bwd_figures(rb, counts, P_px, kernel="rasterize_bwd"):
    """The backward's work counts and rates (design byte model, flops, and the
    counters recorded for it when current)."""
    t = rb["ms"] * 1e-3
    out = {"ms": rb["ms"], "algorithmic_bytes": rb["algorithmic_bytes"], "hbm_gbs": rb["hbm_gbs"],
           "hbm_frac": rb["hbm_frac"], "algorithmic_flop": rb["algorithmic_flop"],
           "tflops": rb["achieved"], "alu_frac": rb["frac"],
           "intersections": counts["K"], "traversed": counts["trav_bwd"],
           "composited_entries": counts["flagged"], "pairs_evaluated": counts["eval_bwd"],
           "pairs_composited": counts["contrib"], "visible_gaussians": counts["visible"],
           "pairs_per_traversed_entry": counts["eval_bwd"] / max(counts["trav_bwd"], 1)}
    tr = recorded_traffic(kernel)
    if tr is not None:
        out["measured_hbm_bytes"] = tr["bytes_per_launch"]
        out["measured_hbm_gbs"] = tr["bytes_per_launch"] / t / 1e9
        out["measured_hbm_frac"] = tr["bytes_per_launch"] / t / 1e9 / HBM_PEAK_GBS
    return out


def headline_roofline(rb, counts, P_px, kernel="rasterize_bwd"):
    """rasterize_bwd against HBM in the metric's byte model (80 B per traversed
    entry + 32 B per pixel), the counter-measured bytes as traffic, and beside
    it the ALU (non-packed fp32) and VALU-issue fractions."""
    t = rb["ms"] * 1e-3
    nbytes = METRIC_BWD_BYTES_TRAVERSED * counts["trav_bwd"] + METRIC_BWD_BYTES_PIXEL * P_px
    gbs = nbytes / t / 1e9
    tr = recorded_traffic(kernel)
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": tr["bytes_per_launch"] if tr else None, "kernel": kernel,
            "algorithmic_bytes": nbytes, "ms": rb["ms"],
            "traffic_source": (f"rocprofv3 FETCH_SIZE + WRITE_SIZE, sources {tr['source_sha']}" if tr else None),
            "alu": {"achieved": rb["achieved"], "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": rb["frac"]}}
    if tr is not None and tr.get("valu_insts_per_launch"):
        ips = tr["valu_insts_per_launch"] / t
        roof["valu_issue"] = {"achieved": ips, "peak": VALU_ISSUE_PEAK, "unit": "wave64 instructions/s",
                              "frac": ips / VALU_ISSUE_PEAK}
    return roof


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--lds-batch", type=int, default=128)
    ap.add_argument("--n", type=int, default=300_000)
    ap.add_argument("--log-scale-mean", type=float, default=-4.0,
                    help="log-scale distribution of the headline scene (N(-6, 0.3): the sparse-footprint "
                         "form, for profiling it on its own)")
    ap.add_argument("--log-scale-std", type=float, default=0.7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-replay", action="store_true", help="skip the work-counting replay")
    ap.add_argument("--no-graph", action="store_true",
                    help="report the eager steps' rate (default: steps replayed as per-camera HIP graphs; "
                         "stage times always come from an eager pass)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--variants", default="sparse,ellipse,ssim,twophase,thompson,batched,learned",
                    help="comma list of extra measurements: sparse, ellipse, ssim, twophase, thompson, "
                         "batched, learned ('none' for none)")
    ap.add_argument("--cull", type=int, default=0, choices=(0, 1),
                    help="tile set of the headline run: 0 = 3-sigma rectangle, 1 = exact ellipse")
    ap.add_argument("--ppl", type=int, default=None, choices=(1, 2, 4),
                    help="pixels per lane of the headline run (default: the layout's, 2 on 16x16 tiles; "
                         "the sparse-footprint variant runs at 1)")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--batched-plain-steps", type=int, default=25)
    ap.add_argument("--learned-steps", type=int, default=10)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; multi-GPU runs are not supported "
                          "(the path is data-parallel over views: one replica of the Gaussians per GPU, "
                          "gradients all-reduced before the optimiser)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic as S
    from paper_2605_00219_amd import pipeline as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating workload")
    w = S.workload_plain_300k(n=args.n, log_scale_mean=args.log_scale_mean, log_scale_std=args.log_scale_std)
    n = w.scene.n
    W, H = int(w.views[0]["width"]), int(w.views[0]["height"])
    ncam = len(w.views)
    views_all = P.views_to_device(w.views)           # ncam x 128 bytes
    vptr = lambda i: views_all[128 * i:128 * (i + 1)]

    # targets: rendered by the GPU forward from the held-out scene (not timed)
    log("rendering targets")
    tgt_model = P.Model(w.target_scene.flat())
    tframe = P.Frame(n, [W], [H], 16)
    targets = torch.empty(ncam, H * W, 3, device=dev)
    variants = [v for v in args.variants.split(",") if v]
    # RGBA8 references for the L1 + D-SSIM variant: the target render quantised
    # to 8 bits, its coverage 1 - T as the alpha mask
    targets8 = torch.empty(ncam, H * W, 4, dtype=torch.uint8, device=dev) if "ssim" in variants else None
    for i in range(ncam):
        P.fit_capacity(tgt_model.params, tframe, vptr(i))
        targets[i].copy_(P.render(tgt_model.params, tframe, vptr(i)))
        if targets8 is not None:
            rgba = torch.cat([targets[i], 1.0 - tframe.T[:, None]], 1)
            targets8[i].copy_(torch.round(rgba.clamp(0, 1) * 255).to(torch.uint8))
    del tgt_model, tframe
    targets_main = targets

    def run_plain(cull, replay, loss="l1", ts_arms=None, bwd_variant=None, graph=False, wk=None, tg=None,
                  ppl=None):
        """Timed plain steps (and the work-counting replay) with the given tile
        culling; loss "l1" (fused into the backward) or "ssim" (L1 + D-SSIM
        against the RGBA8 references, lambda 0.2, alpha mask); wk, tg: another
        scene of the same size with its targets (same cameras); ppl: pixels
        per lane (None: the layout's default, 2 on 16x16 tiles)."""
        wk = wk or w
        targets = tg if tg is not None else targets_main
        model = P.Model(wk.scene.flat(), lr=wk.lr)
        frame = P.Frame(n, [W], [H], 16, cull=cull, pixels_per_lane=ppl)
        lossfn = P.LossL1SSIM(frame, 0.2, True) if loss == "ssim" else None
        # backward LDS batch chosen per step by Thompson sampling over ts_arms
        sbwd = P.ScheduledBackward(ts_arms, seed=0, prior_ms=0.3) if ts_arms else None
        kmax = 0
        for i in range(ncam):
            kmax = max(kmax, P.fit_capacity(model.params, frame, vptr(i)))
        frame.resize(int(kmax * 1.3) + 4096)
        order = [int(x) for x in w.view_order]

        def step(i, ev=None):
            vi = order[i % ncam]
            vd = vptr(vi)
            if ev is not None:
                ev[0].record()
            P.project(model.params, frame, vd)
            if ev is not None:
                ev[1].record()
            P.bin_sort(frame)
            if ev is not None:
                ev[2].record()
            P.rasterize_fwd(frame, vd, args.lds_batch)
            if ev is not None:
                ev[3].record()
            k = 4
            if lossfn is not None:
                lossfn(targets8[vi])
                if ev is not None:
                    ev[4].record()
                k = 5
                P.rasterize_bwd(frame, vd, dLdC=lossfn.dLdC, lds_batch=args.lds_batch)
            elif sbwd is not None:
                sbwd(frame, vd, target=targets[vi])
            elif bwd_variant is not None:
                P.backward(frame, vd, bwd_variant, target=targets[vi])
            else:
                P.rasterize_bwd(frame, vd, target=targets[vi], lds_batch=args.lds_batch)
            if ev is not None:
                ev[k].record()
            P.project_bwd_adam(model, frame, vd)
            if ev is not None:
                ev[k + 1].record()

        log(f"warmup {args.warmup} steps (N={n}, {W}x{H}, K<={kmax})")
        for i in range(args.warmup):
            step(i)
        torch.cuda.synchronize()
        if frame.status_bits():
            raise RuntimeError("intersection capacity exceeded during warmup")
        state0 = [t.clone() for t in (model.params, model.m, model.v, model.step)]
        if graph:
            # one HIP graph per camera (each step reads its own view and target),
            # captured after a launch outside capture; the optimiser state is
            # restored afterwards, so the timed steps start where they would
            graphs = {}
            cs = torch.cuda.Stream()
            for vi in sorted(set(order)):
                cs.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(cs):
                    step(order.index(vi))
                torch.cuda.current_stream().wait_stream(cs)
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    step(order.index(vi))
                graphs[vi] = g
            torch.cuda.synchronize()
            for t, s0 in zip((model.params, model.m, model.v, model.step), state0):
                t.copy_(s0)
            for i in range(args.warmup):
                graphs[order[i % ncam]].replay()
            torch.cuda.synchronize()
            for t, s0 in zip((model.params, model.m, model.v, model.step), state0):
                t.copy_(s0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.steps):
                graphs[order[(args.warmup + i) % ncam]].replay()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if frame.status_bits():
                raise RuntimeError("intersection capacity exceeded in the timed region")
            log(f"plain graph (cull {cull}): {args.steps / wall:.1f} iters/s")
            out = dict(ips=args.steps / wall, wall=wall, stage_ms=None, counts=None, kmax=kmax,
                       ntiles=frame.layout.total_tiles, depth_first=None, loss=None, ts=None)
            del graphs, model, frame, lossfn, sbwd
            torch.cuda.empty_cache()
            return out

        # timed region: plain single-view steps
        stages = ["project", "bin_sort", "rasterize_fwd", "rasterize_bwd", "project_bwd_adam"]
        if lossfn is not None:
            stages.insert(3, "loss_l1_ssim")
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(args.warmup + i, evs[i])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if frame.status_bits():
            raise RuntimeError("intersection capacity exceeded in the timed region")
        wall = t1 - t0
        stage_ms = {s: float(np.mean([evs[i][k].elapsed_time(evs[i][k + 1]) for i in range(args.steps)]))
                    for k, s in enumerate(stages)}
        ips = args.steps / wall
        log(f"plain (cull {cull}, loss {loss}): {ips:.1f} iters/s, {1e3 * wall / args.steps:.3f} ms/step; "
            f"stages {stage_ms}")

        # replay of the timed steps (deterministic) counting the work each kernel did
        counts = None
        if replay:
            for t, s0 in zip((model.params, model.m, model.v, model.step), state0):
                t.copy_(s0)
            rframe = P.Frame(n, [W], [H], 16, capacity=frame.capacity, tile_stats=True, cull=cull,
                             row_capacity=frame.row_capacity, pixels_per_lane=ppl)
            gx = (W + 15) // 16
            tile_of_px = torch.arange(H * W, device=dev)
            tile_of_px = (tile_of_px // W // 16) * gx + (tile_of_px % W) // 16
            acc = dict(K=0, trav_bwd=0, eval_bwd=0, contrib=0, eval_fwd=0, trav_fwd=0, visible=0, flagged=0,
                       rows=0)
            for i in range(args.steps):
                vi = order[(args.warmup + i) % ncam]
                vd = vptr(vi)
                P.project(model.params, rframe, vd)
                P.bin_sort(rframe)
                P.rasterize_fwd(rframe, vd, args.lds_batch)
                last = rframe.last.to(torch.int64)
                per_tile = torch.zeros(rframe.layout.total_tiles, dtype=torch.int64, device=dev)
                per_tile.scatter_reduce_(0, tile_of_px, last, reduce="amax")
                ts = rframe.tile_stats.to(torch.int64)
                acc["K"] += rframe.intersections()
                acc["rows"] += int(rframe.row_offsets[-1].item())
                acc["visible"] += int((rframe.tiles != 0).sum().item())
                acc["trav_bwd"] += int(per_tile.sum().item())
                acc["eval_bwd"] += int(last.sum().item())
                acc["contrib"] += int(ts[:, 2].sum().item())
                acc["eval_fwd"] += int(ts[:, 1].sum().item())
                acc["trav_fwd"] += int(ts[:, 0].sum().item())
                P.rasterize_bwd(rframe, vd, target=targets[vi], lds_batch=args.lds_batch)
                nw = (rframe.intersections() + 31) // 32
                acc["flagged"] += int(np.unpackbits(rframe.rec_mask[:nw].cpu().numpy().view(np.uint8)).sum())
                P.project_bwd_adam(model, rframe, vd)
            torch.cuda.synchronize()
            counts = {k: v / args.steps for k, v in acc.items()}
            log(f"per-step work: {counts}")
        if lossfn is not None:
            out_loss = lossfn.loss()
        ts_out = None
        if sbwd is not None:
            sbwd.harvest(block=True)
            timed = sbwd.history[-args.steps:]
            ts_out = {"arms": [str(a) for a in sbwd.arms],
                      "picks_timed": [timed.count(a) for a in range(len(sbwd.arms))],
                      "picks_all": sbwd.ts.counts(),
                      "posterior_mean_ms": [sbwd.ts.posterior(a)[0] for a in range(len(sbwd.arms))]}
        out = dict(stage_ms=stage_ms, ips=ips, wall=wall, counts=counts, kmax=kmax,
                   loss=out_loss if lossfn is not None else None, ts=ts_out,
                   ntiles=frame.layout.total_tiles,
                   depth_first=frame.capacity >= SORT_DEPTH_FIRST_RATIO * n)
        del model, frame, lossfn, sbwd
        torch.cuda.empty_cache()
        return out

    order = [int(x) for x in w.view_order]
    res = run_plain(args.cull, not args.no_replay, ppl=args.ppl)
    stage_ms, ips, wall, counts = res["stage_ms"], res["ips"], res["wall"], res["counts"]
    cull_variant = None
    if "ellipse" in variants and args.cull == 0:
        r2 = run_plain(1, True)
        c2 = r2["counts"]
        cull_variant = {"culling": "ellipse", "iters_per_s": r2["ips"],
                        "ms_per_step": 1e3 * r2["wall"] / args.steps, "stage_ms": r2["stage_ms"],
                        "intersections": c2["K"] if c2 else None,
                        "traversed": c2["trav_bwd"] if c2 else None,
                        "pairs_evaluated_bwd": c2["eval_bwd"] if c2 else None,
                        "speedup_vs_rect": r2["ips"] / ips}
    # headline: the same steps replayed from one HIP graph per camera
    eager = {"iters_per_s": ips, "ms_per_step": 1e3 * wall / args.steps}
    value, value_wall = ips, wall
    if not args.no_graph:
        rg = run_plain(args.cull, False, graph=True, ppl=args.ppl)
        value, value_wall = rg["ips"], rg["wall"]
    tp_variant = None
    if "twophase" in variants:
        tp_variant = {}
        for sb in (16, 32):
            r5 = run_plain(args.cull, False, bwd_variant=("twophase", sb))
            tp_variant[f"S{sb}"] = {"iters_per_s": r5["ips"], "ms_per_step": 1e3 * r5["wall"] / args.steps,
                                   "rasterize_bwd_ms": r5["stage_ms"]["rasterize_bwd"],
                                   "vs_first_backward": stage_ms["rasterize_bwd"] / r5["stage_ms"]["rasterize_bwd"]}
    ts_variant = None
    if "thompson" in variants:
        r4 = run_plain(args.cull, False, ts_arms=(128, 256, -128, ("twophase", 16), ("twophase", 32)))
        ts_variant = {"arms": "first backward with LDS batch 128, 256, per tile (cap 128); two-phase "
                              "backward with batch 16, 32",
                      "iters_per_s": r4["ips"], "ms_per_step": 1e3 * r4["wall"] / args.steps,
                      "stage_ms": r4["stage_ms"], "vs_fixed": r4["ips"] / ips, **r4["ts"]}
    ssim_variant = None
    if "ssim" in variants:
        r3 = run_plain(args.cull, False, loss="ssim")
        t_loss = r3["stage_ms"]["loss_l1_ssim"] * 1e-3
        px = H * W
        ssim_variant = {
            "loss": "0.8 L1 + 0.2 D-SSIM, RGBA8 reference, alpha mask", "iters_per_s": r3["ips"],
            "ms_per_step": 1e3 * r3["wall"] / args.steps, "stage_ms": r3["stage_ms"],
            "final_loss": r3["loss"], "slowdown_vs_l1": ips / r3["ips"],
            "loss_roofline": {
                "bound": "alu", "kernel": "loss_l1_ssim", "ms": 1e3 * t_loss,
                "achieved": LOSS_FLOP_PX * px / t_loss / 1e12, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": LOSS_FLOP_PX * px / t_loss / 1e12 / FP32_PEAK_TFLOPS,
                "algorithmic_flop": LOSS_FLOP_PX * px,
                "algorithmic_bytes": LOSS_BYTES_PX * px,
                "hbm_gbs": LOSS_BYTES_PX * px / t_loss / 1e9,
                "kernel_bytes": LOSS_KERNEL_BYTES_PX * px,
                "kernel_bytes_gbs": LOSS_KERNEL_BYTES_PX * px / t_loss / 1e9}}
        del targets8

    # per-stage rooflines (each stage's own bound and algorithmic work) under
    # stage_roofline; the headline `roofline` is rasterize_bwd's (the kernel the
    # metric names, and the step's longest single kernel) against HBM, with its
    # ALU and VALU-issue figures beside it
    roof = None
    extra = {}
    P_px = H * W
    ntiles = res["ntiles"]
    if counts is not None:
        def hbm(name, nbytes, kernel):
            t = stage_ms[name] * 1e-3
            gbs = nbytes / t / 1e9
            tr = recorded_traffic(kernel)
            return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "traffic": tr["bytes_per_launch"] if tr else None,
                    "kernel": kernel, "algorithmic_bytes": nbytes, "ms": stage_ms[name]}

        def alu(name, flop, nbytes, kernel):
            t = stage_ms[name] * 1e-3
            tf = flop / t / 1e12
            tr = recorded_traffic(kernel)
            return {"bound": "alu", "achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tf / FP32_PEAK_TFLOPS, "traffic": tr["bytes_per_launch"] if tr else None,
                    "kernel": kernel, "algorithmic_flop": flop, "algorithmic_bytes": nbytes,
                    "hbm_gbs": nbytes / t / 1e9, "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS,
                    "ms": stage_ms[name]}

        vis = counts["visible"]
        per_stage = {
            "project": hbm("project", PROJ_BYTES_G * n, "project"),
            "bin_sort": hbm("bin_sort", SORT_BYTES_G * n + SORT_BYTES_ROW * counts["rows"]
                            + SORT_BYTES_K * counts["K"] if res["depth_first"] else
                            SORT_DIRECT_BYTES_G * n + SORT_BYTES_ROW * counts["rows"]
                            + SORT_DIRECT_BYTES_K * counts["K"], "bin_sort"),
            "rasterize_fwd": alu("rasterize_fwd",
                                 FWD_FLOP_EVAL * counts["eval_fwd"] + FWD_FLOP_COMP * counts["contrib"],
                                 68 * counts["trav_fwd"] + 20 * P_px + 8 * ntiles, "rasterize_fwd"),
            "rasterize_bwd": alu("rasterize_bwd",
                                 BWD_FLOP_EVAL * counts["eval_bwd"] + BWD_FLOP_CONTRIB * counts["contrib"],
                                 BWD_BYTES_TRAVERSED * counts["trav_bwd"]
                                 + BWD_BYTES_FLAGGED * counts["flagged"] + BWD_BYTES_PIXEL * P_px
                                 + BWD_BYTES_TILE * ntiles, "rasterize_bwd"),
            "project_bwd_adam": hbm("project_bwd_adam",
                                    ADAM_BYTES_G * n + ADAM_BYTES_FLAGGED * counts["flagged"]
                                    + counts["K"] / 8, "project_bwd_adam"),
        }
        rb = per_stage["rasterize_bwd"]
        extra["rasterize_bwd"] = bwd_figures(rb, counts, P_px)
        extra["stage_roofline"] = {k: {kk: v[kk] for kk in ("bound", "achieved", "unit", "frac")}
                                   for k, v in per_stage.items()}
        roof = headline_roofline(rb, counts, P_px)
    if roof is None:
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": "rasterize_bwd"}

    if "sparse" in variants:
        log("sparse-footprint variant: log-scales N(-6, 0.3)")
        ws_ = S.workload_plain_300k(n=args.n, log_scale_mean=-6.0, log_scale_std=0.3)
        tm = P.Model(ws_.target_scene.flat())
        tf_ = P.Frame(n, [W], [H], 16)
        tg_s = torch.empty(ncam, H * W, 3, device=dev)
        for i in range(ncam):
            P.fit_capacity(tm.params, tf_, vptr(i))
            tg_s[i].copy_(P.render(tm.params, tf_, vptr(i)))
        del tm, tf_
        # one pixel per lane: with footprints of about a pixel a wavefront
        # covering four tile rows instead of eight has fewer staged Gaussians
        # within reach to test and evaluate (rasterisers 0.24 against 0.29 ms
        # per step, event-timed)
        rs = run_plain(0, True, wk=ws_, tg=tg_s, ppl=1)
        cs = rs["counts"]
        t_s = rs["stage_ms"]["rasterize_bwd"] * 1e-3
        bytes_s = (BWD_BYTES_TRAVERSED * cs["trav_bwd"] + BWD_BYTES_FLAGGED * cs["flagged"]
                   + BWD_BYTES_PIXEL * P_px + BWD_BYTES_TILE * rs["ntiles"])
        rb_s = {"ms": rs["stage_ms"]["rasterize_bwd"], "algorithmic_bytes": bytes_s,
                "hbm_gbs": bytes_s / t_s / 1e9, "hbm_frac": bytes_s / t_s / 1e9 / HBM_PEAK_GBS,
                "algorithmic_flop": BWD_FLOP_EVAL * cs["eval_bwd"] + BWD_FLOP_CONTRIB * cs["contrib"]}
        rb_s["achieved"] = rb_s["algorithmic_flop"] / t_s / 1e12
        rb_s["frac"] = rb_s["achieved"] / FP32_PEAK_TFLOPS
        extra["sparse"] = {"workload": ws_.name, "log_scales": "N(-6, 0.3)", "pixels_per_lane": 1,
                           "iters_per_s": rs["ips"],
                           "ms_per_step": 1e3 * rs["wall"] / args.steps, "stage_ms": rs["stage_ms"],
                           "rasterize_bwd": bwd_figures(rb_s, cs, P_px, "rasterize_bwd_sparse"),
                           "roofline": headline_roofline(rb_s, cs, P_px, "rasterize_bwd_sparse")}
        del ws_, tg_s
        torch.cuda.empty_cache()

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    targets = targets_main = None                       # free the plain workload's buffers
    torch.cuda.empty_cache()
    if cull_variant is not None:
        extra["cull_ellipse"] = cull_variant
    if ssim_variant is not None:
        extra["ssim"] = ssim_variant
    if ts_variant is not None:
        extra["thompson"] = ts_variant
    if tp_variant is not None:
        extra["twophase"] = tp_variant

    if "batched" in variants:
        from paper_2605_00219_amd import experiments as X
        log("batched variant: 3M Gaussians, 8 uneven views per step")
        wb = S.workload_batched()
        cams, res = wb.extra["cameras"], wb.extra["resolutions"]
        extra["batched"] = X.run_batched(wb, lambda i: S.batched_views(cams, res, i),
                                         steps=args.batched_steps,
                                         plain_steps=args.batched_plain_steps, log=log)
        del wb
        torch.cuda.empty_cache()
    if "learned" in variants:
        from paper_2605_00219_amd import experiments as X
        log("learned-schedule variant: 6M Gaussians, 4 x 1920x1080 per step")
        wl = S.workload_learned()
        # traversal logs of differentiation-check-distribution scenes (anisotropic
        # scales, long-tailed opacity) from sparse to dense: 100k, 300k, 1M and
        # 3M Gaussians, 4 views each, so that both unsaturated tiles (cost grows
        # with the list) and saturated ones (cost set by the early stop) occur
        train_cams = S.fibonacci_sphere(50, 5.0)
        train_sets = [(S.scene_anisotropic(nk, 3000 + 10 * k),
                       S.views_array([S.make_view(1920, 1080, train_cams[(7 * k + j) % 50])
                                      for j in range(4)]))
                      for k, nk in enumerate((100_000, 300_000, 1_000_000, 3_000_000))]
        extra["learned"] = X.run_learned(wl, train_sets, steps=args.learned_steps, log=log)
        del wl, train_sets
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, order)

    out = {
        "metric": METRIC, "value": value, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * value_wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "gaussians": n, "width": W,
                   "height": H, "views_per_step": 1, "cameras": ncam, "tile": 16,
                   "lds_batch": args.lds_batch, "loss": "L1", "lr": w.lr,
                   "culling": "ellipse" if args.cull else "3-sigma rectangle",
                   "execution": "eager" if args.no_graph else "one HIP graph per camera, replayed"},
        "eager": eager,
        "stage_ms": stage_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(w, order, n_steps=3):
    """The CPU oracle, as it stands, on 3 full training steps of the same
    workload (one view each, the first 3 views of the step sequence); its
    targets are rendered by the oracle itself, outside the timed region."""
    import oracle
    log(f"cpu baseline: oracle, {n_steps} full steps, {oracle.threads()} threads")
    vis = [order[i] for i in range(n_steps)]
    tg = {vi: oracle.render(w.target_scene, w.views[vi:vi + 1], 16) for vi in vis}
    t0 = time.perf_counter()
    for vi in vis:
        oracle.train_step(w.scene, w.views[vi:vi + 1], 16, tg[vi], lr=w.lr)
    dt = time.perf_counter() - t0
    return {"value": n_steps / dt, "unit": "iters/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{n_steps} full L1 training steps (300k Gaussians, 1280x720, one view each)",
            "seconds": dt}


if __name__ == "__main__":
    main()
