"""Run by test_gpu_graph_capture.py in a fresh process: the process's first
gs_bin_sort call is made inside a HIP graph capture; replays must equal an
eager call bit for bit.  argv[1]: "side" (the frame's side stream takes the
depth sort) or "single" (one stream)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import synthetic as S  # noqa: E402
from paper_2605_00219_amd import pipeline as P  # noqa: E402


def main():
    side = sys.argv[1] == "side"
    w = S.workload_plain_small()
    n = w.scene.n
    vd = P.views_to_device(w.views)
    params = P.pack_flat(w.scene.flat())
    # capacity >= 12 x views x n: the depth-first order, the one with a side stream
    cap = 16 * n
    frame = P.Frame(n, [256], [256], 16, capacity=cap, side_stream=side)
    P.project(params, frame, vd)          # eager: loads the library's kernels
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.project(params, frame, vd)
        P.bin_sort(frame)                 # the first gs_bin_sort of this process
    torch.cuda.synchronize()
    ref = P.Frame(n, [256], [256], 16, capacity=cap, side_stream=side)
    P.project(params, ref, vd)
    P.bin_sort(ref)
    torch.cuda.synchronize()
    K = ref.intersections()
    assert 0 < K <= cap and ref.status_bits() == 0
    for r in range(3):
        for t in (frame.keys, frame.vals, frame.ranges, frame.offsets, frame.rows):
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert frame.status_bits() == 0
        for name in ("offsets", "row_offsets", "ranges"):
            assert torch.equal(getattr(frame, name), getattr(ref, name)), (r, name)
        assert torch.equal(frame.keys[:K], ref.keys[:K]), (r, "keys")
        assert torch.equal(frame.vals[:K], ref.vals[:K]), (r, "vals")
        # eager work between replays
        P.project(params, ref, vd)
        torch.cuda.synchronize()
    print(f"CAPTURE_OK side={side} K={K}", flush=True)


if __name__ == "__main__":
    main()
