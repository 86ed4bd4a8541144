"""Times the single-instance sweeps at every tile G in {16, 32, 64} over a grid of shapes.

    python -m paper_2510_27351_amd.tile_sweep [--sizes 256,1024,4096,16384] [--reps 10] [--rounds 3] [--dtype f32|f64]

For each (m, n) of the grid it prints, per tile, the time of the forward (table, score,
checkpoint grid K=64), of the selection recompute alone and of the adjoint (selection
recompute followed by the reverse sweep, as every backward runs them), each the best of
`rounds` rounds of `reps` back-to-back calls, and the fastest tile for the forward and for
the adjoint.  The selection recompute does not depend on the tile; the reverse sweep is
timed behind it because that is where it always runs (the selections it reads were just
written).  The table is the training set of the library's tile predictor (wf_tile_predict:
the tile of the nearest timed shape in (log2 m, log2 n)); after a change to the kernels,
sweep again and replace the table in the library and its copy in the tests.  Inputs are
normal(0,1) clipped to [-4,4], float32 (or float64), seeded per shape.
"""
from __future__ import annotations

import argparse

import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import inputs

TILES = (16, 32, 64)
K = 64


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def sweep(sizes, reps: int, rounds: int, dtype=torch.float32):
    rows = []
    one = torch.ones((), device="cuda", dtype=dtype)
    for m in sizes:
        for n in sizes:
            C = inputs.normal_clipped(m, n, seed=m * 31 + n, dtype=dtype).cuda()
            D = torch.empty_like(C)
            gC = torch.empty_like(C)
            times = {t: (float("inf"),) * 3 for t in TILES}
            # the tiles take turns, round after round, and each keeps its best round: slow
            # drift of the clocks then favours no tile
            for _ in range(rounds):
                for tile in TILES:
                    wf.set_tile(tile)
                    try:
                        ck = None

                        def fwd():
                            nonlocal ck
                            _, _, ck = wf.forward(C, D=D, ckpt_k=K)

                        def adj():
                            wf.select(C, ckpt=ck, ckpt_k=K)
                            wf.reverse(m, n, dtype=dtype, g_score=one, g_C=gC)

                        t_f = _time(fwd, reps)
                        t_s = _time(lambda: wf.select(C, ckpt=ck, ckpt_k=K), reps)
                        t_r = _time(adj, reps)
                    finally:
                        wf.set_tile(0)
                    wf.last_async_error()
                    times[tile] = tuple(min(a, b) for a, b in zip(times[tile], (t_f, t_s, t_r)))
            best_f = min(TILES, key=lambda t: times[t][0])
            best_r = min(TILES, key=lambda t: times[t][2])
            rows.append((m, n, times, best_f, best_r))
            cells = " | ".join(f"G={t}: {times[t][0]:.3f} {times[t][1]:.3f} {times[t][2]:.3f}" for t in TILES)
            print(f"{m:6d} {n:6d} | {cells} | best forward G={best_f}, reverse G={best_r}", flush=True)
    return rows


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--sizes", default="256,1024,4096,16384")
    p.add_argument("--reps", type=int, default=10)
    p.add_argument("--rounds", type=int, default=3)
    p.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    args = p.parse_args()
    sizes = [int(x) for x in args.sizes.split(",")]
    print("m n | per tile G: forward, selection, selection + reverse [ms] | fastest tiles", flush=True)
    sweep(sizes, args.reps, args.rounds, torch.float64 if args.dtype == "f64" else torch.float32)


if __name__ == "__main__":
    main()
