"""Times the tridiagonal partition solver over system sizes, sub-system sizes and recursion depths.

    python -m paper_2510_27351_amd.tri_sweep [--sizes paper|N1,N2,..] [--ms 4,8,16,..]
        [--rs 0,1,2,3,4] [--reps 10] [--rounds 3] [--dtype f64|f32] [--max-deep 131072]

The paper finds the fastest sub-system size m for each of its system sizes by timing a range
of m (its Table I), and the fastest number of recursive steps R likewise (its Table II), then
fits a 1-NN rule on N to each.  This script does the same on MI355X, for the device-only
solver: for each N it times every (m, R) pair with the recursive steps' sizes m_1 = m when
R = 1, m_1 = 10 when R >= 2 (the paper fixes m_1 = 10), and m_l = m for l >= 2, and reports
the fastest pair.  A configuration whose deepest interface system exceeds --max-deep rows is
not timed: its one-lane Thomas solve alone would take longer than the whole solve of the
configurations that cut it further.  Each time is the best of `rounds` rounds of `reps`
back-to-back solves (the configurations take turns within a round), timed with HIP events on
the launch stream.  Systems are diagonally dominant (inputs.tridiagonal_dd), seeded per N.

The rows "N m R" are the training set of the library's predictor (tri_predict); after a
change to the kernels, sweep again and replace the table in tri.hip and its copy in
tests/golden/mi355x_tri_table.txt.
"""
from __future__ import annotations

import argparse

import torch

from paper_2510_27351_amd import inputs, tri

# the 37 system sizes of the paper's Table I
PAPER_SIZES = [
    100, 200, 400, 500, 800, 1000, 2000, 4000, 4500, 5000, 8000, 10000, 20000, 25000, 30000, 40000, 50000,
    60000, 70000, 75000, 80000, 100000, 200000, 400000, 500000, 800000, 1000000, 2000000, 4000000, 5000000,
    8000000, 10000000, 20000000, 40000000, 50000000, 80000000, 100000000,
]


def levels(m: int, R: int):
    """[m, m_1 .. m_R] of the sweep."""
    if R == 0:
        return [m]
    return [m, m if R == 1 else 10] + [m] * (R - 1)


def deepest(N: int, ms) -> int:
    n = N
    for m in ms:
        n = 2 * tri.subsystems(n, m)
    return n


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


def sweep(sizes, ms_list, rs, reps, rounds, dtype, max_deep):
    rows = []
    for N in sizes:
        a, b, c, d = (v.to(dtype).cuda() for v in inputs.tridiagonal_dd(N, seed=N % 100003))
        x = torch.empty_like(a)
        cfgs = []
        for m in ms_list:
            if m > N:
                continue
            for R in rs:
                ms = levels(m, R)
                if deepest(N, ms) > max_deep:
                    continue
                cfgs.append((m, R, tri.Plan(1, N, dtype, m=m, R=R, ms=ms[1:])))
        best = {(m, R): float("inf") for m, R, _ in cfgs}
        for _ in range(rounds):
            for m, R, plan in cfgs:
                t = _time(lambda: plan.solve(a, b, c, d, x), reps)
                best[(m, R)] = min(best[(m, R)], t)
        del cfgs
        (bm, bR), bt = min(best.items(), key=lambda kv: kv[1])
        rows.append((N, bm, bR, bt, best))
        per_r = {}
        for (m, R), t in best.items():
            if t < per_r.get(R, (float("inf"),))[0]:
                per_r[R] = (t, m)
        detail = " ".join(f"R={R}:{per_r[R][0]:.4f}ms@m={per_r[R][1]}" for R in sorted(per_r))
        gbs = N * (9 * a.element_size()) / (bt * 1e-3) / 1e9
        print(f"{N:10d} best m={bm:4d} R={bR} {bt:.4f} ms ({N / (bt * 1e-3):.3e} unknowns/s, {gbs:.0f} GB/s "
              f"at 9 elements per unknown) | {detail}", flush=True)
        del a, b, c, d, x
        torch.cuda.empty_cache()
    return rows


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--sizes", default="paper")
    p.add_argument("--ms", default="4,8,16,20,32,40,64,128")
    p.add_argument("--rs", default="0,1,2,3,4")
    p.add_argument("--reps", type=int, default=10)
    p.add_argument("--rounds", type=int, default=3)
    p.add_argument("--dtype", choices=("f32", "f64"), default="f64")
    p.add_argument("--max-deep", type=int, default=131072)
    args = p.parse_args()
    sizes = PAPER_SIZES if args.sizes == "paper" else [int(float(v)) for v in args.sizes.split(",")]
    ms_list = [int(v) for v in args.ms.split(",")]
    rs = [int(v) for v in args.rs.split(",")]
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    print(f"N | fastest (m, R), time | best time per R [{args.dtype}]", flush=True)
    sweep(sizes, ms_list, rs, args.reps, args.rounds, dtype, args.max_deep)


if __name__ == "__main__":
    main()
