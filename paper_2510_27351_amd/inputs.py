"""Seeded synthetic workloads (shared by the tests, the benchmark and the smoke check).

This module only draws random numbers; it holds none of the recurrence's arithmetic.  All
draws use a CPU ``torch.Generator`` so that the oracle and the device see identical bits;
the caller moves the tensors to the GPU.  The paper has no dataset for this path, so these
recipes stand in for one; the shapes and distributions are the five workload
configurations the library is measured on.
"""
from __future__ import annotations

import torch


def _gen(seed: int) -> torch.Generator:
    return torch.Generator().manual_seed(seed)


def single_256_f64() -> torch.Tensor:
    """256 x 256 FP64, i.i.d. uniform [0,1), seed 0."""
    return torch.rand(256, 256, dtype=torch.float64, generator=_gen(0))


def single_4096_f32() -> torch.Tensor:
    """4096 x 4096 FP32, i.i.d. uniform [0,1), seed 1."""
    return torch.rand(4096, 4096, dtype=torch.float32, generator=_gen(1))


def single_16384_f32(n: int = 16384) -> torch.Tensor:
    """n x n FP32 (default 16384: 1 GiB), i.i.d. normal(0,1) clipped to [-4, 4], seed 2."""
    return torch.randn(n, n, dtype=torch.float32, generator=_gen(2)).clamp_(-4.0, 4.0)


def ragged_batch_shapes(batch: int = 512, lo: int = 64, hi: int = 2048, seed: int = 3):
    """Shapes of the ragged batch: m then n, each uniform in [lo, hi], from one generator."""
    g = _gen(seed)
    m = torch.randint(lo, hi + 1, (batch,), generator=g)
    n = torch.randint(lo, hi + 1, (batch,), generator=g)
    return g, [int(x) for x in m], [int(x) for x in n]


def ragged_batch_f32(batch: int = 512, lo: int = 64, hi: int = 2048, seed: int = 3):
    """Ragged batch: 512 instances, m and n uniform in [64, 2048] (seed 3), then every
    instance's values uniform [0,1) in order from the same generator."""
    g, ms, ns = ragged_batch_shapes(batch, lo, hi, seed)
    mats = [torch.rand(m, n, dtype=torch.float32, generator=g) for m, n in zip(ms, ns)]
    return ms, ns, mats


def batch_2048_f32(batch: int = 64, size: int = 2048, seed: int = 4):
    """64 instances of 2048 x 2048 FP32 uniform [0,1) (seed 4); returns the tensor and the
    generator, continued, for the finite-difference cell draw."""
    g = _gen(seed)
    return torch.rand(batch, size, size, dtype=torch.float32, generator=g), g


def uniform(m: int, n: int, seed: int, dtype=torch.float32, lo: float = 0.0, hi: float = 1.0) -> torch.Tensor:
    return torch.rand(m, n, dtype=dtype, generator=_gen(seed)) * (hi - lo) + lo


def normal_clipped(m: int, n: int, seed: int, dtype=torch.float32) -> torch.Tensor:
    return torch.randn(m, n, dtype=dtype, generator=_gen(seed)).clamp_(-4.0, 4.0)


def integers(m: int, n: int, seed: int, lo: int = 0, hi: int = 1000) -> torch.Tensor:
    return torch.randint(lo, hi + 1, (m, n), dtype=torch.int32, generator=_gen(seed))


def tridiagonal_dd(N: int, seed: int, margin: float = 1.0):
    """A diagonally dominant tridiagonal system of size N as float64 diagonals (a, b, c) and
    right-hand side d: off-diagonals uniform [-1, 1), |b[i]| = |a[i]| + |c[i]| + margin +
    uniform [0, 1) with a random sign, d uniform [-1, 1); a[0] and c[N-1] (outside the
    matrix) are 0."""
    g = _gen(seed)
    a = torch.rand(N, dtype=torch.float64, generator=g) * 2 - 1
    c = torch.rand(N, dtype=torch.float64, generator=g) * 2 - 1
    a[0] = 0.0
    c[N - 1] = 0.0
    sign = torch.where(torch.rand(N, dtype=torch.float64, generator=g) < 0.5, -1.0, 1.0)
    b = sign * (a.abs() + c.abs() + margin + torch.rand(N, dtype=torch.float64, generator=g))
    d = torch.rand(N, dtype=torch.float64, generator=g) * 2 - 1
    return a, b, c, d
