"""Parity of the tridiagonal partition solver on the GPU (through the C ABI).

Every stage is compared element by element with the oracle (oracle/tridiag.py and its C
twin, which the CPU tests hold to the Python stages bit for bit):
  - Stage 1's interface systems, Stage 3's solutions and the Thomas solve are bitwise equal
    to the oracle's in float64 and in float32 (the kernels take the same operations in the
    same order; IEEE division, no contraction);
  - the full recursive solve is bitwise equal to the oracle's partition method, and within a
    conditioning bound of the plain definition x = A^-1 d (the float64 Thomas solve).
Bound: the systems are diagonally dominant by a margin of at least 1, so ||A^-1||_inf <= 1,
and the rows of |A| sum to at most 6; a backward-stable elimination (the interface systems
stay diagonally dominant at every level) then leaves a forward error of a small multiple of
6 u ||x||_inf per level; the tests allow 64 * 6 * (R + 2) * u * ||x||_inf.
"""
import numpy as np
import pytest
import torch

from oracle import tridiag
from paper_2510_27351_amd import inputs
from paper_2510_27351_amd import tri

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PREC = {torch.float64: "f64", torch.float32: "f32"}


def system(N, seed, batch=None, dtype=torch.float64):
    """(a, b, c, d) as CPU tensors, (N,) or (batch, N); float32 systems are the float64 ones
    rounded once."""
    if batch is None:
        return tuple(v.to(dtype) for v in inputs.tridiagonal_dd(N, seed))
    parts = [inputs.tridiagonal_dd(N, seed + i) for i in range(batch)]
    return tuple(torch.stack([p[k] for p in parts]).to(dtype) for k in range(4))


def dev(*vs):
    return tuple(v.to(DEV) for v in vs)


def rows(v):
    """The systems of a (N,) or (batch, N) tensor as numpy rows."""
    v = v.cpu().numpy()
    return [v] if v.ndim == 1 else list(v)


def bound(x_ref, R, dtype):
    u = np.finfo(np.float64 if dtype == torch.float64 else np.float32).eps / 2
    return 64 * 6 * (R + 2) * u * max(1.0, float(np.max(np.abs(x_ref))))


STAGE_CASES = [  # (N, m): remainders of every kind, m larger than N, the smallest sizes
    (2, 2), (3, 2), (5, 2), (9, 4), (10, 4), (64, 8), (65, 8), (66, 8), (1000, 32), (1001, 32), (1023, 32),
    (4097, 64), (3000, 37), (7, 100), (20000, 300), (50000, 16),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,m", STAGE_CASES)
def test_stage1_bitwise(N, m, dtype):
    a, b, c, d = system(N, seed=N + m, dtype=dtype)
    got = tri.stage1(*dev(a, b, c, d), m)
    want = tridiag.c_interface_system(a.numpy(), b.numpy(), c.numpy(), d.numpy(), m, PREC[dtype])
    for name, g, w in zip("ABCD", got, want):
        assert np.array_equal(g.cpu().numpy(), w), (name, N, m)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,m", STAGE_CASES)
def test_stage3_bitwise(N, m, dtype):
    a, b, c, d = system(N, seed=7 * N + m, dtype=dtype)
    an, bn, cn, dn = (v.numpy() for v in (a, b, c, d))
    A, B, C, D = tridiag.c_interface_system(an, bn, cn, dn, m, PREC[dtype])
    z = tridiag.c_thomas(A, B, C, D, PREC[dtype])
    got = tri.stage3(*dev(a, b, c, d), torch.from_numpy(z).to(DEV), m)
    want = tridiag.c_back_solve(an, bn, cn, dn, m, z, PREC[dtype])
    assert np.array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_stage_kernels_batched(dtype):
    """Several systems per launch, a workgroup never spans two of them."""
    N, m, batch = 1037, 24, 5
    a, b, c, d = system(N, seed=11, batch=batch, dtype=dtype)
    A, B, C, D = tri.stage1(*dev(a, b, c, d), m)
    zs = []
    for k, (an, bn, cn, dn) in enumerate(zip(*(rows(v) for v in (a, b, c, d)))):
        want = tridiag.c_interface_system(an, bn, cn, dn, m, PREC[dtype])
        for g, w in zip((A, B, C, D), want):
            assert np.array_equal(g[k].cpu().numpy(), w)
        zs.append(tridiag.c_thomas(*want, PREC[dtype]))
    z = torch.from_numpy(np.stack(zs)).to(DEV)
    x = tri.stage3(*dev(a, b, c, d), z, m)
    for k, (an, bn, cn, dn) in enumerate(zip(*(rows(v) for v in (a, b, c, d)))):
        assert np.array_equal(x[k].cpu().numpy(), tridiag.c_back_solve(an, bn, cn, dn, m, zs[k], PREC[dtype]))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 2, 7, 1023, 1024, 1025, 2048, 2049, 10000])
def test_thomas_bitwise(n, dtype):
    a, b, c, d = system(n, seed=3 * n + 1, dtype=dtype)
    got = tri.thomas(*dev(a, b, c, d))
    want = tridiag.c_thomas(a.numpy(), b.numpy(), c.numpy(), d.numpy(), PREC[dtype])
    assert np.array_equal(got.cpu().numpy(), want)


def test_thomas_batched():
    a, b, c, d = system(3001, seed=5, batch=4)
    x = tri.thomas(*dev(a, b, c, d))
    for k, sysk in enumerate(zip(*(rows(v) for v in (a, b, c, d)))):
        assert np.array_equal(x[k].cpu().numpy(), tridiag.c_thomas(*sysk))


SOLVE_CASES = [  # (N, [m, m_1, .., m_R])
    (1, None), (2, [2]), (3, [2]), (100, [4]), (4500, [4, 10]), (25000, [8, 10, 4]), (100001, [32, 10, 32]),
    (200000, [64]), (1000000, [32, 10, 32, 32]), (777777, [40, 10, 16, 8, 4]), (300000, [20, 5, 5, 5, 5, 5, 5]),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,ms", SOLVE_CASES)
def test_solve_bitwise_and_bound(N, ms, dtype):
    a, b, c, d = system(N, seed=N % 1000 + 17, dtype=dtype)
    if ms is None:
        plan = tri.Plan(1, N, dtype)
    else:
        plan = tri.Plan(1, N, dtype, m=ms[0], R=len(ms) - 1, ms=ms[1:])
        assert [plan.m] + plan.ms == ms
    x = plan.solve(*dev(a, b, c, d)).cpu().numpy()
    an, bn, cn, dn = (v.numpy() for v in (a, b, c, d))
    want = tridiag.c_partition_solve(an, bn, cn, dn, [] if N == 1 else [plan.m] + plan.ms, PREC[dtype])
    assert np.array_equal(x, want)
    ref = tridiag.c_thomas(an, bn, cn, dn, "f64")
    err = float(np.max(np.abs(x.astype(np.float64) - ref)))
    print(f"N={N} ms={ms} {PREC[dtype]}: max |x - A^-1 d| = {err:.3e}")
    assert err <= bound(ref, max(plan.R, 0), dtype)


def test_solve_batched_and_levels():
    N, batch, ms = 50003, 3, [16, 10, 8]
    a, b, c, d = system(N, seed=23, batch=batch)
    plan = tri.Plan(batch, N, torch.float64, m=ms[0], R=2, ms=ms[1:])
    x = plan.solve(*dev(a, b, c, d))
    for k, sysk in enumerate(zip(*(rows(v) for v in (a, b, c, d)))):
        assert np.array_equal(x[k].cpu().numpy(), tridiag.c_partition_solve(*sysk, ms))
        # the interface system of every level
        level = tuple(sysk)
        for lv in range(1, plan.R + 2):
            level = tridiag.c_interface_system(*level, ([plan.m] + plan.ms)[lv - 1])
            got = plan.level(lv)
            for g, w in zip(got, level):
                assert np.array_equal(g[k].cpu().numpy(), w)


def test_solve_repeated_calls_and_manufactured_solution():
    """Two solves with one plan give the same bits; a manufactured solution comes back within
    the bound."""
    N = 300001
    a, b, c, _ = system(N, seed=31)
    xt = torch.rand(N, dtype=torch.float64, generator=torch.Generator().manual_seed(32)) * 2 - 1
    an, bn, cn = (v.numpy() for v in (a, b, c))
    xn = xt.numpy()
    dn = bn * xn
    dn[1:] += an[1:] * xn[:-1]
    dn[:-1] += cn[:-1] * xn[1:]
    plan = tri.Plan(1, N, torch.float64)
    ad, bd, cd, dd = dev(a, b, c, torch.from_numpy(dn))
    x1 = plan.solve(ad, bd, cd, dd).cpu()
    x2 = plan.solve(ad, bd, cd, dd).cpu()
    assert torch.equal(x1, x2)
    assert float((x1 - xt).abs().max()) <= bound(xn, plan.R, torch.float64)


def test_full_size_bitwise():
    """10^8 unknowns in float64 (the paper's largest system) with the predicted plan: every
    element equal to the C oracle's partition method."""
    N = 100_000_000
    a, b, c, d = system(N, seed=8)
    plan = tri.Plan(1, N, torch.float64)
    print(f"N=1e8: m={plan.m} R={plan.R} ms={plan.ms} sizes={plan.sizes}", flush=True)
    x = plan.solve(*dev(a, b, c, d)).cpu().numpy()
    want = tridiag.c_partition_solve(a.numpy(), b.numpy(), c.numpy(), d.numpy(), [plan.m] + plan.ms)
    assert np.array_equal(x, want)


def test_plan_rejects_bad_sizes():
    with pytest.raises(tri._lib.WfError):
        tri.Plan(1, 100, torch.float64, m=1, R=0)
    with pytest.raises(tri._lib.WfError):
        tri.Plan(1, 100, torch.float64, m=4, R=2, ms=[1, 4])
    with pytest.raises(tri._lib.WfError):
        tri.Plan(1, 100, torch.float64, m=100000, R=0)
    with pytest.raises(tri._lib.WfError):
        tri.Plan(0, 100, torch.float64, m=4, R=0)
