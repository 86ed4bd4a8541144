"""Parity of the smooth (soft-min) sweeps on the GPU (wf_soft_forward / wf_soft_backward).

The device evaluates its exponentials and logarithms with its own base-2 functions, so the
comparison with the float64 oracle (oracle/softmin.c, pinned by path enumeration) is within
rounding, not bitwise.  Bars:
  - float64: every table element within 1e-10 relative of the oracle (a few units in the
    last place per cell, accumulated along paths of at most m+n-1 cells).  The gradient
    multiplies the weights along paths, and their exponents telescope, so its relative error
    is the absolute rounding drift of the forward table over a path divided by gamma; each
    side's drift is a sum of L = m+n-1 roundings of at most a few u max|D| (u = 2^-53), which
    the probabilistic rounding-error bound of Higham and Mary (SISC 2019) holds to
    lambda sqrt(L) u max|D| with overwhelming probability.  Bar: max(1e-10,
    12 sqrt(L) u max|D*| / gamma) (two sides, lambda times rounding count 6).  At 70000 x 6
    this is what separates two correct evaluations: the oracle's own adjoint differs by
    5e-10 from that of the exactly rounded table (long double evaluation);
  - float32: error <= 1e-4 against the float64 oracle (the library's float32 bar), stated
    per result.  Each soft minimum lies up to gamma log 3 below the plain minimum, so the
    table crosses zero even for positive inputs and a relative error is ill-posed at the
    cells near zero: the table is held normwise (max |dD| / max |D*| <= 1e-4) and
    elementwise on the cells with |D*| >= 1e-2 max |D*|.  The gradient's weights are
    2^((V - D) log2e / gamma) with V and D float32 values of the table's magnitude.  Along a
    path the exponents telescope, so what is left is the float32 table's own drift at the
    path's ends and one rounding of V = D - C per cell (u max|D|, u = 2^-24): the same
    sqrt(L) law as in float64, with u = 2^-24.  Bar: max(1e-4, 12 sqrt(L) u max|D*| / gamma),
    elementwise over entries >= 1e-3 of the largest and normwise (entries span many orders
    of magnitude).  At 300 x 2500 (tables to 1.2e3) the measured elementwise error is 2e-3,
    above the per-weight error 8 u max|D*| / gamma that the bar used to be, which holds only
    for short paths.  Tall cases, whose tables grow to 10^4, run in float64;
  - the float64 gradient against central finite differences of the device's own float64
    forward (h = 1e-3, 32 cells: 16 on the heaviest path cells, 16 uniform), which the smooth
    recurrence makes exact up to O(h^2).
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(got, want):
    got = got.astype(np.float64)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300)))


def f64_grad_bar(m, n, Dmax, gamma):
    return max(1e-10, 12 * np.sqrt(m + n - 1) * 2.0 ** -53 * Dmax / gamma)


def f32_grad_bar(m, n, Dmax, gamma):
    return max(1e-4, 12 * np.sqrt(m + n - 1) * 2.0 ** -24 * Dmax / gamma)


def grad_err(got, want, cut=1e-3):
    """(elementwise max rel err over entries >= cut * max, normwise err / max)."""
    got = got.astype(np.float64)
    big = np.abs(want) >= cut * np.max(np.abs(want))
    el = float(np.max(np.abs(got - want)[big] / np.abs(want[big])))
    nw = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    return el, nw


SHAPES = [(1, 1), (1, 37), (53, 1), (200, 1), (129, 3), (64, 64), (65, 63), (130, 257), (300, 200), (257, 1031),
          (300, 2500)]


@pytest.mark.parametrize("gamma", [0.1, 1.0])
@pytest.mark.parametrize("shape", SHAPES)
def test_forward_f64(shape, gamma, oracle_mod):
    C = inputs.uniform(*shape, seed=sum(shape), dtype=torch.float64)
    D, score = wf.soft_forward(C.to(DEV), gamma)
    want = oracle_mod.soft_forward(C.numpy(), gamma)
    err = rel(D.cpu().numpy(), want)
    print(f"soft forward f64 {shape} gamma={gamma}: max rel err {err:.2e}")
    assert err <= 1e-10
    assert float(score) == float(D[-1, -1])


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_f32(shape, oracle_mod):
    gamma = 0.5
    C = inputs.uniform(*shape, seed=3 * sum(shape), dtype=torch.float32)
    D, score = wf.soft_forward(C.to(DEV), gamma)
    want = oracle_mod.soft_forward(C.numpy().astype(np.float64), gamma)
    el, nw = grad_err(D.cpu().numpy(), want, cut=1e-2)
    print(f"soft forward f32 {shape}: normwise {nw:.2e}, elementwise (|D| >= 1e-2 max) {el:.2e}, "
          f"elementwise over all cells {rel(D.cpu().numpy(), want):.2e} vs f64 oracle")
    assert nw <= 1e-4 and el <= 1e-4


@pytest.mark.parametrize("gamma", [0.1, 1.0])
@pytest.mark.parametrize("shape", SHAPES)
def test_backward_f64(shape, gamma, oracle_mod):
    C = inputs.uniform(*shape, seed=5 + sum(shape), dtype=torch.float64)
    gD = inputs.uniform(*shape, seed=6 + sum(shape), dtype=torch.float64, lo=-1.0, hi=1.0)
    Cd = C.to(DEV)
    D, _ = wf.soft_forward(Cd, gamma)
    g = wf.soft_backward(Cd, D, gamma, g_score=torch.tensor(0.75, dtype=torch.float64), g_D=gD.to(DEV))
    Dn = oracle_mod.soft_forward(C.numpy(), gamma)
    want = oracle_mod.soft_backward(C.numpy(), Dn, gamma, gD=gD.numpy(), gscore=0.75)
    err = float(np.max(np.abs(g.cpu().numpy() - want)) / max(1e-300, np.max(np.abs(want))))
    bar = f64_grad_bar(*shape, float(np.max(np.abs(Dn))), gamma)
    print(f"soft adjoint f64 {shape} gamma={gamma}: max err / max|g| {err:.2e} (bar {bar:.2e})")
    assert err <= bar


@pytest.mark.parametrize("shape", SHAPES[2:])
def test_backward_f32(shape, oracle_mod):
    gamma = 0.5
    C = inputs.uniform(*shape, seed=9 + sum(shape), dtype=torch.float32)
    Cd = C.to(DEV)
    D, _ = wf.soft_forward(Cd, gamma)
    g = wf.soft_backward(Cd, D, gamma, g_score=torch.tensor(1.0))
    C64 = C.numpy().astype(np.float64)
    want = oracle_mod.soft_backward(C64, oracle_mod.soft_forward(C64, gamma), gamma, gscore=1.0)
    el, nw = grad_err(g.cpu().numpy(), want)
    Dmax = float(np.max(np.abs(oracle_mod.soft_forward(C64, gamma))))
    bar = f32_grad_bar(*shape, Dmax, gamma)
    print(f"soft adjoint f32 {shape}: elementwise {el:.2e}, normwise {nw:.2e} vs f64 oracle (bar {bar:.2e})")
    assert el <= bar and nw <= bar


@pytest.mark.parametrize("shape", [(65, 63), (257, 1031), (1100, 3000)])
def test_backward_f32_with_upstream(shape, oracle_mod):
    """float32 adjoint with an upstream gD (its own code path: gD read along each row).  gD in
    [0, 1), so every term of every sum is non-negative and the elementwise bar is
    well-posed; 1100 x 3000 has 18 bands and rows longer than the handoff ring."""
    gamma = 0.5
    C = inputs.uniform(*shape, seed=13 + sum(shape), dtype=torch.float32)
    gD = inputs.uniform(*shape, seed=14 + sum(shape), dtype=torch.float32)
    Cd = C.to(DEV)
    D, _ = wf.soft_forward(Cd, gamma)
    g = wf.soft_backward(Cd, D, gamma, g_score=torch.tensor(0.5), g_D=gD.to(DEV))
    C64 = C.numpy().astype(np.float64)
    Dn = oracle_mod.soft_forward(C64, gamma)
    want = oracle_mod.soft_backward(C64, Dn, gamma, gD=gD.numpy().astype(np.float64), gscore=0.5)
    el, nw = grad_err(g.cpu().numpy(), want)
    bar = f32_grad_bar(*shape, float(np.max(np.abs(Dn))), gamma)
    print(f"soft adjoint f32 with gD {shape}: elementwise {el:.2e}, normwise {nw:.2e} vs f64 oracle (bar {bar:.2e})")
    assert el <= bar and nw <= bar


@pytest.mark.parametrize("gamma", [0.01, 10.0])
def test_temperature_extremes(gamma, oracle_mod):
    """gamma = 0.01 (weights of 2^(-100 x) for a unit gap: nearly the min-plus sweep, most
    exponentials underflow to 0) and gamma = 10 (nearly uniform weights), float64, forward
    and adjoint with an upstream gD, across three bands."""
    shape = (130, 257)
    C = inputs.uniform(*shape, seed=61, dtype=torch.float64)
    gD = inputs.uniform(*shape, seed=62, dtype=torch.float64, lo=-1.0, hi=1.0)
    Cd = C.to(DEV)
    D, score = wf.soft_forward(Cd, gamma)
    Dn = oracle_mod.soft_forward(C.numpy(), gamma)
    ferr = rel(D.cpu().numpy(), Dn)
    g = wf.soft_backward(Cd, D, gamma, g_score=torch.tensor(0.5, dtype=torch.float64), g_D=gD.to(DEV))
    want = oracle_mod.soft_backward(C.numpy(), Dn, gamma, gD=gD.numpy(), gscore=0.5)
    gerr = float(np.max(np.abs(g.cpu().numpy() - want)) / max(1e-300, np.max(np.abs(want))))
    bar = f64_grad_bar(*shape, float(np.max(np.abs(Dn))), gamma)
    print(f"soft gamma={gamma}: forward max rel err {ferr:.2e}, adjoint {gerr:.2e} (bar {bar:.2e})")
    assert ferr <= 1e-10 and gerr <= bar


def test_leading_dimensions(oracle_mod):
    m, n, gamma = 150, 90, 0.3
    C = inputs.uniform(m, n, seed=41, dtype=torch.float64)
    big = torch.full((m, n + 13), 7.0, dtype=torch.float64, device=DEV)
    big[:, :n] = C.to(DEV)
    Cv = big[:, :n]
    Dbig = torch.full((m, n + 5), float("nan"), dtype=torch.float64, device=DEV)
    D, _ = wf.soft_forward(Cv, gamma, D=Dbig[:, :n])
    assert torch.isnan(Dbig[:, n:]).all()
    want = oracle_mod.soft_forward(C.numpy(), gamma)
    assert rel(D.cpu().numpy(), want) <= 1e-10
    gbig = torch.full((m, n + 3), float("nan"), dtype=torch.float64, device=DEV)
    g = wf.soft_backward(Cv, D, gamma, g_score=torch.tensor(1.0, dtype=torch.float64), g_C=gbig[:, :n])
    assert torch.isnan(gbig[:, n:]).all()
    wantg = oracle_mod.soft_backward(C.numpy(), want, gamma, gscore=1.0)
    assert float(np.max(np.abs(g.cpu().numpy() - wantg))) <= 1e-10


def test_more_bands_than_workgroups(oracle_mod):
    """70000 rows: 1094 bands, more than the 4 workgroups per CU of the launch, so workgroups
    claim second bands; float64 (the table grows to ~10^4, beyond float32's weight accuracy),
    and the float32 forward normwise."""
    m, n, gamma = 70000, 6, 0.5
    C = inputs.uniform(m, n, seed=43, dtype=torch.float64)
    Cd = C.to(DEV)
    D, _ = wf.soft_forward(Cd, gamma)
    Dn = oracle_mod.soft_forward(C.numpy(), gamma)
    assert rel(D.cpu().numpy(), Dn) <= 1e-10
    g = wf.soft_backward(Cd, D, gamma, g_score=torch.tensor(1.0, dtype=torch.float64))
    want = oracle_mod.soft_backward(C.numpy(), Dn, gamma, gscore=1.0)
    err = float(np.max(np.abs(g.cpu().numpy() - want)) / np.max(np.abs(want)))
    D32, _ = wf.soft_forward(Cd.float(), gamma)
    fel, fnw = grad_err(D32.cpu().numpy(), oracle_mod.soft_forward(C.float().numpy().astype(np.float64), gamma),
                        cut=1e-2)
    bar = f64_grad_bar(m, n, float(np.max(np.abs(Dn))), gamma)
    print(f"70000x6: f64 adjoint {err:.2e} (bar {bar:.2e}); f32 forward normwise {fnw:.2e} elementwise {fel:.2e}")
    assert err <= bar and fnw <= 1e-4 and fel <= 1e-4


def test_bench_matrix_full_size(oracle_mod):
    """The bench's 16384 x 16384 soft-min workload (normal(0,1) clipped to [-4, 4], seed 2,
    gamma = 1), in the bench's launch configuration.

    float64: the adjoint of the score against its closed form.  The gradient of the score
    with respect to C[i][j] is the Gibbs probability that a path passes through (i, j),
    exp((score - R[i][j] - Q[i][j] + C[i][j]) / gamma), where R is the forward table and Q
    the same recurrence run from the far corner (the oracle's forward on the matrix reversed
    in both axes).  Two oracle sweeps pin every one of the 2.7e8 gradient entries, relative,
    to the float64 bar of the other adjoint tests.
    float32: the table's top-left 2048 x 2048 block against the float64 oracle (D[i][j]
    depends on C[:i+1, :j+1] only), and properties of the adjoint that hold at any size:
    every entry finite and non-negative (a sum of products of non-negative weights) and the
    last cell exactly g_score.  (The first cell, which every path visits, is 1 in exact
    arithmetic; its float32 value, 0.9992, is printed, not held to a bar: with tables of 4e4
    the float32 bar of the other adjoint tests exceeds 1 at this size.)"""
    m = n = 16384
    gamma = 1.0
    C = inputs.normal_clipped(m, n, seed=2)
    Cd = C.to(DEV)
    D32, s32 = wf.soft_forward(Cd, gamma)
    g32 = wf.soft_backward(Cd, D32, gamma, g_score=torch.tensor(1.0))
    blk = C[:2048, :2048].numpy().astype(np.float64)
    want_blk = oracle_mod.soft_forward(blk, gamma)
    el, nw = grad_err(D32[:2048, :2048].cpu().numpy(), want_blk, cut=1e-2)
    assert bool(torch.isfinite(g32).all()) and float(g32.min()) >= 0.0
    assert float(g32[-1, -1]) == 1.0
    del D32

    C64 = C.numpy().astype(np.float64)
    del C
    R = oracle_mod.soft_forward(C64, gamma)
    Q = oracle_mod.soft_forward(np.ascontiguousarray(C64[::-1, ::-1]), gamma)[::-1, ::-1]
    Dmax = float(max(np.abs(R).max(), np.abs(Q).max()))
    first = float(g32[0, 0])
    del g32
    print(f"soft 16384^2 f32: table block normwise {nw:.2e}, elementwise {el:.2e}; gC[0][0] = {first:.6f}, "
          f"max|D| {Dmax:.3e}")
    assert nw <= 1e-4 and el <= 1e-4

    Cd64 = torch.from_numpy(C64).to(DEV)
    D64, s64 = wf.soft_forward(Cd64, gamma)
    g64 = wf.soft_backward(Cd64, D64, gamma, g_score=torch.tensor(1.0, dtype=torch.float64)).cpu().numpy()
    del D64, Cd64
    score = float(R[-1, -1])
    P = np.exp((score - R - Q + C64) / gamma)
    del R, Q
    big = P >= 1e-200
    rel = float(np.max(np.abs(g64[big] - P[big]) / P[big]))
    tiny = float(np.max(np.abs(g64[~big]))) if (~big).any() else 0.0
    bar = f64_grad_bar(m, n, Dmax, gamma)
    print(f"soft 16384^2 f64 adjoint vs closed form: max rel err {rel:.2e} over {int(big.sum())} entries "
          f"(bar {bar:.2e}); score {float(s64):.6f} vs oracle {score:.6f}")
    assert rel <= bar and tiny <= 1e-190
    assert abs(float(s64) - score) <= 1e-10 * abs(score)


def test_finite_differences_f64():
    """Central differences (h = 1e-3) of the device's float64 score on 32 cells: the 16
    cells of largest gradient and 16 uniform ones (seeded).  The truncation error is about
    h^2/6 times the third derivative, which the soft minimum bounds by a small multiple of
    1/gamma^2 (7e-7 here); rounding adds about eps |score| / h (1e-11)."""
    m, n, gamma, h = 96, 140, 0.5, 1e-3
    C = inputs.uniform(m, n, seed=47, dtype=torch.float64).to(DEV)
    D, _ = wf.soft_forward(C, gamma)
    g = wf.soft_backward(C, D, gamma, g_score=torch.tensor(1.0, dtype=torch.float64)).cpu().numpy()
    flat = np.argsort(-g.ravel())[:16]
    rng = torch.Generator().manual_seed(48)
    uni = torch.randint(0, m * n, (16,), generator=rng).numpy()
    worst = 0.0
    for idx in list(flat) + list(uni):
        i, j = divmod(int(idx), n)
        Cp, Cm = C.clone(), C.clone()
        Cp[i, j] += h
        Cm[i, j] -= h
        fd = (float(wf.soft_forward(Cp, gamma)[1]) - float(wf.soft_forward(Cm, gamma)[1])) / (2 * h)
        worst = max(worst, abs(fd - g[i, j]))
    print(f"soft FD f64: max |FD - adjoint| over 32 cells {worst:.2e}")
    assert worst <= 1e-5


def test_autograd_matches_adjoint():
    m, n, gamma = 80, 70, 0.4
    C = inputs.uniform(m, n, seed=51, dtype=torch.float64).to(DEV).requires_grad_(True)
    D, score = wf.soft_sweep(C, gamma)
    W = inputs.uniform(m, n, seed=52, dtype=torch.float64).to(DEV)
    (2.0 * score + (W * D).sum()).backward()
    D2, _ = wf.soft_forward(C.detach(), gamma)
    want = wf.soft_backward(C.detach(), D2, gamma, g_score=torch.tensor(2.0, dtype=torch.float64), g_D=W)
    assert torch.equal(C.grad, want)


def test_argument_errors():
    C = torch.zeros(4, 4, device=DEV)
    for gamma in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(wf.WfError):
            wf.soft_forward(C, gamma)
    with pytest.raises(wf.WfError):
        wf.soft_forward(torch.zeros(4, 4, dtype=torch.int32, device=DEV), 1.0)
