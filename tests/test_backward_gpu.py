"""Adjoint sweep on the GPU (through the C ABI) against the CPU oracle.

The device recomputes the predecessor selections from C and either the forward table or
the band rows of the checkpoint grid, then runs the reverse sweep.  Bars:
  - float32: bitwise equal to the single-precision oracle's adjoint on the oracle's own
    float32 selection map (the selections match because the forward values match bitwise,
    and both sides sum the routed terms in the order gD, gscore, NW, N, W), and, free of
    that order, within 1e-4 of the float64 adjoint on the same selections with every
    float32/float64 selection flip certified as a near-tie (adjoint_checks.f32_adjoint);
  - float64: bitwise equal to the double oracle;
  - integer-valued inputs and upstream values (heavy ties, exact sums): bitwise equal to the
    oracle in both precisions, whatever the summation order;
  - the score gradient against central finite differences of the double forward.
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import inputs

from adjoint_checks import f32_adjoint

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def oracle_grad(oracle_mod, C, gD, gscore, precision):
    _, sel = oracle_mod.forward(C.numpy(), precision, want_sel=True)
    g = oracle_mod.backward(sel, None if gD is None else gD.numpy(), gscore, precision)
    return torch.from_numpy(g)


def gpu_grad(C, gD, gscore, source, tile=None, ckpt_k=64):
    if tile is not None:
        wf.set_tile(tile)
    try:
        Cd = C.to(DEV)
        gDd = None if gD is None else gD.to(DEV)
        gs = torch.tensor(gscore, dtype=C.dtype, device=DEV)
        if source == "table":
            D, _, _ = wf.forward(Cd)
            gC = wf.backward(Cd, g_score=gs, g_D=gDd, D=D)
        else:
            _, _, ck = wf.forward(Cd, table=False, ckpt_k=ckpt_k)
            gC = wf.backward(Cd, g_score=gs, g_D=gDd, ckpt=ck, ckpt_k=ckpt_k)
        wf.last_async_error()
        return gC.cpu()
    finally:
        if tile is not None:
            wf.set_tile(0)


SHAPES = [(1, 1), (1, 7), (7, 1), (1, 300), (300, 1), (2, 2), (63, 64), (64, 64), (65, 65), (64, 1000),
          (130, 257), (200, 200), (257, 513), (129, 16), (16, 129)]


@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("shape", SHAPES)
def test_f32_adjoint_bitwise(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.uniform(m, n, seed=m * 1000 + n + 5)
    gD = inputs.normal_clipped(m, n, seed=m + n)
    got = gpu_grad(C, gD, 0.75, "table", tile)
    f32_adjoint(oracle_mod, C, gD, 0.75, got, f"{m}x{n} tile {tile}")


@pytest.mark.parametrize("shape", [(1, 1), (70, 33), (64, 64), (190, 300), (300, 190)])
def test_f32_adjoint_from_checkpoints(oracle_mod, shape):
    m, n = shape
    C = inputs.normal_clipped(m, n, seed=17)
    gD = inputs.uniform(m, n, seed=18, lo=-1.0, hi=1.0)
    for k in (1, 64, 100):
        got = gpu_grad(C, gD, -2.0, "ckpt", ckpt_k=k)
        f32_adjoint(oracle_mod, C, gD, -2.0, got, f"{m}x{n} ckpt_k={k}")


@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("shape", [(1, 1), (5, 300), (100, 70), (200, 333)])
def test_f64_adjoint_bitwise(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.uniform(m, n, seed=23, dtype=torch.float64)
    gD = inputs.uniform(m, n, seed=24, dtype=torch.float64, lo=-1.0, hi=1.0)
    for source in ("table", "ckpt"):
        got = gpu_grad(C, gD, 1.5, source, tile)
        ref = oracle_grad(oracle_mod, C, gD, 1.5, "f64")
        assert torch.equal(got, ref), source


@pytest.mark.parametrize("shape", [(1, 1), (64, 65), (129, 300), (300, 129)])
def test_score_gradient_is_the_optimal_path(oracle_mod, shape):
    """With g_D = 0 and g_score = 1 the gradient is the 0/1 indicator of the selected
    monotone path from (0,0) to (m-1,n-1): m+n-1 ... down to max(m,n) cells, each step
    to a neighbour."""
    m, n = shape
    C = inputs.uniform(m, n, seed=31)
    got = gpu_grad(C, None, 1.0, "ckpt")
    f32_adjoint(oracle_mod, C, None, 1.0, got, f"{m}x{n} score path")
    assert set(torch.unique(got).tolist()) <= {0.0, 1.0}
    assert max(m, n) <= int(got.sum()) <= m + n - 1
    assert got[0, 0] == 1 and got[-1, -1] == 1


def test_score_gradient_central_differences():
    """d score / d C[i][j] against central differences of the double forward on the device,
    at cells on and off the path (no selection flips within the step for these draws)."""
    m, n = 96, 140
    C = inputs.uniform(m, n, seed=41, dtype=torch.float64).to(DEV)
    _, _, ck = wf.forward(C, table=False, ckpt_k=64)
    g = wf.backward(C, g_score=torch.tensor(1.0, dtype=torch.float64, device=DEV), ckpt=ck, ckpt_k=64)
    on = torch.nonzero(g > 0)[::17]
    off = torch.nonzero(g == 0)[::997]
    h = 1e-7
    for i, j in torch.cat([on, off]).tolist():
        Cp, Cm = C.clone(), C.clone()
        Cp[i, j] += h
        Cm[i, j] -= h
        sp = wf.forward(Cp, table=False)[1].item()
        sm = wf.forward(Cm, table=False)[1].item()
        fd = (sp - sm) / (2 * h)
        assert abs(fd - g[i, j].item()) < 1e-6, (i, j, fd, g[i, j].item())
    wf.last_async_error()


def test_autograd_matches_entry_points(oracle_mod):
    m, n = 150, 210
    C = inputs.uniform(m, n, seed=51).to(DEV).requires_grad_(True)
    score = wf.sweep(C)
    score.backward()
    f32_adjoint(oracle_mod, C.detach().cpu(), None, 1.0, C.grad.cpu(), "autograd score")

    C2 = C.detach().clone().requires_grad_(True)
    gD = inputs.normal_clipped(m, n, seed=52).to(DEV)
    D, s = wf.sweep(C2, table=True)
    ((D * gD).sum() + 3.0 * s).backward()
    # The autograd product sum(D * gD) reaches the table as gD exactly; 3 * s as g_score = 3.
    f32_adjoint(oracle_mod, C.detach().cpu(), gD.cpu(), 3.0, C2.grad.cpu(), "autograd table")
    wf.last_async_error()


def test_blocked_cells_adjoint(oracle_mod):
    """+inf cells: the gradient of a finite score routes around them."""
    m, n = 130, 150
    C = inputs.uniform(m, n, seed=61)
    C[10:80, 20:30] = float("inf")
    C[100, :140] = float("inf")
    got = gpu_grad(C, None, 1.0, "table")
    f32_adjoint(oracle_mod, C, None, 1.0, got, "blocked cells")
    assert got[10:80, 20:30].abs().sum() == 0


@pytest.mark.parametrize("shape", [(130, 1500), (64, 2048), (257, 1100), (1, 1024)])
@pytest.mark.parametrize("source,ckpt_k", [("table", 64), ("ckpt", 64), ("ckpt", 192)])
def test_f32_adjoint_split_selection(oracle_mod, shape, source, ckpt_k):
    """n >= 1024 with few bands: the selection recompute sweeps each band as two column
    pieces, the second entering from a column of the table or of the checkpoint grid
    (a multiple of lcm(K, 64) near n/2); the adjoint stays bitwise equal to the oracle's."""
    m, n = shape
    C = inputs.normal_clipped(m, n, seed=m * 7 + n)
    got = gpu_grad(C, None, 1.0, source, ckpt_k=ckpt_k)
    f32_adjoint(oracle_mod, C, None, 1.0, got, f"{m}x{n} {source} K={ckpt_k}")


def test_f64_adjoint_split_selection(oracle_mod):
    C = inputs.normal_clipped(150, 1300, seed=5).double()
    gD = inputs.normal_clipped(150, 1300, seed=6).double()
    got = gpu_grad(C, gD, 0.5, "ckpt", ckpt_k=64)
    ref = oracle_grad(oracle_mod, C, gD, 0.5, "f64")
    assert torch.equal(got, ref)


def test_adjoint_4096_f32(oracle_mod):
    """The 4096 x 4096 workload with a non-negative upstream table: bitwise equal to the
    float32 oracle's adjoint, within 1e-4 (plain relative error, every term being
    non-negative) of the float64 adjoint on the same selections, every float32/float64
    selection flip a certified near-tie."""
    C = inputs.single_4096_f32()
    gD = inputs.uniform(4096, 4096, seed=71)
    got = gpu_grad(C, gD, 1.0, "ckpt", ckpt_k=4096)
    f32_adjoint(oracle_mod, C, gD, 1.0, got, "4096^2 ckpt_k=4096")


TIE_KINDS = ["zeros", "ints_0_3", "walls"]


def tie_input(kind, m, n, seed, dtype):
    """Inputs whose forward sums are exact in float32 and float64 and full of exact ties."""
    if kind == "zeros":
        C = torch.zeros(m, n, dtype=dtype)
    else:
        C = inputs.integers(m, n, seed=seed, lo=0, hi=3).to(dtype)
        if kind == "walls":
            C[m // 5: m // 2, n // 3] = float("inf")   # a wall with a gap above and below
            C[(3 * m) // 4, : n - n // 8] = float("inf")  # a row wall open at the right
    gD = inputs.integers(m, n, seed=seed + 1, lo=-2, hi=2).to(dtype)
    return C, gD


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", TIE_KINDS)
@pytest.mark.parametrize("shape", [(300, 257), (129, 1100)])
def test_adjoint_ties(oracle_mod, shape, kind, dtype):
    """Heavy ties: C = 0, integer C in [0, 3], and integer C with +inf walls, with integer
    upstream values.  Every selection is decided by the tie rule (NW, then N, then W) at many
    cells, and every sum is exact, so the device adjoint must equal the oracle's bitwise in
    both precisions and from both sources (the table, the checkpoint grid), and float32 must
    equal float64."""
    m, n = shape
    prec = "f32" if dtype == torch.float32 else "f64"
    C, gD = tie_input(kind, m, n, seed=m + n, dtype=dtype)
    ref = oracle_grad(oracle_mod, C, gD, 2.0, prec)
    ref64 = oracle_grad(oracle_mod, C.double(), gD.double(), 2.0, "f64")
    assert torch.equal(ref.double(), ref64), "integer sums must be exact in the oracle"
    for source, k in (("table", 64), ("ckpt", 64), ("ckpt", 1)):
        for tile in (16, 64):
            got = gpu_grad(C, gD, 2.0, source, tile=tile, ckpt_k=k)
            assert torch.equal(got, ref), f"{kind} {source} K={k} tile {tile}"


def test_adjoint_zero_input_routing(oracle_mod):
    """C = 0 everywhere: every interior cell ties three ways and takes NW, row 0 can only take
    W and column 0 only N.  Traced back from the last cell, the score's path is the diagonal
    that ends there, down to row 0 (or column 0), then the straight run along row 0 (or
    column 0) to the corner: checked against that closed form for wide and tall shapes."""
    for m, n in ((200, 333), (333, 200), (64, 64)):
        C = torch.zeros(m, n)
        got = gpu_grad(C, None, 1.0, "ckpt")
        want = torch.zeros(m, n)
        if n >= m:
            want[torch.arange(m), torch.arange(m) + (n - m)] = 1.0
            want[0, : n - m + 1] = 1.0
        else:
            want[torch.arange(n) + (m - n), torch.arange(n)] = 1.0
            want[: m - n + 1, 0] = 1.0
        assert torch.equal(got, want), (m, n)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("shape", [(40000, 200), (20000, 130)])
def test_adjoint_more_bands_than_cus(oracle_mod, shape, dtype):
    """Tall matrices with more 64-row bands than compute units (625 and 313 bands): every
    workgroup sweeps several bands in turn, in the selection recompute and in the reverse
    sweep, from the table and from the checkpoint grid."""
    m, n = shape
    C = inputs.uniform(m, n, seed=m + 3, dtype=dtype)
    gD = inputs.normal_clipped(m, n, seed=m + 4).to(dtype)
    for source in ("table", "ckpt"):
        got = gpu_grad(C, gD, 0.5, source, ckpt_k=64)
        if dtype == torch.float32:
            f32_adjoint(oracle_mod, C, gD, 0.5, got, f"{m}x{n} {source}")
        else:
            assert torch.equal(got, oracle_grad(oracle_mod, C, gD, 0.5, "f64")), source


def test_backward_argument_errors():
    C = torch.zeros(10, 10, device=DEV)
    with pytest.raises(ValueError):
        wf.backward(C)  # neither ckpt nor D
    D, _, ck = wf.forward(C, ckpt_k=4)
    with pytest.raises(ValueError):
        wf.backward(C, D=D, ckpt=ck, ckpt_k=4)
    with pytest.raises(wf.WfError):
        wf.backward(C.to(torch.int32), D=D.to(torch.int32))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_select_then_reverse_equals_backward(dtype):
    """wf_select followed by wf_reverse is wf_backward, bit for bit (checkpoint path, with g_D)."""
    m, n, k = 200, 333, 64
    C = inputs.normal_clipped(m, n, seed=41).to(dtype).to(DEV)
    gD = inputs.normal_clipped(m, n, seed=42).to(dtype).to(DEV)
    gs = torch.tensor(0.5, dtype=dtype, device=DEV)
    _, _, ck = wf.forward(C, table=False, ckpt_k=k)
    whole = wf.backward(C, g_score=gs, g_D=gD, ckpt=ck, ckpt_k=k)
    wf.select(C, ckpt=ck, ckpt_k=k)
    split = wf.reverse(m, n, dtype, g_score=gs, g_D=gD)
    wf.last_async_error()
    assert torch.equal(whole, split)


def test_reverse_needs_matching_selections():
    C = inputs.uniform(40, 50, seed=7).to(DEV)
    D, _, _ = wf.forward(C)
    wf.select(C, D=D)
    with pytest.raises(wf.WfError):
        wf.reverse(40, 51)  # other shape
    with pytest.raises(wf.WfError):
        wf.reverse(40, 50, torch.float64)  # other dtype
    g = wf.reverse(40, 50, g_score=torch.tensor(1.0))
    wf.last_async_error()
    assert torch.equal(g, wf.backward(C, g_score=torch.tensor(1.0, device=DEV), D=D))
